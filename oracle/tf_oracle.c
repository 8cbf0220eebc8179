/* FP64 CPU oracle of the tight-frame (TF) cone-beam CT iteration.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It shares no
 * source, header, table or helper with the GPU code.
 *
 * Paper: Jia, Dong, Lou & Jiang, "GPU-based Iterative Cone Beam CT
 * Reconstruction Using Tight Frame Regularization", arXiv 1008.2042.
 *
 * What is computed, section by section of the paper:
 *   section 2.1, Eq. (1)      the cone-beam line integral P (Joseph discretisation)
 *   Appendix 2, Eq. (A1)      its adjoint P^T, here the exact matrix transpose
 *   section 2.1 (filters)     the 27-band piecewise-linear tight frame W and W^T
 *   section 2.1, Eq. (2)      the vector shrinkage T_mu, then positivity H
 *   Appendix 1                CGLS warm-started from v
 *   section 2.1, Alg. A1/A2   the outer iteration, A2 with the t-momentum
 *   section 2.2.3             the coarse-to-fine multigrid schedule
 *   section 2.2.1, Eq. (3)    optionally, the paper's own operator pair:
 *                             Siddon's P with the closed-form backprojection
 *   section 2.3               the TV comparison method: the same CGLS step,
 *                             then the ROF sub-problem by gradient descent
 *   section 3 (comparisons)   FDK, the textbook filtered backprojection
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - geometry: source at (SAD cos t, SAD sin t, 0); flat detector through
 *     -(SDD-SAD)(cos t, sin t, 0) with axes e_u = (-sin t, cos t, 0),
 *     e_v = (0, 0, 1); detector values are point samples at pixel centres
 *     u_c = (c-(nu-1)/2) du, v_r = (r-(nv-1)/2) dv; voxel centres
 *     x_i = (i-(nx-1)/2) dx (same for y, z).
 *   - P: the paper traces rays with Siddon's method; the line integral of
 *     Eq. (1) is discretised here by Joseph's method instead: one stepping
 *     axis per view (x when |cos t| >= |sin t| - 1e-12, else y); on every
 *     voxel-centre plane of that axis crossed at ray parameter 0 < tau < 1
 *     the volume is interpolated bilinearly in the other two axes (zero
 *     outside the grid), and the sum is scaled by the path length between
 *     consecutive planes, l = d_step |a| / |a_step|.
 *   - P^T: the exact transpose of that matrix (the paper's closed form
 *     Eq. (3) is its continuous limit).
 *   - W: convolution with half-sample symmetric extension of f; W^T is its
 *     exact adjoint, so W^T W = I holds exactly.
 *   - CGLS: cgls_steps counts q = P p products; the last P^T is skipped since
 *     the output never uses it; guard 1e-300 on gamma and ||q||^2.
 *   - multigrid: coarse grids halve every axis (ceil), double the voxel size
 *     and stay centred; detector 2x2 binned (mean); prolongation is trilinear
 *     with the coarse index clamped to the grid; A2 restarts (t = 1) per grid.
 *   - TV (section 2.3): the l1 norm of the gradient with forward differences
 *     in index units, smoothed by eps; the ROF energy as printed, without a
 *     factor 1/2 on the data term; the adaptive step and the stop rule are
 *     stated at orc_rof; positivity after the sub-problem, as in A1.
 */
#include "tf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Deterministic FP64 dot product: fixed chunks summed in index order.        */
/* ------------------------------------------------------------------------- */
#define DOT_CHUNK 4096
static double dot(const double* a, const double* b, int64_t n) {
  int64_t nchunk = (n + DOT_CHUNK - 1) / DOT_CHUNK;
  if (nchunk == 0) return 0.0;
  double* part = (double*)malloc(sizeof(double) * (size_t)nchunk);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunk; ++c) {
    int64_t lo = c * DOT_CHUNK, hi = lo + DOT_CHUNK < n ? lo + DOT_CHUNK : n;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += part[c];
  free(part);
  return s;
}

/* ------------------------------------------------------------------------- */
/* Geometry (section 2.1, Eq. (1) and Fig. 1; conventions are this reading)  */
/* ------------------------------------------------------------------------- */
typedef struct {
  int step_x;      /* 1: planes x = x_i; 0: planes y = y_j */
  double cs, sn;   /* cos, sin of the view angle */
  double sx, sy;   /* source position (z = 0) */
} view_t;

static double view_angle(const orc_geom* g, int k) {
  return g->angles ? g->angles[k] : 2.0 * M_PI * (double)k / (double)g->n_views;
}

static view_t make_view(const orc_geom* g, int k) {
  view_t v;
  double t = view_angle(g, k);
  v.cs = cos(t);
  v.sn = sin(t);
  v.sx = g->sad * v.cs;
  v.sy = g->sad * v.sn;
  v.step_x = fabs(v.cs) >= fabs(v.sn) - 1e-12;
  return v;
}

static double hat(double t) {
  double a = 1.0 - fabs(t);
  return a > 0.0 ? a : 0.0;
}

/* The (at most four) voxel taps of ray (c, r) of view v on plane p of the
 * view's stepping axis.  Weights include the path length l.  Returns the
 * number of taps written to idx/w. */
static int plane_taps(const orc_geom* g, const view_t* v, int c, int r, int p,
                      int64_t idx[4], double w[4]) {
  double uc = ((double)c - 0.5 * (g->nu - 1)) * g->du;
  double vr = ((double)r - 0.5 * (g->nv - 1)) * g->dv;
  double ax = -g->sdd * v->cs - uc * v->sn;
  double ay = -g->sdd * v->sn + uc * v->cs;
  double az = vr;
  double alen = sqrt(ax * ax + ay * ay + az * az);
  int nx = g->nx, ny = g->ny, nz = g->nz;
  double th, zh, ell; /* transverse index, z index, path length */
  if (v->step_x) {
    double xp = ((double)p - 0.5 * (nx - 1)) * g->dx;
    double tau = (xp - v->sx) / ax;
    if (!(tau > 0.0 && tau < 1.0)) return 0;
    double Y = v->sy + tau * ay, Z = tau * az;
    th = Y / g->dy + 0.5 * (ny - 1);
    zh = Z / g->dz + 0.5 * (nz - 1);
    ell = g->dx * alen / fabs(ax);
  } else {
    double yp = ((double)p - 0.5 * (ny - 1)) * g->dy;
    double tau = (yp - v->sy) / ay;
    if (!(tau > 0.0 && tau < 1.0)) return 0;
    double X = v->sx + tau * ax, Z = tau * az;
    th = X / g->dx + 0.5 * (nx - 1);
    zh = Z / g->dz + 0.5 * (nz - 1);
    ell = g->dy * alen / fabs(ay);
  }
  int ntr = v->step_x ? ny : nx;
  int t0 = (int)floor(th), z0 = (int)floor(zh);
  int n = 0;
  for (int kk = z0; kk <= z0 + 1; ++kk) {
    if (kk < 0 || kk >= nz) continue;
    for (int tt = t0; tt <= t0 + 1; ++tt) {
      if (tt < 0 || tt >= ntr) continue;
      double wt = hat(th - tt) * hat(zh - kk);
      if (wt == 0.0) continue;
      int i = v->step_x ? p : tt;
      int j = v->step_x ? tt : p;
      idx[n] = ((int64_t)kk * ny + j) * nx + i;
      w[n] = ell * wt;
      ++n;
    }
  }
  return n;
}

static int n_planes(const orc_geom* g, const view_t* v) {
  return v->step_x ? g->nx : g->ny;
}

static double ray_integral(const orc_geom* g, const view_t* v, int c, int r,
                           const double* f) {
  double s = 0.0;
  int np = n_planes(g, v);
  for (int p = 0; p < np; ++p) {
    int64_t idx[4];
    double w[4];
    int n = plane_taps(g, v, c, r, p, idx, w);
    for (int t = 0; t < n; ++t) s += w[t] * f[idx[t]];
  }
  return s;
}

void orc_project(const orc_geom* g, const double* f, double* proj) {
  int nu = g->nu, nv = g->nv;
  for (int k = 0; k < g->n_views; ++k) {
    view_t v = make_view(g, k);
    double* out = proj + (int64_t)k * nu * nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < nv; ++r)
      for (int c = 0; c < nu; ++c) out[(int64_t)r * nu + c] = ray_integral(g, &v, c, r, f);
  }
}

void orc_project_rays(const orc_geom* g, const double* f, int64_t n,
                      const int32_t* vrc, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n; ++q) {
    view_t v = make_view(g, vrc[3 * q]);
    out[q] = ray_integral(g, &v, vrc[3 * q + 2], vrc[3 * q + 1], f);
  }
}

/* Transpose by scatter: a thread owns one plane of the stepping axis and
 * visits every ray of the view, so no two threads write the same voxel. */
void orc_backproject(const orc_geom* g, const double* proj, double* f) {
  int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
  memset(f, 0, sizeof(double) * (size_t)nvox);
  int nu = g->nu, nv = g->nv;
  for (int k = 0; k < g->n_views; ++k) {
    view_t v = make_view(g, k);
    const double* in = proj + (int64_t)k * nu * nv;
    int np = n_planes(g, &v);
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < np; ++p)
      for (int r = 0; r < nv; ++r)
        for (int c = 0; c < nu; ++c) {
          int64_t idx[4];
          double w[4];
          int n = plane_taps(g, &v, c, r, p, idx, w);
          double val = in[(int64_t)r * nu + c];
          for (int t = 0; t < n; ++t) f[idx[t]] += w[t] * val;
        }
  }
}

void orc_backproject_voxels(const orc_geom* g, const double* proj, int64_t n,
                            const int32_t* kji, double* out) {
  int nu = g->nu, nv = g->nv;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n; ++q) {
    int k = kji[3 * q], j = kji[3 * q + 1], i = kji[3 * q + 2];
    int64_t target = ((int64_t)k * g->ny + j) * g->nx + i;
    double s = 0.0;
    for (int vw = 0; vw < g->n_views; ++vw) {
      view_t v = make_view(g, vw);
      int p = v.step_x ? i : j;
      const double* in = proj + (int64_t)vw * nu * nv;
      for (int r = 0; r < nv; ++r)
        for (int c = 0; c < nu; ++c) {
          int64_t idx[4];
          double w[4];
          int m = plane_taps(g, &v, c, r, p, idx, w);
          for (int t = 0; t < m; ++t)
            if (idx[t] == target) s += w[t] * in[(int64_t)r * nu + c];
        }
    }
    out[q] = s;
  }
}

/* ------------------------------------------------------------------------- */
/* The paper's own operator pair (section 2.2.1 and Eq. (3))                  */
/* ------------------------------------------------------------------------- */
/* Ray (c, r) of view v: source s and a = pixel - source (section 2.1 geometry
 * reading above). */
static void ray_vectors(const orc_geom* g, const view_t* v, int c, int r, double s[3],
                        double a[3]) {
  double uc = ((double)c - 0.5 * (g->nu - 1)) * g->du;
  double vr = ((double)r - 0.5 * (g->nv - 1)) * g->dv;
  s[0] = v->sx;
  s[1] = v->sy;
  s[2] = 0.0;
  a[0] = -g->sdd * v->cs - uc * v->sn;
  a[1] = -g->sdd * v->sn + uc * v->cs;
  a[2] = vr;
}

static int cmp_double(const void* x, const void* y) {
  double a = *(const double*)x, b = *(const double*)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* Siddon's method (section 2.2.1): the voxels are boxes of size dx dy dz
 * centred on the voxel centres; the line integral of Eq. (1) over the
 * piecewise-constant volume is the sum over voxels of the value times the
 * length of the source-to-pixel segment inside the box.  The segment
 * s + alpha a, alpha in [0, 1], is cut at every box face it crosses (the
 * parameters alpha of its crossings with the x, y and z face planes,
 * sorted); each piece lies in one voxel.  Along an axis the piece's voxel
 * index follows from how many of that axis's face crossings lie before the
 * piece (the same alpha values that cut it, so a ray almost parallel to a
 * face is never put on the wrong side by rounding).  Boxes are half-open,
 * so a ray lying on a face plane between two voxels is counted once, in the
 * upper one.  `work` holds 2 (nx + ny + nz) + 8 doubles. */
static double siddon_ray(const orc_geom* g, const view_t* v, int c, int r, const double* f,
                         double* work) {
  double s[3], a[3];
  ray_vectors(g, v, c, r, s, a);
  const int n[3] = {g->nx, g->ny, g->nz};
  const double d[3] = {g->dx, g->dy, g->dz};
  double lo[3];
  for (int ax = 0; ax < 3; ++ax) lo[ax] = -0.5 * n[ax] * d[ax];
  /* face crossings per axis, in increasing alpha */
  double* face[3];
  face[0] = work;
  face[1] = face[0] + n[0] + 1;
  face[2] = face[1] + n[1] + 1;
  double* cuts = face[2] + n[2] + 1;
  int fixed[3]; /* voxel index along an axis the ray does not move along */
  for (int ax = 0; ax < 3; ++ax) {
    fixed[ax] = -1;
    if (a[ax] == 0.0) {
      int cnt = 0;
      for (int b = 0; b <= n[ax]; ++b)
        if (lo[ax] + b * d[ax] <= s[ax]) ++cnt;
      if (cnt == 0 || cnt == n[ax] + 1) return 0.0; /* outside [lower, upper) */
      fixed[ax] = cnt - 1;
      continue;
    }
    for (int b = 0; b <= n[ax]; ++b) {
      int bb = a[ax] > 0.0 ? b : n[ax] - b;
      face[ax][b] = (lo[ax] + bb * d[ax] - s[ax]) / a[ax];
    }
  }
  /* the part of [0, 1] inside the box: between the last entry and the first
   * exit over the moving axes */
  double amin = 0.0, amax = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    if (fixed[ax] >= 0) continue;
    if (face[ax][0] > amin) amin = face[ax][0];
    if (face[ax][n[ax]] < amax) amax = face[ax][n[ax]];
  }
  if (!(amax > amin)) return 0.0;
  int m = 0;
  cuts[m++] = amin;
  cuts[m++] = amax;
  for (int ax = 0; ax < 3; ++ax) {
    if (fixed[ax] >= 0) continue;
    for (int b = 0; b <= n[ax]; ++b)
      if (face[ax][b] > amin && face[ax][b] < amax) cuts[m++] = face[ax][b];
  }
  qsort(cuts, (size_t)m, sizeof(double), cmp_double);
  double alen = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  int cnt[3] = {0, 0, 0};
  double sum = 0.0;
  for (int q = 0; q + 1 < m; ++q) {
    double w = cuts[q + 1] - cuts[q];
    if (!(w > 0.0)) continue;
    double mid = 0.5 * (cuts[q] + cuts[q + 1]);
    int idx[3];
    for (int ax = 0; ax < 3; ++ax) {
      if (fixed[ax] >= 0) {
        idx[ax] = fixed[ax];
        continue;
      }
      while (cnt[ax] <= n[ax] && face[ax][cnt[ax]] < mid) ++cnt[ax];
      int t = a[ax] > 0.0 ? cnt[ax] - 1 : n[ax] - cnt[ax];
      idx[ax] = t < 0 ? 0 : (t >= n[ax] ? n[ax] - 1 : t);
    }
    sum += f[((int64_t)idx[2] * g->ny + idx[1]) * g->nx + idx[0]] * w * alen;
  }
  return sum;
}

static int siddon_work(const orc_geom* g) { return 2 * (g->nx + g->ny + g->nz) + 8; }

void orc_project_siddon(const orc_geom* g, const double* f, double* proj) {
  int nu = g->nu, nv = g->nv;
  for (int k = 0; k < g->n_views; ++k) {
    view_t v = make_view(g, k);
    double* out = proj + (int64_t)k * nu * nv;
#pragma omp parallel
    {
      double* al = (double*)malloc(sizeof(double) * (size_t)siddon_work(g));
#pragma omp for schedule(dynamic, 4)
      for (int r = 0; r < nv; ++r)
        for (int c = 0; c < nu; ++c) out[(int64_t)r * nu + c] = siddon_ray(g, &v, c, r, f, al);
      free(al);
    }
  }
}

void orc_project_siddon_rays(const orc_geom* g, const double* f, int64_t n,
                             const int32_t* vrc, double* out) {
#pragma omp parallel
  {
    double* al = (double*)malloc(sizeof(double) * (size_t)siddon_work(g));
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < n; ++q) {
      view_t v = make_view(g, vrc[3 * q]);
      out[q] = siddon_ray(g, &v, vrc[3 * q + 2], vrc[3 * q + 1], f, al);
    }
    free(al);
  }
}

/* Eq. (3): [P^T g](x) = dx dy dz / (du dv) sum_theta L^3(u*) / (L0 l^2(x))
 * g(u*), with u* where the line from the source through x meets the
 * detector, L(u*) = |u* - source|, l(x) = |x - source|, L0 = SDD; g(u*) by
 * bilinear interpolation of the pixel-centre samples (section 2.2.2); taps
 * that fall off the detector read zero. */
static double eq3_voxel(const orc_geom* g, const double* proj, int i, int j, int k) {
  double x = ((double)i - 0.5 * (g->nx - 1)) * g->dx;
  double y = ((double)j - 0.5 * (g->ny - 1)) * g->dy;
  double z = ((double)k - 0.5 * (g->nz - 1)) * g->dz;
  int nu = g->nu, nv = g->nv;
  double sum = 0.0;
  for (int vw = 0; vw < g->n_views; ++vw) {
    view_t v = make_view(g, vw);
    /* distance from the source to x along the central ray, magnification */
    double w = g->sad - (x * v.cs + y * v.sn);
    if (!(w > 0.0)) continue;
    double mag = g->sdd / w;
    double us = mag * (-x * v.sn + y * v.cs), vs = mag * z;
    double L = sqrt(g->sdd * g->sdd + us * us + vs * vs);
    double l2 = (x - v.sx) * (x - v.sx) + (y - v.sy) * (y - v.sy) + z * z;
    double fc = us / g->du + 0.5 * (nu - 1), fr = vs / g->dv + 0.5 * (nv - 1);
    int c0 = (int)floor(fc), r0 = (int)floor(fr);
    double wc = fc - c0, wr = fr - r0;
    const double* in = proj + (int64_t)vw * nu * nv;
    double gv = 0.0;
    for (int rr = 0; rr <= 1; ++rr)
      for (int cc = 0; cc <= 1; ++cc) {
        int c = c0 + cc, r = r0 + rr;
        if (c < 0 || c >= nu || r < 0 || r >= nv) continue;
        gv += (cc ? wc : 1.0 - wc) * (rr ? wr : 1.0 - wr) * in[(int64_t)r * nu + c];
      }
    sum += L * L * L / (g->sdd * l2) * gv;
  }
  return g->dx * g->dy * g->dz / (g->du * g->dv) * sum;
}

void orc_backproject_eq3(const orc_geom* g, const double* proj, double* f) {
  int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) f[((int64_t)k * ny + j) * nx + i] = eq3_voxel(g, proj, i, j, k);
}

void orc_backproject_eq3_voxels(const orc_geom* g, const double* proj, int64_t n,
                                const int32_t* kji, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n; ++q) out[q] = eq3_voxel(g, proj, kji[3 * q + 2], kji[3 * q + 1], kji[3 * q]);
}

/* Operator pair selection: 0 = Joseph P with its exact transpose, 1 = the
 * paper's Siddon P with the Eq. (3) backprojection. */
static void pair_project(int pair, const orc_geom* g, const double* f, double* proj) {
  if (pair == 1) orc_project_siddon(g, f, proj);
  else orc_project(g, f, proj);
}
static void pair_backproject(int pair, const orc_geom* g, const double* proj, double* f) {
  if (pair == 1) orc_backproject_eq3(g, proj, f);
  else orc_backproject(g, proj, f);
}

/* ------------------------------------------------------------------------- */
/* Tight frame (section 2.1): h0 = [1,2,1]/4, h1 = sqrt(2)/4 [1,0,-1],        */
/* h2 = [-1,2,-1]/4; band i = 9n + 3m + l is h_l(x) h_m(y) h_n(z).            */
/* ------------------------------------------------------------------------- */

/* Filter taps listed as h[-1], h[0], h[+1]. */
static double filt(int l, int m) {
  const double q = sqrt(2.0) / 4.0;
  static const double h0[3] = {0.25, 0.5, 0.25};
  static const double h2[3] = {-0.25, 0.5, -0.25};
  if (l == 0) return h0[m + 1];
  if (l == 2) return h2[m + 1];
  return m == -1 ? q : (m == 1 ? -q : 0.0);
}

/* Half-sample symmetric reflection into [0, N). */
static int reflect(int j, int N) {
  while (j < 0 || j >= N) j = (j < 0) ? -1 - j : 2 * N - 1 - j;
  return j;
}

/* One 1-D analysis operator A_l of length N with dilation d, as rows of
 * three (column, value) entries: (A_l f)[n] = sum_m h_l[m] f[R(n - m d)]. */
typedef struct {
  int N;
  int* col;    /* 3N */
  double* val; /* 3N */
} op1d;

static op1d make_op(int N, int d, int l) {
  op1d o;
  o.N = N;
  o.col = (int*)malloc(sizeof(int) * 3 * (size_t)N);
  o.val = (double*)malloc(sizeof(double) * 3 * (size_t)N);
  for (int n = 0; n < N; ++n)
    for (int m = -1; m <= 1; ++m) {
      o.col[3 * n + m + 1] = reflect(n - m * d, N);
      o.val[3 * n + m + 1] = filt(l, m);
    }
  return o;
}
static void free_op(op1d* o) {
  free(o->col);
  free(o->val);
}

/* out (+)= A in along one axis (axis 0 = x, 1 = y, 2 = z), or A^T in when
 * transpose is set: element n of every line along the axis receives
 * sum_e val * in[col] (A), or element col receives val * in[n] (A^T).  The
 * innermost loop always runs over contiguous x; each thread owns whole
 * lines (or rows) of the output, so there are no write races. */
static void apply_axis(int nx, int ny, int nz, int axis, const op1d* A,
                       int transpose, const double* in, double* out, int accumulate) {
  int64_t nvox = (int64_t)nx * ny * nz;
  if (!accumulate) memset(out, 0, sizeof(double) * (size_t)nvox);
  if (axis == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t L = 0; L < (int64_t)ny * nz; ++L) {
      const double* a = in + L * nx;
      double* b = out + L * nx;
      for (int n = 0; n < nx; ++n)
        for (int e = 0; e < 3; ++e) {
          int col = A->col[3 * n + e];
          double v = A->val[3 * n + e];
          if (!transpose) b[n] += v * a[col];
          else b[col] += v * a[n];
        }
    }
  } else if (axis == 1) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
      const double* a = in + (int64_t)z * nx * ny;
      double* b = out + (int64_t)z * nx * ny;
      for (int n = 0; n < ny; ++n)
        for (int e = 0; e < 3; ++e) {
          int col = A->col[3 * n + e];
          double v = A->val[3 * n + e];
          int src = transpose ? n : col, dst = transpose ? col : n;
          for (int i = 0; i < nx; ++i) b[(int64_t)dst * nx + i] += v * a[(int64_t)src * nx + i];
        }
    }
  } else {
    int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int n = 0; n < nz; ++n)
        for (int e = 0; e < 3; ++e) {
          int col = A->col[3 * n + e];
          double v = A->val[3 * n + e];
          int src = transpose ? n : col, dst = transpose ? col : n;
          const double* a = in + src * plane + (int64_t)y * nx;
          double* b = out + dst * plane + (int64_t)y * nx;
          for (int i = 0; i < nx; ++i) b[i] += v * a[i];
        }
  }
}

void orc_framelet_analysis(int32_t nx, int32_t ny, int32_t nz, int32_t dil,
                           const double* f, double* coeff) {
  int64_t V = (int64_t)nx * ny * nz;
  double* tx = (double*)malloc(sizeof(double) * (size_t)V);
  double* txy = (double*)malloc(sizeof(double) * (size_t)V);
  for (int l = 0; l < 3; ++l) {
    op1d Ax = make_op(nx, dil, l);
    apply_axis(nx, ny, nz, 0, &Ax, 0, f, tx, 0);
    for (int m = 0; m < 3; ++m) {
      op1d Ay = make_op(ny, dil, m);
      apply_axis(nx, ny, nz, 1, &Ay, 0, tx, txy, 0);
      for (int n = 0; n < 3; ++n) {
        op1d Az = make_op(nz, dil, n);
        apply_axis(nx, ny, nz, 2, &Az, 0, txy, coeff + (int64_t)(9 * n + 3 * m + l) * V, 0);
        free_op(&Az);
      }
      free_op(&Ay);
    }
    free_op(&Ax);
  }
  free(tx);
  free(txy);
}

void orc_framelet_synthesis(int32_t nx, int32_t ny, int32_t nz, int32_t dil,
                            const double* coeff, double* f) {
  int64_t V = (int64_t)nx * ny * nz;
  double* az = (double*)malloc(sizeof(double) * (size_t)V);
  double* ayz = (double*)malloc(sizeof(double) * (size_t)V);
  memset(f, 0, sizeof(double) * (size_t)V);
  for (int l = 0; l < 3; ++l) {
    memset(ayz, 0, sizeof(double) * (size_t)V);
    for (int m = 0; m < 3; ++m) {
      memset(az, 0, sizeof(double) * (size_t)V);
      for (int n = 0; n < 3; ++n) {
        op1d Az = make_op(nz, dil, n);
        apply_axis(nx, ny, nz, 2, &Az, 1, coeff + (int64_t)(9 * n + 3 * m + l) * V, az, 1);
        free_op(&Az);
      }
      op1d Ay = make_op(ny, dil, m);
      apply_axis(nx, ny, nz, 1, &Ay, 1, az, ayz, 1);
      free_op(&Ay);
    }
    op1d Ax = make_op(nx, dil, l);
    apply_axis(nx, ny, nz, 0, &Ax, 1, ayz, f, 1);
    free_op(&Ax);
  }
  free(az);
  free(ayz);
}

/* Eq. (2): the low band is kept; the 26 high bands at a voxel are scaled by
 * max(1 - mu / ||alpha_h||, 0), taken as 0 when ||alpha_h|| <= mu. */
void orc_shrink(int64_t nvox, double lambda, double* coeff) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < nvox; ++x) {
    double n2 = 0.0;
    for (int b = 1; b < 27; ++b) n2 += coeff[b * nvox + x] * coeff[b * nvox + x];
    double nrm = sqrt(n2);
    double s = nrm <= lambda ? 0.0 : 1.0 - lambda / nrm;
    for (int b = 1; b < 27; ++b) coeff[b * nvox + x] *= s;
  }
}

void orc_framelet_shrink(int32_t nx, int32_t ny, int32_t nz, int32_t levels,
                         double lambda, int32_t positivity, const double* in,
                         double* out) {
  int64_t V = (int64_t)nx * ny * nz;
  double* c1 = (double*)malloc(sizeof(double) * 27 * (size_t)V);
  orc_framelet_analysis(nx, ny, nz, 1, in, c1);
  if (levels >= 2) {
    /* Second level: the dilated (taps -2, 0, +2) frame applied to the level-1
     * low band; each level is shrunk on its own 26 high bands. */
    double* c2 = (double*)malloc(sizeof(double) * 27 * (size_t)V);
    orc_framelet_analysis(nx, ny, nz, 2, c1, c2);
    orc_shrink(V, lambda, c2);
    orc_framelet_synthesis(nx, ny, nz, 2, c2, c1);
    free(c2);
  }
  orc_shrink(V, lambda, c1);
  orc_framelet_synthesis(nx, ny, nz, 1, c1, out);
  free(c1);
  if (positivity)
    for (int64_t x = 0; x < V; ++x)
      if (out[x] < 0.0) out[x] = 0.0;
}

/* ------------------------------------------------------------------------- */
/* CGLS (Appendix 1)                                                         */
/* ------------------------------------------------------------------------- */
int orc_cgls(const orc_geom* g, double* x, const double* proj, int32_t n,
             double* resid2, double* resid_hist) {
  return orc_cgls_pair(g, 0, x, proj, n, resid2, resid_hist);
}

int orc_cgls_pair(const orc_geom* g, int32_t pair, double* x, const double* proj, int32_t n,
                  double* resid2, double* resid_hist) {
  int64_t V = (int64_t)g->nx * g->ny * g->nz;
  int64_t S = (int64_t)g->n_views * g->nu * g->nv;
  double* r = (double*)malloc(sizeof(double) * (size_t)S);
  double* q = (double*)malloc(sizeof(double) * (size_t)S);
  double* s = (double*)malloc(sizeof(double) * (size_t)V);
  double* p = (double*)malloc(sizeof(double) * (size_t)V);
  const double tiny = 1e-300;
  int broke = 0;

  pair_project(pair, g, x, r);
  for (int64_t i = 0; i < S; ++i) r[i] = proj[i] - r[i];
  if (resid_hist) {
    for (int l = 0; l <= n; ++l) resid_hist[l] = NAN;
    resid_hist[0] = dot(r, r, S);
  }
  pair_backproject(pair, g, r, s);
  memcpy(p, s, sizeof(double) * (size_t)V);
  double gamma = dot(s, s, V);

  for (int l = 0; l < n; ++l) {
    pair_project(pair, g, p, q);
    double delta = dot(q, q, S);
    if (gamma <= tiny || delta <= tiny) {
      broke = 1;
      break;
    }
    double alpha = gamma / delta;
    for (int64_t i = 0; i < V; ++i) x[i] += alpha * p[i];
    for (int64_t i = 0; i < S; ++i) r[i] -= alpha * q[i];
    if (resid_hist) resid_hist[l + 1] = dot(r, r, S);
    if (l < n - 1) {
      pair_backproject(pair, g, r, s);
      double gnew = dot(s, s, V);
      double beta = gnew / gamma;
      for (int64_t i = 0; i < V; ++i) p[i] = s[i] + beta * p[i];
      gamma = gnew;
    }
  }
  if (resid2) *resid2 = dot(r, r, S);
  free(r);
  free(q);
  free(s);
  free(p);
  return broke;
}

/* ------------------------------------------------------------------------- */
/* Multigrid transfer (section 2.2.3)                                         */
/* ------------------------------------------------------------------------- */
void orc_coarse_geom(const orc_geom* fine, int32_t bin_detector, orc_geom* c) {
  *c = *fine;
  c->nx = (fine->nx + 1) / 2;
  c->ny = (fine->ny + 1) / 2;
  c->nz = (fine->nz + 1) / 2;
  c->dx = 2.0 * fine->dx;
  c->dy = 2.0 * fine->dy;
  c->dz = 2.0 * fine->dz;
  if (bin_detector) {
    c->nu = (fine->nu + 1) / 2;
    c->nv = (fine->nv + 1) / 2;
    c->du = 2.0 * fine->du;
    c->dv = 2.0 * fine->dv;
  }
}

/* Coarse pixel (r, c) is the mean of the fine pixels {2r, 2r+1} x {2c, 2c+1}
 * that exist. */
void orc_restrict_sino(const orc_geom* fine, const double* in, double* out) {
  int nu = fine->nu, nv = fine->nv, nuc = (nu + 1) / 2, nvc = (nv + 1) / 2;
  for (int k = 0; k < fine->n_views; ++k) {
    const double* a = in + (int64_t)k * nu * nv;
    double* b = out + (int64_t)k * nuc * nvc;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nvc; ++r)
      for (int c = 0; c < nuc; ++c) {
        double s = 0.0;
        int cnt = 0;
        for (int dr = 0; dr < 2; ++dr)
          for (int dc = 0; dc < 2; ++dc) {
            int rr = 2 * r + dr, cc = 2 * c + dc;
            if (rr < nv && cc < nu) {
              s += a[(int64_t)rr * nu + cc];
              ++cnt;
            }
          }
        b[(int64_t)r * nuc + c] = s / cnt;
      }
  }
}

/* Linear interpolation of the coarse solution at each fine voxel centre, the
 * coarse fractional index clamped to the coarse grid on every axis. */
static void lin_index(double pos, double dc, int nc, int* i0, int* i1, double* w1) {
  double t = pos / dc + 0.5 * (nc - 1);
  if (t < 0.0) t = 0.0;
  if (t > nc - 1) t = nc - 1;
  int a = (int)floor(t);
  if (a > nc - 1) a = nc - 1;
  *i0 = a;
  *i1 = a + 1 < nc ? a + 1 : nc - 1;
  *w1 = t - a;
}

void orc_prolong_vol(const orc_geom* co, const orc_geom* fi, const double* in,
                     double* out) {
  int nx = fi->nx, ny = fi->ny, nz = fi->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int x0, x1, y0, y1, z0, z1;
        double wx, wy, wz;
        lin_index((i - 0.5 * (nx - 1)) * fi->dx, co->dx, co->nx, &x0, &x1, &wx);
        lin_index((j - 0.5 * (ny - 1)) * fi->dy, co->dy, co->ny, &y0, &y1, &wy);
        lin_index((k - 0.5 * (nz - 1)) * fi->dz, co->dz, co->nz, &z0, &z1, &wz);
        int xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1};
        double wxs[2] = {1 - wx, wx}, wys[2] = {1 - wy, wy}, wzs[2] = {1 - wz, wz};
        double s = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              s += wzs[c] * wys[b] * wxs[a] *
                   in[((int64_t)zs[c] * co->ny + ys[b]) * co->nx + xs[a]];
        out[((int64_t)k * ny + j) * nx + i] = s;
      }
}

/* ------------------------------------------------------------------------- */
/* Algorithm A2 (A1 with momentum = 0) and the multigrid driver               */
/* ------------------------------------------------------------------------- */
int orc_tf_iterations(const orc_geom* g, const orc_opts* o, const double* proj,
                      int32_t n_iters, double* vol, orc_report* rep) {
  int64_t V = (int64_t)g->nx * g->ny * g->nz;
  double* f_prev = (double*)malloc(sizeof(double) * (size_t)V);
  double* f_cur = (double*)malloc(sizeof(double) * (size_t)V);
  double* x = (double*)malloc(sizeof(double) * (size_t)V);
  memcpy(f_cur, vol, sizeof(double) * (size_t)V);
  memcpy(f_prev, vol, sizeof(double) * (size_t)V);
  double t_prev = 1.0, t_cur = 1.0;
  for (int k = 0; k < n_iters; ++k) {
    double c = o->momentum ? (t_prev - 1.0) / t_cur : 0.0;
    for (int64_t i = 0; i < V; ++i) x[i] = f_cur[i] + c * (f_cur[i] - f_prev[i]);
    double r2 = 0.0;
    int broke = orc_cgls_pair(g, o->op_pair, x, proj, o->cgls_steps, &r2, NULL);
    if (rep) {
      rep->cgls_breakdowns += broke;
      rep->resid2_last = r2;
    }
    double* tmp = f_prev;
    f_prev = f_cur;
    f_cur = tmp;
    orc_framelet_shrink(g->nx, g->ny, g->nz, o->framelet_levels, o->lambda,
                        o->positivity, x, f_cur);
    double t_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t_cur * t_cur));
    t_prev = t_cur;
    t_cur = t_next;
  }
  memcpy(vol, f_cur, sizeof(double) * (size_t)V);
  free(f_prev);
  free(f_cur);
  free(x);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* The TV comparison method (section 2.3)                                     */
/* ------------------------------------------------------------------------- */
/* The ROF energy ||f - x||^2 + mu TV(f).  TV is the integral of the l1 norm
 * of the gradient (section 2.3), discretised with forward differences in
 * index units (d_a = f[i + e_a] - f[i] where voxel i + e_a exists) and
 * smoothed, |d| ~ sqrt(d^2 + eps^2), so that gradient descent applies.  Per
 * z-slice partial sums, added in slice order (deterministic). */
double orc_tv_energy(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv,
                     const double* x, const double* f) {
  double* part = (double*)malloc(sizeof(double) * (size_t)nz);
  const double e2 = tv->eps * tv->eps;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k) {
    double data = 0.0, tvs = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = ((int64_t)k * ny + j) * nx + i;
        double r = f[q] - x[q];
        data += r * r;
        if (i + 1 < nx) {
          double d = f[q + 1] - f[q];
          tvs += sqrt(d * d + e2);
        }
        if (j + 1 < ny) {
          double d = f[q + nx] - f[q];
          tvs += sqrt(d * d + e2);
        }
        if (k + 1 < nz) {
          double d = f[q + (int64_t)nx * ny] - f[q];
          tvs += sqrt(d * d + e2);
        }
      }
    part[k] = data + tv->mu * tvs;
  }
  double e = 0.0;
  for (int k = 0; k < nz; ++k) e += part[k];
  free(part);
  return e;
}

/* dE/df: 2 (f - x) + mu sum_a [psi(d_a at i - e_a) - psi(d_a at i)], with
 * psi(d) = d / sqrt(d^2 + eps^2) the derivative of the smoothed |d|. */
void orc_tv_gradient(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv,
                     const double* x, const double* f, double* grad) {
  const double e2 = tv->eps * tv->eps;
  const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = ((int64_t)k * ny + j) * nx + i;
        double gq = 2.0 * (f[q] - x[q]);
        double t = 0.0, d;
        if (i + 1 < nx) { d = f[q + sx] - f[q]; t -= d / sqrt(d * d + e2); }
        if (i > 0)      { d = f[q] - f[q - sx]; t += d / sqrt(d * d + e2); }
        if (j + 1 < ny) { d = f[q + sy] - f[q]; t -= d / sqrt(d * d + e2); }
        if (j > 0)      { d = f[q] - f[q - sy]; t += d / sqrt(d * d + e2); }
        if (k + 1 < nz) { d = f[q + sz] - f[q]; t -= d / sqrt(d * d + e2); }
        if (k > 0)      { d = f[q] - f[q - sz]; t += d / sqrt(d * d + e2); }
        grad[q] = gq + tv->mu * t;
      }
}

/* Gradient descent on the ROF energy from f = x (section 2.3).  The paper
 * gives the rule only as "an adaptively adjusted step length" and the stop
 * as a decrease under 0.1 %; the reading taken: the step s starts at 1/2
 * (the exact minimiser of the data term alone); a trial f - s grad is
 * accepted if it lowers the energy, otherwise s is halved and the trial
 * repeated (at most 40 halvings, after which the descent ends); after an
 * accepted step s doubles, up to 1/2; the descent ends after the first
 * accepted step whose relative decrease is below tol, or after max_steps
 * accepted steps. */
int orc_rof(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv, const double* x,
            double* f, double* energies) {
  int64_t V = (int64_t)nx * ny * nz;
  double* g = (double*)malloc(sizeof(double) * (size_t)V);
  double* ft = (double*)malloc(sizeof(double) * (size_t)V);
  memcpy(f, x, sizeof(double) * (size_t)V);
  double E = orc_tv_energy(nx, ny, nz, tv, x, f);
  if (energies) energies[0] = E;
  double s = 0.5;
  int steps = 0;
  while (steps < tv->max_steps && E > 0.0) {
    orc_tv_gradient(nx, ny, nz, tv, x, f, g);
    int accepted = 0;
    double Et = E;
    for (int h = 0; h <= 40; ++h) {
      for (int64_t q = 0; q < V; ++q) ft[q] = f[q] - s * g[q];
      Et = orc_tv_energy(nx, ny, nz, tv, x, ft);
      if (Et < E) {
        accepted = 1;
        break;
      }
      s *= 0.5;
    }
    if (!accepted) break;
    double rel = (E - Et) / E;
    memcpy(f, ft, sizeof(double) * (size_t)V);
    E = Et;
    ++steps;
    if (energies) energies[steps] = E;
    s = 2.0 * s < 0.5 ? 2.0 * s : 0.5;
    if (rel < tv->tol) break;
  }
  free(g);
  free(ft);
  return steps;
}

/* n_iters outer iterations of the TV method on one grid from vol. */
static int tv_iterations(const orc_geom* g, const orc_opts* o, const orc_tv* tv,
                         const double* proj, int32_t n_iters, double* vol, orc_report* rep,
                         int32_t* rof_steps) {
  int64_t V = (int64_t)g->nx * g->ny * g->nz;
  double* x = (double*)malloc(sizeof(double) * (size_t)V);
  for (int k = 0; k < n_iters; ++k) {
    memcpy(x, vol, sizeof(double) * (size_t)V);
    double r2 = 0.0;
    int broke = orc_cgls_pair(g, o->op_pair, x, proj, o->cgls_steps, &r2, NULL);
    if (rep) {
      rep->cgls_breakdowns += broke;
      rep->resid2_last = r2;
    }
    int st = orc_rof(g->nx, g->ny, g->nz, tv, x, vol, NULL);
    if (rof_steps) *rof_steps += st;
    if (o->positivity)
      for (int64_t i = 0; i < V; ++i)
        if (vol[i] < 0.0) vol[i] = 0.0;
  }
  free(x);
  return 0;
}

/* The coarse-to-fine schedule of section 2.2.3 around either method: the
 * TF iteration (tv == NULL) or the TV one. */
static int schedule(const orc_geom* g, const orc_opts* o, const orc_tv* tv, const double* proj,
                    double* vol, orc_report* rep, int32_t* rof_steps) {
  int ng = o->n_grids;
  if (ng < 1 || ng > 4) return -1;
  orc_geom geo[4];
  double* sino[4];
  geo[0] = *g;
  sino[0] = (double*)proj;
  for (int l = 1; l < ng; ++l) {
    orc_coarse_geom(&geo[l - 1], o->bin_coarse_detector, &geo[l]);
    int64_t S = (int64_t)geo[l].n_views * geo[l].nu * geo[l].nv;
    sino[l] = (double*)malloc(sizeof(double) * (size_t)S);
    if (o->bin_coarse_detector) orc_restrict_sino(&geo[l - 1], sino[l - 1], sino[l]);
    else memcpy(sino[l], sino[l - 1], sizeof(double) * (size_t)S);
  }
  if (rep) memset(rep, 0, sizeof(*rep));
  if (rof_steps) *rof_steps = 0;
  double* cur = NULL;
  for (int l = ng - 1; l >= 0; --l) {
    int64_t V = (int64_t)geo[l].nx * geo[l].ny * geo[l].nz;
    double* f = (double*)malloc(sizeof(double) * (size_t)V);
    if (cur == NULL) memset(f, 0, sizeof(double) * (size_t)V);
    else {
      orc_prolong_vol(&geo[l + 1], &geo[l], cur, f);
      free(cur);
    }
    int it = o->iters[ng - 1 - l];
    if (tv) tv_iterations(&geo[l], o, tv, sino[l], it, f, rep, rof_steps);
    else orc_tf_iterations(&geo[l], o, sino[l], it, f, rep);
    if (rep) rep->iters_done[ng - 1 - l] = it;
    cur = f;
  }
  memcpy(vol, cur, sizeof(double) * (size_t)g->nx * g->ny * g->nz);
  free(cur);
  for (int l = 1; l < ng; ++l) free(sino[l]);
  return 0;
}

int orc_reconstruct(const orc_geom* g, const orc_opts* o, const double* proj,
                    double* vol, orc_report* rep) {
  return schedule(g, o, NULL, proj, vol, rep, NULL);
}

int orc_reconstruct_tv(const orc_geom* g, const orc_opts* o, const orc_tv* tv,
                       const double* proj, double* vol, orc_report* rep,
                       int32_t* rof_steps) {
  if (!tv || tv->mu < 0.0 || !(tv->eps > 0.0) || tv->max_steps < 0) return -1;
  return schedule(g, o, tv, proj, vol, rep, rof_steps);
}

/* ------------------------------------------------------------------------- */
/* FDK, the comparison baseline of section 3 (the paper names it only):      */
/* the textbook Feldkamp-Davis-Kress algorithm for a full circular orbit     */
/* with equally spaced views and a flat detector.  Coordinates are scaled to */
/* a virtual detector through the rotation axis: p = u SAD / SDD,            */
/* zeta = v SAD / SDD, pitch dp = du SAD / SDD.                              */
/*   1. weight each pixel by SAD / sqrt(SAD^2 + p^2 + zeta^2)                */
/*      (= SDD / sqrt(SDD^2 + u^2 + v^2));                                   */
/*   2. filter every detector row with the band-limited ramp (Ram-Lak)       */
/*      kernel h, linear convolution with zero extension:                    */
/*      Q(p_c) = dp sum_m w g(p_m) h((c - m) dp);                            */
/*   3. backproject: f(x) = (pi / N) sum_views (SAD / U)^2 Q(p*, zeta*),     */
/*      U = SAD - x.s_hat the source-to-voxel depth along the central ray,   */
/*      p* = SAD (x.e_u) / U, zeta* = SAD z / U, Q bilinear between pixel    */
/*      centres (zero off the detector).                                     */
/* ------------------------------------------------------------------------- */
/* The Ram-Lak kernel at lag n, spacing dp: the inverse Fourier transform of */
/* |w| band-limited to |w| <= 1 / (2 dp), sampled at n dp.                   */
double orc_ramlak(int32_t n, double dp) {
  if (n == 0) return 1.0 / (4.0 * dp * dp);
  if (n % 2 == 0) return 0.0;
  return -1.0 / ((double)n * (double)n * M_PI * M_PI * dp * dp);
}

void orc_fdk_filter(const orc_geom* g, const double* proj, double* q) {
  const int nu = g->nu, nv = g->nv;
  const double mag = g->sad / g->sdd;
  const double dp = g->du * mag;
#pragma omp parallel
  {
    double* w = (double*)malloc(sizeof(double) * (size_t)nu);
#pragma omp for schedule(static)
    for (int64_t row = 0; row < (int64_t)g->n_views * nv; ++row) {
      const int r = (int)(row % nv);
      const double v = ((double)r - 0.5 * (nv - 1)) * g->dv;
      const double* in = proj + row * nu;
      for (int c = 0; c < nu; ++c) {
        const double u = ((double)c - 0.5 * (nu - 1)) * g->du;
        w[c] = in[c] * g->sdd / sqrt(g->sdd * g->sdd + u * u + v * v);
      }
      double* out = q + row * nu;
      for (int c = 0; c < nu; ++c) {
        double s = 0.0;
        for (int m = 0; m < nu; ++m) s += w[m] * orc_ramlak(c - m, dp);
        out[c] = dp * s;
      }
    }
    free(w);
  }
}

static double fdk_voxel(const orc_geom* g, const double* q, int i, int j, int k) {
  const double x = ((double)i - 0.5 * (g->nx - 1)) * g->dx;
  const double y = ((double)j - 0.5 * (g->ny - 1)) * g->dy;
  const double z = ((double)k - 0.5 * (g->nz - 1)) * g->dz;
  double s = 0.0;
  for (int vw = 0; vw < g->n_views; ++vw) {
    const double th = 2.0 * M_PI * (double)vw / (double)g->n_views;
    const double cs = cos(th), sn = sin(th);
    const double U = g->sad - (x * cs + y * sn);
    const double t = -x * sn + y * cs;
    /* detector position of the voxel centre, in pixel indices */
    const double uc = g->sdd * t / U / g->du + 0.5 * (g->nu - 1);
    const double vr = g->sdd * z / U / g->dv + 0.5 * (g->nv - 1);
    const int c0 = (int)floor(uc), r0 = (int)floor(vr);
    const double fc = uc - c0, fr = vr - r0;
    double val = 0.0;
    for (int dr = 0; dr < 2; ++dr)
      for (int dc = 0; dc < 2; ++dc) {
        const int c = c0 + dc, r = r0 + dr;
        if (c < 0 || c >= g->nu || r < 0 || r >= g->nv) continue;
        const double wgt = (dc ? fc : 1.0 - fc) * (dr ? fr : 1.0 - fr);
        val += wgt * q[((int64_t)vw * g->nv + r) * g->nu + c];
      }
    s += (g->sad / U) * (g->sad / U) * val;
  }
  return M_PI / (double)g->n_views * s;
}

void orc_fdk_backproject(const orc_geom* g, const double* q, double* vol) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i)
        vol[((int64_t)k * g->ny + j) * g->nx + i] = fdk_voxel(g, q, i, j, k);
}

int orc_fdk(const orc_geom* g, const double* proj, double* vol) {
  if (g->angles) return -1; /* equally spaced full orbit only */
  int64_t S = (int64_t)g->n_views * g->nu * g->nv;
  double* q = (double*)malloc(sizeof(double) * (size_t)S);
  orc_fdk_filter(g, proj, q);
  orc_fdk_backproject(g, q, vol);
  free(q);
  return 0;
}
