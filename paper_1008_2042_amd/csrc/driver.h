// Host-side driver pieces shared by the reconstruction entry points and the
// serving loop: validation, workspace plans, and the launch sequences of one
// CGLS call and one framelet regularisation step.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tfcb_internal.h"

namespace tfcb {

// detail string of the last failure on this thread (tfcb_last_error)
inline thread_local std::string g_last_error;

namespace {



tfcb_status fail(tfcb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define TFCB_HIP(expr)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(TFCB_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                  __FILE__, __LINE__);                                                       \
  } while (0)

#define TFCB_TRY(expr)                 \
  do {                                 \
    tfcb_status st_ = (expr);          \
    if (st_ != TFCB_OK) return st_;    \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

tfcb_status validate_geometry(const tfcb_geometry* g) {
  if (!g) return fail(TFCB_EINVAL, "geometry is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nu < 1 || g->nv < 1 || g->n_views < 1)
    return fail(TFCB_EINVAL, "geometry sizes must be >= 1 (nx=%d ny=%d nz=%d nu=%d nv=%d views=%d)",
                g->nx, g->ny, g->nz, g->nu, g->nv, g->n_views);
  if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz) || !finite_pos(g->du) ||
      !finite_pos(g->dv))
    return fail(TFCB_EINVAL, "voxel and pixel sizes must be finite and > 0");
  if (!finite_pos(g->sad) || !std::isfinite(g->sdd) || !(g->sdd > g->sad))
    return fail(TFCB_EINVAL, "need 0 < sad < sdd (sad=%g sdd=%g)", g->sad, g->sdd);
  // the volume grown by two voxels (the backprojector's footprint boxes)
  // must stay inside the source orbit
  const double hx = (0.5 * g->nx + 2.0) * g->dx, hy = (0.5 * g->ny + 2.0) * g->dy;
  if (!(std::sqrt(hx * hx + hy * hy) < g->sad))
    return fail(TFCB_EINVAL, "the volume must lie inside the source orbit (half-diagonal %g >= sad %g)",
                std::sqrt(hx * hx + hy * hy), g->sad);
  const double nvox = (double)g->nx * g->ny * g->nz;
  const double npix = (double)g->n_views * g->nu * g->nv;
  if (nvox >= 2147483647.0 || npix >= 2147483647.0)
    return fail(TFCB_EUNSUPPORTED, "volume or projection set exceeds 2^31 elements");
  if (g->nx > 65535 || g->ny > 65535 || g->nz > 65535 || g->n_views > 65535)
    return fail(TFCB_EUNSUPPORTED, "an axis exceeds 65535");
  if (g->nv > 16384 || g->nu > 65535)
    return fail(TFCB_EUNSUPPORTED, "detector larger than 65535 x 16384 pixels");
  const double pad = (double)(g->nz + 2 * kZPad) * std::max(g->nx, g->ny) * (std::max(g->nx, g->ny) + 4) + 8;
  if (pad >= 2147483647.0)
    return fail(TFCB_EUNSUPPORTED, "padded volume copy exceeds 2^31 elements");
  if (g->angles)
    for (int k = 0; k < g->n_views; ++k)
      if (!std::isfinite(g->angles[k])) return fail(TFCB_EINVAL, "angle %d is not finite", k);
  return TFCB_OK;
}

tfcb_status validate_dtype(tfcb_dtype dt) {
  if (dt != TFCB_F32 && dt != TFCB_F16 && dt != TFCB_BF16)
    return fail(TFCB_EINVAL, "unknown dtype %d", (int)dt);
  return TFCB_OK;
}

tfcb_status validate_options(const tfcb_options* o) {
  if (!o) return fail(TFCB_EINVAL, "options is NULL");
  if (!std::isfinite(o->lambda) || o->lambda < 0.0)
    return fail(TFCB_EINVAL, "lambda must be finite and >= 0");
  if (o->n_grids < 1 || o->n_grids > 4) return fail(TFCB_EINVAL, "n_grids must be in 1..4");
  for (int l = 0; l < o->n_grids; ++l)
    if (o->iters[l] < 0 || o->iters[l] > 100000)
      return fail(TFCB_EINVAL, "iters[%d] out of range", l);
  if (o->cgls_steps < 1 || o->cgls_steps > 64) return fail(TFCB_EINVAL, "cgls_steps must be 1..64");
  if (o->framelet_levels != 1 && o->framelet_levels != 2)
    return fail(TFCB_EINVAL, "framelet_levels must be 1 or 2");
  TFCB_TRY(validate_dtype(o->storage));
  if (o->op_pair != 0 && o->op_pair != 1) return fail(TFCB_EINVAL, "op_pair must be 0 or 1");
  if (o->regulariser != 0 && o->regulariser != 1)
    return fail(TFCB_EINVAL, "regulariser must be 0 (tight frame) or 1 (TV)");
  if (o->regulariser == 1) {
    if (!std::isfinite(o->tv_eps) || !(o->tv_eps > 0.0))
      return fail(TFCB_EINVAL, "tv_eps must be finite and > 0");
    if (!std::isfinite(o->tv_tol) || o->tv_tol < 0.0)
      return fail(TFCB_EINVAL, "tv_tol must be finite and >= 0");
    if (o->tv_max_steps < 0 || o->tv_max_steps > 100000)
      return fail(TFCB_EINVAL, "tv_max_steps must be 0..100000");
  }
  return TFCB_OK;
}

// Caller data buffers (volumes, projections) need element alignment only:
// every kernel that reads them with wider vectors reads an internal copy.
tfcb_status check_ptr(const void* p, const char* name, size_t elem_bytes) {
  if (!p) return fail(TFCB_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % elem_bytes != 0)
    return fail(TFCB_EINVAL, "%s is not aligned to its %zu-byte elements", name, elem_bytes);
  return TFCB_OK;
}

tfcb_status check_ws(const void* ws, size_t have, size_t need) {
  if (need == 0) return TFCB_OK;
  if (!ws) return fail(TFCB_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
    return fail(TFCB_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (have < need) return fail(TFCB_ENOMEM, "workspace too small (%zu < %zu bytes)", have, need);
  return TFCB_OK;
}

size_t nvox(const tfcb_geometry& g) { return (size_t)g.nx * g.ny * g.nz; }
size_t npix(const tfcb_geometry& g) { return (size_t)g.n_views * g.nu * g.nv; }

tfcb_geometry coarse_of(const tfcb_geometry& f, bool bin) {
  tfcb_geometry c = f;
  c.nx = (f.nx + 1) / 2;
  c.ny = (f.ny + 1) / 2;
  c.nz = (f.nz + 1) / 2;
  c.dx = 2.0 * f.dx;
  c.dy = 2.0 * f.dy;
  c.dz = 2.0 * f.dz;
  if (bin) {
    c.nu = (f.nu + 1) / 2;
    c.nv = (f.nv + 1) / 2;
    c.du = 2.0 * f.du;
    c.dv = 2.0 * f.dv;
  }
  return c;
}

// Every grid of the schedule must pass the geometry checks (a coarser grid
// is larger in mm: ceil sizes at twice the voxel), and a detector binned
// 2 x 2 for the next-coarser grid must have even sizes, so each coarse pixel
// centre is the mean of the four fine centres it averages.
tfcb_status validate_schedule(const tfcb_geometry& g, const tfcb_options& o) {
  tfcb_geometry cur = g;
  for (int l = 1; l < o.n_grids; ++l) {
    if (o.bin_coarse_detector && (cur.nu % 2 != 0 || cur.nv % 2 != 0))
      return fail(TFCB_EUNSUPPORTED,
                  "2x2 detector binning needs even detector sizes on every grid but the "
                  "coarsest (grid %d is %d x %d)", l - 1, cur.nu, cur.nv);
    cur = coarse_of(cur, o.bin_coarse_detector != 0);
    const tfcb_status st = validate_geometry(&cur);
    if (st != TFCB_OK)
      return fail(st, "coarse grid %d (%d x %d x %d): %s", l, cur.nx, cur.ny, cur.nz,
                  g_last_error.c_str());
  }
  return TFCB_OK;
}

// Sequential carving of a workspace into aligned sub-buffers.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  }
};

// ----------------------------------------------------- per-grid buffers
struct GridBufs {
  tfcb_geometry geom;
  GeomDev gd;
  ViewInfo* views;
  ColInfo* cols;
  void *x0, *x1, *s, *f0, *f1;  // volumes [z][y][x]
  void *pN, *pT;                // CGLS direction: padded native / transposed copies
  void* t2;                     // second framelet scratch (two levels only)
  float* tvg;                   // TV: gradient of the ROF energy (FP32 volume)
  void* rof_state;              // TV: descent state
  size_t pN_elems, pT_elems;
  void *g, *r, *rl, *q;         // projections
  double* partials;
  int max_partials;
  int op_pair;  // 0: Joseph P + exact transpose; 1: Siddon P + Eq. (3)
};

struct Plan {
  int n_grids = 1;
  GridBufs grid[4];
  CglsScalars* sc = nullptr;
  int* flag = nullptr;  // non-finite flag + 1024 doubles of partials
  size_t bytes = 0;
};

// Lays out every buffer of a reconstruction (or of a single-grid CGLS call
// when n_grids = 1).  ws == nullptr only measures.
void make_plan(const tfcb_geometry& g, const tfcb_options& o, void* ws, Plan& P) {
  Carver cv(ws);
  const size_t es = dtype_size(o.storage);
  P.n_grids = o.n_grids;
  P.sc = static_cast<CglsScalars*>(cv.take(sizeof(CglsScalars)));
  P.flag = static_cast<int*>(cv.take(8 + 1024 * sizeof(double)));
  tfcb_geometry cur = g;
  for (int l = 0; l < o.n_grids; ++l) {
    if (l > 0) cur = coarse_of(cur, o.bin_coarse_detector != 0);
    GridBufs& b = P.grid[l];
    b.geom = cur;
    b.gd = make_geom_dev(cur);
    b.op_pair = o.op_pair;
    b.views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * cur.n_views));
    b.cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)cur.n_views * cur.nu));
    const size_t V = nvox(cur) * es, S = npix(cur) * es;
    b.x0 = cv.take(V);
    b.x1 = cv.take(V);
    b.pN_elems = pad_elems(cur.ny, cur.nx, cur.nz);
    b.pT_elems = pad_elems(cur.nx, cur.ny, cur.nz);
    b.pN = cv.take(b.pN_elems * es);
    b.pT = cv.take(b.pT_elems * es);
    b.s = cv.take(V);
    b.t2 = (o.framelet_levels == 2 && o.regulariser == 0) ? cv.take(V) : nullptr;
    b.tvg = o.regulariser == 1 ? static_cast<float*>(cv.take(nvox(cur) * sizeof(float)))
                               : nullptr;
    b.rof_state = o.regulariser == 1 ? cv.take(rof_state_bytes()) : nullptr;
    b.f0 = cv.take(V);
    b.f1 = cv.take(V);
    b.g = cv.take(S);
    b.r = cv.take(S);
    b.rl = cv.take(S);
    b.q = cv.take(S);
    b.max_partials = std::max(project_num_blocks(b.gd), backproject_num_blocks(b.gd));
    if (o.regulariser == 1)
      b.max_partials = std::max(b.max_partials, rof_num_partials(cur.nx, cur.ny, cur.nz));
    b.partials = static_cast<double*>(cv.take(sizeof(double) * b.max_partials));
  }
  P.bytes = cv.off;
}

// Device-side tables of one grid (the view angles of b.geom, if any, are
// read from the host array during this call), and the zero pads of its
// padded direction copies (never written later).
template <typename T>
tfcb_status setup_grid(const GridBufs& b, hipStream_t s) {
  TFCB_HIP(launch_geom_tables(b.geom, b.views, b.cols, s));
  TFCB_HIP(launch_fill(b.pN_elems, 0.f, static_cast<T*>(b.pN), s));
  TFCB_HIP(launch_fill(b.pT_elems, 0.f, static_cast<T*>(b.pT), s));
  return TFCB_OK;
}

// Optional event timing of the P, P^T and framelet launches (classes 0-2),
// recorded on the launching stream.
struct Profiler {
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  ~Profiler() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipError_t mark(int c) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    ev.push_back(e);
    cls.push_back(c);
    return hipEventRecord(e, s);
  }
  // after a synchronisation: per-class sums of (end - start)
  hipError_t totals(double ms[4], int32_t n[4]) const {
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
      float t = 0.f;
      hipError_t err = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      if (err != hipSuccess) return err;
      ms[cls[i]] += t;
      n[cls[i]] += 1;
    }
    return hipSuccess;
  }
};

#define TFCB_TIMED(prof, c, expr)                  \
  do {                                             \
    if (prof) TFCB_HIP((prof)->mark(c));           \
    TFCB_HIP(expr);                                \
    if (prof) TFCB_HIP((prof)->mark(c));           \
  } while (0)

// --------------------------------------------------------------- CGLS
// The grid's operator pair: P of a direction held as its padded copies
// (mode 1: r = g - P x with rl = l r for the Joseph pair; mode 2: q = P p),
// and the backprojection that stands for P^T (the exact transpose of the
// length-prescaled rl, or Eq. (3) of plain r).
template <typename T>
hipError_t pair_project(const GridBufs& b, const T* pN, const T* pT, int mode, const T* gin,
                        T* out, T* rl, int* np, hipStream_t s) {
  if (b.op_pair == 1)
    return launch_project_siddon(b.gd, b.views, pN, pT, mode, gin, out, b.partials, np, s);
  return launch_project(b.gd, b.views, b.cols, pN, pT, mode, gin, out, rl, b.partials, np, s);
}
template <typename T>
hipError_t pair_backproject(const GridBufs& b, const T* r, const T* rl, T* out, int* np,
                            hipStream_t s) {
  if (b.op_pair == 1) return launch_backproject_eq3(b.gd, b.views, r, out, b.partials, np, s);
  return launch_backproject(b.gd, b.views, b.cols, rl, out, b.partials, np, s);
}

template <typename T>
tfcb_status run_cgls(const GridBufs& b, CglsScalars* sc, T* x, const T* gin, int n,
                     hipStream_t s, Profiler* prof = nullptr) {
  const GeomDev& g = b.gd;
  T* pN = static_cast<T*>(b.pN);
  T* pT = static_cast<T*>(b.pT);
  T* sv = static_cast<T*>(b.s);
  T* r = static_cast<T*>(b.r);
  T* rl = static_cast<T*>(b.rl);
  T* q = static_cast<T*>(b.q);
  int np = 0;
  const double nv = (double)g.nx * g.ny * g.nz;
  // r = g - P x (rl = l r)   (x reaches P through the padded copies)
  TFCB_HIP(launch_pad_copies(g.nx, g.ny, g.nz, (const T*)x, pN, pT, s));
  TFCB_TIMED(prof, 0, pair_project(b, (const T*)pN, (const T*)pT, 1, gin, r, rl, &np, s));
  TFCB_HIP(launch_finalize(b.partials, np, FIN_RESID, sc, nv, s));
  // s = P^T r; gamma = ||s||^2
  TFCB_TIMED(prof, 1, pair_backproject(b, (const T*)r, (const T*)rl, sv, &np, s));
  TFCB_HIP(launch_finalize(b.partials, np, FIN_GAMMA_INIT, sc, nv, s));
  // pn = s / sigma, as its two padded copies
  TFCB_HIP(launch_xp_update(g.nx, g.ny, g.nz, 0, x, pN, pT, (const T*)sv, sc, s));
  for (int l = 0; l < n; ++l) {
    // q = P p; alpha = gamma / ||q||^2 (or stop)
    TFCB_TIMED(prof, 0, pair_project(b, (const T*)pN, (const T*)pT, 2,
                                     static_cast<const T*>(nullptr), q, static_cast<T*>(nullptr),
                                     &np, s));
    TFCB_HIP(launch_finalize(b.partials, np, FIN_ALPHA, sc, nv, s));
    // r -= alpha q; rl = l r
    TFCB_HIP(launch_residual_update(g, b.views, b.cols, r, q, rl, sc, b.partials, &np, s));
    TFCB_HIP(launch_finalize(b.partials, np, FIN_RESID, sc, nv, s));
    if (l < n - 1) {
      // s = P^T r; beta = ||s||^2 / gamma; x += alpha p; p = s + beta p
      TFCB_TIMED(prof, 1, pair_backproject(b, (const T*)r, (const T*)rl, sv, &np, s));
      TFCB_HIP(launch_finalize(b.partials, np, FIN_BETA, sc, nv, s));
      TFCB_HIP(launch_xp_update(g.nx, g.ny, g.nz, 1, x, pN, pT, (const T*)sv, sc, s));
    } else {
      TFCB_HIP(launch_xp_update(g.nx, g.ny, g.nz, 2, x, pN, pT, (const T*)sv, sc, s));
    }
  }
  return TFCB_OK;
}

// Momentum coefficients of Algorithm A2: c[k] = (t_{k-1} - 1) / t_k with
// t_{-1} = t_0 = 1 and t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2.
std::vector<double> momentum_schedule(int n, bool momentum) {
  std::vector<double> c(n + 2, 0.0);
  double tp = 1.0, tc = 1.0;
  for (int k = 0; k < n + 2; ++k) {
    c[k] = momentum ? (tp - 1.0) / tc : 0.0;
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tc * tc));
    tp = tc;
    tc = tn;
  }
  return c;
}

// One framelet regularisation step: out = H(W^T T W x) and vnext =
// out + mom (out - fcur).  tmp1/tmp2 are volume scratch for two levels.
template <typename T>
tfcb_status run_framelet(const tfcb_geometry& g, int levels, float lambda, int positivity,
                         const T* x, T* out, const T* fcur, T* vnext, float mom, T* tmp1,
                         T* tmp2, hipStream_t s, Profiler* prof = nullptr) {
  if (prof) TFCB_HIP(prof->mark(2));
  const T* low = nullptr;
  if (levels == 2) {
    TFCB_HIP(launch_lowpass(g.nx, g.ny, g.nz, x, tmp1, s));
    TFCB_HIP(launch_framelet(g.nx, g.ny, g.nz, 2, lambda, 0, (const T*)tmp1,
                             static_cast<const T*>(nullptr), tmp2, static_cast<const T*>(nullptr),
                             static_cast<T*>(nullptr), 0.f, s));
    low = tmp2;
  }
  TFCB_HIP(launch_framelet(g.nx, g.ny, g.nz, 1, lambda, positivity, x, low, out, fcur, vnext,
                           mom, s));
  if (prof) TFCB_HIP(prof->mark(2));
  return TFCB_OK;
}

template <typename T>
tfcb_status reconstruct_t(const tfcb_geometry& g, const tfcb_options& o, const float* proj,
                          float* vol, const Plan& P, hipStream_t s, tfcb_report* rep) {
  TFCB_HIP(launch_cgls_reset(P.sc, s));
  const int ng = o.n_grids;
  for (int l = 0; l < ng; ++l) TFCB_TRY(setup_grid<T>(P.grid[l], s));
  // projections of every grid: the finest converted to the storage type,
  // coarser ones binned (or copied) from the next finer
  TFCB_HIP((launch_cast<float, T>(npix(g), proj, static_cast<T*>(P.grid[0].g), s)));
  for (int l = 1; l < ng; ++l) {
    const GridBufs& f = P.grid[l - 1];
    const GridBufs& c = P.grid[l];
    if (o.bin_coarse_detector)
      TFCB_HIP(launch_restrict(f.geom.n_views, f.geom.nu, f.geom.nv,
                               static_cast<const T*>(f.g), static_cast<T*>(c.g), s));
    else
      TFCB_HIP(launch_copy(npix(c.geom), static_cast<const T*>(f.g), static_cast<T*>(c.g), s));
  }
  hipEvent_t ev[5];
  for (int e = 0; e <= ng; ++e) TFCB_HIP(hipEventCreate(&ev[e]));
  struct EvGuard {
    hipEvent_t* e;
    int n;
    ~EvGuard() {
      for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev, ng + 1};
  TFCB_HIP(hipEventRecord(ev[0], s));

  Profiler prof;
  prof.s = s;
  int rof_steps = 0;
  T* cur = nullptr;  // f_cur of the previous (coarser) grid
  for (int l = ng - 1; l >= 0; --l) {
    const GridBufs& b = P.grid[l];
    const tfcb_geometry& gg = b.geom;
    const size_t V = nvox(gg);
    T* f_cur = static_cast<T*>(b.f0);
    T* f_nxt = static_cast<T*>(b.f1);
    T* xa = static_cast<T*>(b.x0);
    T* xb = static_cast<T*>(b.x1);
    if (l == ng - 1) {
      TFCB_HIP(launch_fill(V, 0.f, f_cur, s));
    } else {
      TFCB_HIP(launch_prolong(P.grid[l + 1].geom, gg, (const T*)cur, f_cur, s));
    }
    // v_0 = f_0 (the first momentum coefficient is 0)
    TFCB_HIP(launch_copy(V, (const T*)f_cur, xa, s));
    const int K = o.iters[ng - 1 - l];
    const std::vector<double> mom = momentum_schedule(K, o.momentum != 0);
    for (int k = 0; k < K; ++k) {
      Profiler* pf = (o.profile && l == 0) ? &prof : nullptr;
      if (o.regulariser == 1) {
        // the TV method (section 2.3): x = CGLS(f) from v = f, f = H(ROF(x))
        if (k > 0) TFCB_HIP(launch_copy(V, (const T*)f_cur, xa, s));
        TFCB_TRY(run_cgls<T>(b, P.sc, xa, static_cast<const T*>(b.g), o.cgls_steps, s, pf));
        int steps = 0;
        if (pf) TFCB_HIP(pf->mark(2));
        TFCB_HIP(launch_rof<T>(gg.nx, gg.ny, gg.nz, (float)o.lambda, (float)o.tv_eps, o.tv_tol,
                               o.tv_max_steps, o.positivity, (const T*)xa, f_nxt, b.tvg,
                               b.rof_state, b.partials, &steps, s));
        if (pf) TFCB_HIP(pf->mark(2));
        rof_steps += steps;
        std::swap(f_cur, f_nxt);
        continue;
      }
      TFCB_TRY(run_cgls<T>(b, P.sc, xa, static_cast<const T*>(b.g), o.cgls_steps, s, pf));
      TFCB_TRY(run_framelet<T>(gg, o.framelet_levels, (float)o.lambda, o.positivity, xa, f_nxt,
                               f_cur, xb, (float)mom[k + 1], static_cast<T*>(b.s),
                               static_cast<T*>(b.t2), s, pf));
      std::swap(f_cur, f_nxt);
      std::swap(xa, xb);
    }
    cur = f_cur;
    TFCB_HIP(hipEventRecord(ev[ng - l], s));
  }
  TFCB_HIP((launch_cast<T, float>(nvox(g), (const T*)cur, vol, s)));
  TFCB_HIP(launch_nonfinite(nvox(g), (const float*)vol, P.flag, s));
  CglsScalars sc_host;
  int flag_host = 0;
  TFCB_HIP(hipMemcpyAsync(&sc_host, P.sc, sizeof sc_host, hipMemcpyDeviceToHost, s));
  TFCB_HIP(hipMemcpyAsync(&flag_host, P.flag, sizeof flag_host, hipMemcpyDeviceToHost, s));
  TFCB_HIP(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof *rep);
    float ms = 0.f;
    TFCB_HIP(hipEventElapsedTime(&ms, ev[0], ev[ng]));
    rep->seconds_total = ms * 1e-3;
    for (int i = 0; i < ng; ++i) {
      TFCB_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      rep->seconds_per_grid[i] = ms * 1e-3;
      rep->iters_done[i] = o.iters[i];
    }
    rep->resid2_last = sc_host.resid2;
    rep->cgls_breakdowns = sc_host.breakdowns;
    rep->rof_steps = rof_steps;
    if (o.profile) {
      TFCB_HIP(prof.totals(rep->kernel_ms, rep->kernel_launches));
      rep->kernel_ms[3] =
          rep->seconds_per_grid[ng - 1] * 1e3 - rep->kernel_ms[0] - rep->kernel_ms[1] -
          rep->kernel_ms[2];
    }
  }
  if (flag_host) return fail(TFCB_ENUMERIC, "the reconstruction holds non-finite values");
  return TFCB_OK;
}

template <typename F>
tfcb_status dispatch(tfcb_dtype dt, F&& f) {
  switch (dt) {
    case TFCB_F32: return f(float{});
    case TFCB_F16: return f(__half{});
    case TFCB_BF16: return f(__hip_bfloat16{});
    default: return fail(TFCB_EINVAL, "unknown dtype %d", (int)dt);
  }
}

size_t operator_ws_bytes(const tfcb_geometry& g, tfcb_dtype dt) {
  Carver cv(nullptr);
  cv.take(sizeof(ViewInfo) * g.n_views);
  cv.take(sizeof(ColInfo) * (size_t)g.n_views * g.nu);
  // project: the two padded copies; backproject: the prescaled projections
  const size_t es = dtype_size(dt);
  const size_t proj_ws = align_up(pad_elems(g.ny, g.nx, g.nz) * es) +
                         align_up(pad_elems(g.nx, g.ny, g.nz) * es);
  cv.take(std::max(proj_ws, npix(g) * es));
  return cv.off;
}

}  // namespace
}  // namespace tfcb
