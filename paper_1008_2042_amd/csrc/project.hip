// Forward projector P: the line integral of Eq. (1) discretised by Joseph's
// method.
//
// Mapping: a 256-thread block covers 64 detector columns x 4 RPT rows of one
// view.  Each wavefront takes RPT adjacent detector rows; its 64 lanes are
// adjacent columns, whose crossings with a plane of the stepping axis are
// adjacent in the trans axis, the fastest axis of the volume copy the view
// reads (native [z][y][x] for y-stepping views, [z][x][y] for x-stepping
// views).  The rows of one column cross a plane at the same trans position
// (it depends on the column only) and at z positions less than NL - 2 slices
// apart, so one thread loads a stack of NL consecutive z levels of the plane
// (one 8-byte load of the two trans taps per level), interpolates each level
// in trans once, and takes every row's bilinear sample from the two levels
// around it.  RPT = 1 (NL = 2) is the one-ray-per-thread kernel.  PU planes
// per iteration, alternating between two accumulator sets.
#include <cmath>

#include "tfcb_internal.h"

namespace tfcb {

// The sample of plane p: fractional trans and z indices, evaluated exactly
// as the backprojector evaluates its weights.
__device__ __forceinline__ float trans_index(const ColInfo& ci, int p) {
  return fmaf((float)p, ci.dt, ci.t0);
}
__device__ __forceinline__ float z_index(const ColInfo& ci, int p, float vz, float zc) {
  return fmaf(fmaf((float)p, ci.dtau, ci.tau0), vz, zc);
}
__device__ __forceinline__ bool sample_inside(const ColInfo& ci, int p, float vz, float zc,
                                              int nt, int nz) {
  const float th = trans_index(ci, p), zh = z_index(ci, p, vz, zc);
  return th > -1.f && th < (float)nt && zh > -1.f && zh < (float)nz;
}

// The planes [lo, hi] whose sample has trans index in (-1, nt) and z index
// in (-1, nz), exactly as the loop evaluates them: both indices are
// monotone in p, so the set is an interval; a division gives it to within a
// plane, and the ends are then trimmed by evaluating the samples themselves.
__device__ __forceinline__ void plane_range(const ColInfo& ci, float vz, float zc, int nt, int nz,
                                            int& lo, int& hi) {
  float a = (float)ci.p_lo, b = (float)ci.p_hi;
  // trans: t0 + p dt in (-1, nt)
  if (ci.dt != 0.f) {
    float q1 = (-1.f - ci.t0) / ci.dt, q2 = ((float)nt - ci.t0) / ci.dt;
    a = fmaxf(a, floorf(fminf(q1, q2)) - 1.f);
    b = fminf(b, ceilf(fmaxf(q1, q2)) + 1.f);
  } else if (!(ci.t0 > -1.f && ci.t0 < (float)nt)) {
    b = a - 1.f;
  }
  // z: (tau0 + p dtau) vz + zc in (-1, nz)
  const float z0 = fmaf(ci.tau0, vz, zc), dz = ci.dtau * vz;
  if (dz != 0.f) {
    float q1 = (-1.f - z0) / dz, q2 = ((float)nz - z0) / dz;
    a = fmaxf(a, floorf(fminf(q1, q2)) - 1.f);
    b = fminf(b, ceilf(fmaxf(q1, q2)) + 1.f);
  } else if (!(z0 > -1.f && z0 < (float)nz)) {
    b = a - 1.f;
  }
  lo = (int)a;
  hi = (int)b;
  while (lo <= hi && !sample_inside(ci, lo, vz, zc, nt, nz)) ++lo;
  while (hi >= lo && !sample_inside(ci, hi, vz, zc, nt, nz)) --hi;
}

// The samples of plane p for the RPT rows of one column (row j's z factor
// vz[j], increasing in j).  The padded copy `vb` points at element
// (0, 0, 0); trans stride 1, plane stride ntp, z stride zs.
//
// Within the union of the rows' plane windows the lowest row's z index is
// above -(NL - 1) and below nz, so the NL levels from its floor lie in
// [-kZPad, nz + kZPad) (the host picks RPT and NL so that the rows span fewer
// than NL - 2 slices).  A row outside its own window there has both taps in
// the zero pads, or one with weight exactly zero, and adds exactly 0; inside
// its window its sample is the one-ray bilinear sample bit for bit.
template <typename T, int RPT, int NL>
__device__ __forceinline__ void sample_rows(const T* __restrict__ vb, const ColInfo& ci, int p,
                                            const float (&vz)[RPT], float zc, int nt, int nz,
                                            int ns, int ntp, int zs, float (&acc)[RPT]) {
  const float th = trans_index(ci, p);
  const float tf = floorf(th);
  // inside the window it is already in [-1, nt-1]; the clamps only
  // guarantee in-buffer addresses
  const int it = min(max((int)tf, -1), nt - 1);
  const float wt = th - tf;
  float zh[RPT], zf[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    zh[j] = z_index(ci, p, vz[j], zc);
    zf[j] = floorf(zh[j]);
  }
  const int iz0 = min(max((int)zf[0], -kZPad), nz - 1);
  const T* __restrict__ q = vb + ((iz0 * ns + p) * ntp + it);
  float lev[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const float v0 = ld(q + l * zs), v1 = ld(q + l * zs + 1);
    lev[l] = fmaf(wt, v1 - v0, v0);
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    float lo = lev[0], up = lev[1];
    if (j > 0) {
      const int d = (int)zf[j] - iz0;
#pragma unroll
      for (int l = 1; l < NL - 1; ++l)
        if (d >= l) {
          lo = lev[l];
          up = lev[l + 1];
        }
    }
    acc[j] += fmaf(zh[j] - zf[j], up - lo, lo);
  }
}

template <typename T, int MODE, int RPT, int NL, int PU = 2>
__global__ __launch_bounds__(256) void k_project(GeomDev g, const ViewInfo* __restrict__ views,
                                                 const ColInfo* __restrict__ cols,
                                                 const T* __restrict__ padN,
                                                 const T* __restrict__ padT,
                                                 const T* __restrict__ gin, T* __restrict__ out,
                                                 T* __restrict__ rl, double* __restrict__ partials) {
  static_assert(NL >= 2 && NL <= kZPad + 1 && (RPT > 1 || NL == 2), "level stack");
  static_assert(PU >= 2 && PU % 2 == 0, "planes per iteration");
  __shared__ double red[4];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * RPT;
  const int view = blockIdx.z;
  double part = 0.0;
  if (c < g.nu && r0 < g.nv) {
    const ViewInfo vi = views[view];
    const ColInfo ci = cols[(size_t)view * g.nu + c];
    const int nt = vi.step_x ? g.ny : g.nx;
    const int ns = vi.step_x ? g.nx : g.ny;
    const int nz = g.nz;
    const int ntp = nt + 1, zs = ns * ntp;
    const T* __restrict__ vb = (vi.step_x ? padT : padN) + pad_index(ns, nt, 0, 0, 0);
    const float zc = 0.5f * (float)(nz - 1);
    float vz[RPT];
    int lo = ns, hi = -1;  // union of the rows' windows
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      vz[j] = ((float)(r0 + j) - 0.5f * (float)(g.nv - 1)) * g.dvdz;
      if (r0 + j < g.nv) {
        int l, h;
        plane_range(ci, vz[j], zc, nt, nz, l, h);
        if (l <= h) {
          lo = min(lo, l);
          hi = max(hi, h);
        }
      }
    }
    // PU planes per iteration, alternate planes into two accumulator sets
    float acc0[RPT], acc1[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) acc0[j] = acc1[j] = 0.f;
    int p = lo;
    for (; p + PU - 1 <= hi; p += PU) {
#pragma unroll
      for (int u = 0; u < PU; u += 2) {
        sample_rows<T, RPT, NL>(vb, ci, p + u, vz, zc, nt, nz, ns, ntp, zs, acc0);
        sample_rows<T, RPT, NL>(vb, ci, p + u + 1, vz, zc, nt, nz, ns, ntp, zs, acc1);
      }
    }
    for (; p <= hi; ++p) sample_rows<T, RPT, NL>(vb, ci, p, vz, zc, nt, nz, ns, ntp, zs, acc0);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = r0 + j;
      if (r >= g.nv) break;
      const float ell = ray_length(g, vi, ci, r);
      const size_t o = ((size_t)view * g.nv + r) * g.nu + c;
      const float val = ell * (acc0[j] + acc1[j]);
      if (MODE == 0) {
        st(out + o, val);
      } else if (MODE == 1) {
        const float res = ld(gin + o) - val;
        st(out + o, res);
        const float rs = ld(out + o);  // the stored (rounded) residual
        st(rl + o, ell * rs);
        part += (double)rs * (double)rs;
      } else {
        st(out + o, val);
        const float qs = ld(out + o);
        part += (double)qs * (double)qs;
      }
    }
  }
  if (MODE != 0) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

// Rows per thread and z levels per plane for a geometry.  On a plane inside
// the volume the ray parameter is below tau_max = (sad + half-diagonal of
// the volume grown by two voxels) / sdd (the sample is at most that far from
// the source, the detector at least sdd), so adjacent rows are less than
// dv/dz tau_max slices apart; RPT rows then span less than
// (RPT - 1) dv/dz tau_max slices and need that many levels plus two (with a
// margin for FP32 rounding).  Of the admissible pairs the one with the
// fewest loads per sample, NL / RPT, is taken.
struct RowPlan {
  int rpt, nl;
};
static RowPlan row_plan(const GeomDev& g) {
  const double hx = (0.5 * g.nx + 2.0) * g.dx, hy = (0.5 * g.ny + 2.0) * g.dy;
  const double tau_max = ((double)g.sad + std::sqrt(hx * hx + hy * hy)) / (double)g.sdd;
  const double row_span = (double)g.dvdz * tau_max;
  const RowPlan cand[] = {{16, 6}, {8, 4}, {8, 6}, {4, 3}, {4, 4}, {2, 3}};
  for (const RowPlan& c : cand)
    if (std::ceil((c.rpt - 1) * row_span + 0.05) + 2.0 <= (double)c.nl) return c;
  return {1, 2};
}

int project_num_blocks(const GeomDev& g) {
  // the largest grid of any row plan (one row per thread)
  return ((g.nu + 63) / 64) * ((g.nv + 3) / 4) * g.n_views;
}

template <typename T, int MODE, int RPT, int NL>
static void launch_project_rows(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                                const T* padN, const T* padT, const T* gin, T* out, T* rl,
                                double* partials, int* n_partials, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nu + 63) / 64, (g.nv + 4 * RPT - 1) / (4 * RPT), g.n_views);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL((k_project<T, MODE, RPT, NL>), grid, block, 0, s, g, views, cols, padN, padT,
                     gin, out, rl, partials);
}

template <typename T, int MODE>
static void launch_project_mode(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                                const T* padN, const T* padT, const T* gin, T* out, T* rl,
                                double* partials, int* n_partials, hipStream_t s) {
  const RowPlan rp = row_plan(g);
  if (rp.rpt == 16)
    launch_project_rows<T, MODE, 16, 6>(g, views, cols, padN, padT, gin, out, rl, partials,
                                        n_partials, s);
  else if (rp.rpt == 8 && rp.nl == 4)
    launch_project_rows<T, MODE, 8, 4>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else if (rp.rpt == 8)
    launch_project_rows<T, MODE, 8, 6>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else if (rp.rpt == 4 && rp.nl == 3)
    launch_project_rows<T, MODE, 4, 3>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else if (rp.rpt == 4)
    launch_project_rows<T, MODE, 4, 4>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else if (rp.rpt == 2)
    launch_project_rows<T, MODE, 2, 3>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else
    launch_project_rows<T, MODE, 1, 2>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
}

template <typename T>
hipError_t launch_project(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                          const T* padN, const T* padT, int mode, const T* gin, T* out, T* rl,
                          double* partials, int* n_partials, hipStream_t s) {
  if (mode == 0)
    launch_project_mode<T, 0>(g, views, cols, padN, padT, gin, out, rl, partials, n_partials, s);
  else if (mode == 1)
    launch_project_mode<T, 1>(g, views, cols, padN, padT, gin, out, rl, partials, n_partials, s);
  else
    launch_project_mode<T, 2>(g, views, cols, padN, padT, gin, out, rl, partials, n_partials, s);
  return hipGetLastError();
}

// rl = l * in for every ray.
template <typename T>
__global__ __launch_bounds__(256) void k_prescale(GeomDev g, const ViewInfo* __restrict__ views,
                                                  const ColInfo* __restrict__ cols,
                                                  const T* __restrict__ in, T* __restrict__ out) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int view = blockIdx.z;
  if (c >= g.nu || r >= g.nv) return;
  const ViewInfo vi = views[view];
  const ColInfo ci = cols[(size_t)view * g.nu + c];
  const size_t o = ((size_t)view * g.nv + r) * g.nu + c;
  st(out + o, ray_length(g, vi, ci, r) * ld(in + o));
}

template <typename T>
hipError_t launch_prescale(const GeomDev& g, const ColInfo* cols, const ViewInfo* views,
                           const T* in, T* out, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nu + 63) / 64, (g.nv + 3) / 4, g.n_views);
  hipLaunchKernelGGL((k_prescale<T>), grid, block, 0, s, g, views, cols, in, out);
  return hipGetLastError();
}

// r -= alpha q (skipped after a breakdown); rl = l * r; partial ||r||^2.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_update(GeomDev g,
                                                         const ViewInfo* __restrict__ views,
                                                         const ColInfo* __restrict__ cols,
                                                         T* __restrict__ r, const T* __restrict__ q,
                                                         T* __restrict__ rl,
                                                         const CglsScalars* __restrict__ sc,
                                                         double* __restrict__ partials) {
  __shared__ double red[4];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int row = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int view = blockIdx.z;
  double part = 0.0;
  if (c < g.nu && row < g.nv) {
    const ViewInfo vi = views[view];
    const ColInfo ci = cols[(size_t)view * g.nu + c];
    const size_t o = ((size_t)view * g.nv + row) * g.nu + c;
    float rv = ld(r + o);
    if (!sc->stopped) {
      rv = rv - (float)sc->alpha * ld(q + o);
      st(r + o, rv);
      rv = ld(r + o);
    }
    st(rl + o, ray_length(g, vi, ci, row) * rv);
    part = (double)rv * (double)rv;
  }
  const double s = wave_block_sum(part, red);
  if (threadIdx.x == 0)
    partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

template <typename T>
hipError_t launch_residual_update(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                                  T* r, const T* q, T* rl, const CglsScalars* sc,
                                  double* partials, int* n_partials, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nu + 63) / 64, (g.nv + 3) / 4, g.n_views);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL((k_residual_update<T>), grid, block, 0, s, g, views, cols, r, q, rl, sc,
                     partials);
  return hipGetLastError();
}

#define TFCB_INST(T)                                                                            \
  template hipError_t launch_project<T>(const GeomDev&, const ViewInfo*, const ColInfo*,         \
                                        const T*, const T*, int, const T*, T*, T*, double*,     \
                                        int*, hipStream_t);                                     \
  template hipError_t launch_prescale<T>(const GeomDev&, const ColInfo*, const ViewInfo*,        \
                                         const T*, T*, hipStream_t);                            \
  template hipError_t launch_residual_update<T>(const GeomDev&, const ViewInfo*, const ColInfo*, \
                                                T*, const T*, T*, const CglsScalars*, double*,   \
                                                int*, hipStream_t);
TFCB_INST(float)
TFCB_INST(__half)
TFCB_INST(__hip_bfloat16)
#undef TFCB_INST

}  // namespace tfcb
