// Forward projector P: the line integral of Eq. (1) discretised by Joseph's
// method, one thread per ray.
//
// Mapping: a 256-thread block covers 64 detector columns x 4 rows of one
// view.  Each wavefront is one detector row; its 64 lanes are adjacent
// columns, whose crossings with a plane of the stepping axis are adjacent in
// the trans axis, which is the fastest axis of the volume copy the view
// reads (native [z][y][x] for y-stepping views, [z][x][y] for x-stepping
// views).  So the four bilinear taps of a plane are two short contiguous
// runs per wavefront, and the four rows of a block share their z taps in L1.
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

// One plane sample: bilinear interpolation of the padded copy `vb` (pointer
// at element (0, 0, 0)), trans stride 1, plane stride ntp, z stride zs.
template <typename T>
__device__ __forceinline__ float sample(const T* __restrict__ vb, const ColInfo& ci, int p,
                                        float vz, float zc, int nt, int nz, int ns, int ntp,
                                        int zs) {
  const float th = trans_index(ci, p);
  const float zh = z_index(ci, p, vz, zc);
  const float tf = floorf(th), zf = floorf(zh);
  // inside the plane window these are already in [-1, nt-1] and [-1, nz-1];
  // the clamps only guarantee in-buffer addresses
  const int it = min(max((int)tf, -1), nt - 1);
  const int iz = min(max((int)zf, -1), nz - 1);
  const float wt = th - tf, wz = zh - zf;
  const int o = (iz * ns + p) * ntp + it;
  const float v00 = ld(vb + o), v01 = ld(vb + o + 1);
  const float v10 = ld(vb + o + zs), v11 = ld(vb + o + zs + 1);
  const float a = fmaf(wt, v01 - v00, v00);
  const float b = fmaf(wt, v11 - v10, v10);
  return fmaf(wz, b - a, a);
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_project(GeomDev g, const ViewInfo* __restrict__ views,
                                                 const ColInfo* __restrict__ cols,
                                                 const T* __restrict__ padN,
                                                 const T* __restrict__ padT,
                                                 const T* __restrict__ gin, T* __restrict__ out,
                                                 T* __restrict__ rl, double* __restrict__ partials) {
  __shared__ double red[4];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int view = blockIdx.z;
  const bool active = c < g.nu && r < g.nv;
  double part = 0.0;
  if (active) {
    const ViewInfo vi = views[view];
    const ColInfo ci = cols[(size_t)view * g.nu + c];
    const int nt = vi.step_x ? g.ny : g.nx;
    const int ns = vi.step_x ? g.nx : g.ny;
    const int nz = g.nz;
    const int ntp = nt + 1, zs = ns * ntp;
    const T* __restrict__ vb = (vi.step_x ? padT : padN) + pad_index(ns, nt, 0, 0, 0);
    const float vz = ((float)r - 0.5f * (float)(g.nv - 1)) * g.dvdz;
    const float zc = 0.5f * (float)(nz - 1);
    int lo, hi;
    plane_range(ci, vz, zc, nt, nz, lo, hi);
    float acc0 = 0.f, acc1 = 0.f;
    int p = lo;
    for (; p < hi; p += 2) {
      acc0 += sample(vb, ci, p, vz, zc, nt, nz, ns, ntp, zs);
      acc1 += sample(vb, ci, p + 1, vz, zc, nt, nz, ns, ntp, zs);
    }
    if (p == hi) acc0 += sample(vb, ci, p, vz, zc, nt, nz, ns, ntp, zs);
    const float acc = acc0 + acc1;
    const float ell = ray_length(g, vi, ci, r);
    const size_t o = ((size_t)view * g.nv + r) * g.nu + c;
    const float val = ell * acc;
    if (MODE == 0) {
      st(out + o, val);
    } else if (MODE == 1) {
      const float res = ld(gin + o) - val;
      st(out + o, res);
      const float rs = ld(out + o);  // the stored (rounded) residual
      st(rl + o, ell * rs);
      part = (double)rs * (double)rs;
    } else {
      st(out + o, val);
      const float qs = ld(out + o);
      part = (double)qs * (double)qs;
    }
  }
  if (MODE != 0) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

int project_num_blocks(const GeomDev& g) {
  return ((g.nu + 63) / 64) * ((g.nv + 3) / 4) * g.n_views;
}

template <typename T>
hipError_t launch_project(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                          const T* padN, const T* padT, int mode, const T* gin, T* out, T* rl,
                          double* partials, int* n_partials, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nu + 63) / 64, (g.nv + 3) / 4, g.n_views);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  if (mode == 0)
    hipLaunchKernelGGL((k_project<T, 0>), grid, block, 0, s, g, views, cols, padN, padT, gin, out,
                       rl, partials);
  else if (mode == 1)
    hipLaunchKernelGGL((k_project<T, 1>), grid, block, 0, s, g, views, cols, padN, padT, gin, out,
                       rl, partials);
  else
    hipLaunchKernelGGL((k_project<T, 2>), grid, block, 0, s, g, views, cols, padN, padT, gin, out,
                       rl, partials);
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
