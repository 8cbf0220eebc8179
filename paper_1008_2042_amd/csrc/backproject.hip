// Backprojector P^T: the exact transpose of the Joseph projector, evaluated
// as a gather, one thread per voxel, no atomics (the paper's section 2.2.2
// motivates a voxel-driven P^T by the write conflicts of a ray-driven one;
// here the voxel-driven form is the exact matrix transpose rather than the
// continuous closed form of Eq. (3)).
//
// For voxel (i, j, k) and a view stepping along axis s, the voxel lies on
// plane p (its index along s) at trans index t.  Ray (c, r) weights it by
// l(c,r) * hat(t_p(c) - t) * hat(z_p(c,r) - k), the same FP32 expressions
// (same table entries, same operation order) as the projector.  The columns
// with hat(t_p(c) - t) > 0 are those whose detector coordinate lies between
// the projections of the trans neighbours t - 1 and t + 1 on plane p; for
// each such column the rows follow from |tau_p(c) vz_r + zc - k| < 1.  The
// projections are prescaled by l (rl = l * g) once per application.
//
// Mapping: 256-thread blocks of 64 (x) x 4 (y) voxels of one z slice.  For a
// y-stepping view the lanes of a wavefront read adjacent detector columns;
// for an x-stepping view they sit on adjacent planes and read nearly the
// same (column, row) footprint.  Both are served by one or two cache lines
// per tap.
#include "tfcb_internal.h"

namespace tfcb {

// Voxels per thread along z: one thread accumulates K consecutive voxels of
// an (x, y) column, sharing the per-view and per-column work, and loads each
// detector row of a column's footprint once.
constexpr int kZRun = 8;

template <typename T, int K>
__global__ __launch_bounds__(256) void k_backproject(GeomDev g, const ViewInfo* __restrict__ views,
                                                     const ColInfo* __restrict__ cols,
                                                     const T* __restrict__ rl,
                                                     T* __restrict__ vol,
                                                     double* __restrict__ partials) {
  __shared__ double red[4];
  extern __shared__ float vz_tab[];  // vz_r = (r - (nv-1)/2) dv/dz, as the projector forms it
  const float rc = 0.5f * (float)(g.nv - 1);
  for (int r = threadIdx.x; r < g.nv; r += blockDim.x) vz_tab[r] = ((float)r - rc) * g.dvdz;
  __syncthreads();
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k0 = blockIdx.z * K;
  const bool active = i < g.nx && j < g.ny;
  double part = 0.0;
  if (active) {
    const float xc = 0.5f * (float)(g.nx - 1), yc = 0.5f * (float)(g.ny - 1);
    const float zc = 0.5f * (float)(g.nz - 1);
    const float cu = 0.5f * (float)(g.nu - 1);
    const float inv_du = 1.f / g.du;
    const float X = ((float)i - xc) * g.dx, Y = ((float)j - yc) * g.dy;
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.f;
    for (int view = 0; view < g.n_views; ++view) {
      const ViewInfo vi = views[view];
      int p, t;
      float Xa, Ya, Xb, Yb;  // the trans neighbours t - 1 and t + 1 on plane p
      if (vi.step_x) {
        p = i;
        t = j;
        Xa = X; Xb = X;
        Ya = Y - g.dy; Yb = Y + g.dy;
      } else {
        p = j;
        t = i;
        Ya = Y; Yb = Y;
        Xa = X - g.dx; Xb = X + g.dx;
      }
      // detector column of a point: u = sdd (-x sn + y cs) / (sad - (x cs + y sn));
      // the columns are only bracketed here (one column of slack each side),
      // so the hardware reciprocal is accurate enough
      const float ua = g.sdd * (-Xa * vi.sn + Ya * vi.cs) *
                       __builtin_amdgcn_rcpf(g.sad - (Xa * vi.cs + Ya * vi.sn));
      const float ub = g.sdd * (-Xb * vi.sn + Yb * vi.cs) *
                       __builtin_amdgcn_rcpf(g.sad - (Xb * vi.cs + Yb * vi.sn));
      const float ca = fmaf(ua, inv_du, cu), cb = fmaf(ub, inv_du, cu);
      const int clo = max(0, (int)floorf(fminf(ca, cb)));
      const int chi = min(g.nu - 1, (int)ceilf(fmaxf(ca, cb)));
      const ColInfo* __restrict__ cview = cols + (size_t)view * g.nu;
      const T* __restrict__ rview = rl + (size_t)view * g.nv * g.nu;
      const float fp = (float)p;
      for (int c = clo; c <= chi; ++c) {
        // both halves of the 32-byte record in two vector loads, issued together
        const float4 h0 = reinterpret_cast<const float4*>(cview + c)[0];
        const int4 h1 = reinterpret_cast<const int4*>(cview + c)[1];
        ColInfo ci;
        ci.t0 = h0.x;
        ci.dt = h0.y;
        ci.tau0 = h0.z;
        ci.dtau = h0.w;
        ci.p_lo = h1.z;
        ci.p_hi = h1.w;
        if (p < ci.p_lo || p > ci.p_hi) continue;
        const float th = fmaf(fp, ci.dt, ci.t0);
        const float wt = 1.f - fabsf(th - (float)t);
        if (wt <= 0.f) continue;
        const float tau = fmaf(fp, ci.dtau, ci.tau0);
        // The z index of row r is zh_r = tau vz_r + zc (increasing in r).
        // Segment m = the rows with floor(zh_r) = k0 - 1 + m, m = 0..K: its
        // rows give (1 - fr) of their value to voxel k0 - 1 + m and fr to
        // voxel k0 + m, fr = zh_r - (k0 - 1 + m).  Segment bounds come from
        // the inverse of the row map; a row misplaced by rounding at a bound
        // has fr within an ulp of 0 or 1, so its weights are still right.
        const float inv_s = __builtin_amdgcn_rcpf(tau * g.dvdz);
        const T* __restrict__ colp = rview + c;
        float s0[K + 1], s1[K + 1];
        int rb = min(g.nv, max(0, (int)ceilf(fmaf((float)(k0 - 1) - zc, inv_s, rc))));
#pragma unroll
        for (int m = 0; m <= K; ++m) {
          const float base = (float)(k0 - 1 + m);
          const int re = min(g.nv, max(rb, (int)ceilf(fmaf(base + 1.f - zc, inv_s, rc))));
          float a0 = 0.f, a1 = 0.f;
          for (int r = rb; r < re; ++r) {
            const float fr = fmaf(tau, vz_tab[r], zc) - base;
            const float gv = ld(colp + r * g.nu);
            a0 += gv;
            a1 = fmaf(fr, gv, a1);
          }
          s0[m] = a0;
          s1[m] = a1;
          rb = re;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fmaf(wt, s1[q] + (s0[q + 1] - s1[q + 1]), acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (k0 + q < g.nz) {
        const size_t o = ((size_t)(k0 + q) * g.ny + j) * g.nx + i;
        st(vol + o, acc[q]);
        if (partials) {
          const float sv = ld(vol + o);
          part += (double)sv * (double)sv;
        }
      }
    }
  }
  if (partials) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

int backproject_num_blocks(const GeomDev& g) {
  return ((g.nx + 63) / 64) * ((g.ny + 3) / 4) * ((g.nz + kZRun - 1) / kZRun);
}

template <typename T>
hipError_t launch_backproject(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                              const T* rl, T* vol, double* partials, int* n_partials,
                              hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, (g.nz + kZRun - 1) / kZRun);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  const size_t lds = sizeof(float) * (size_t)g.nv;
  hipLaunchKernelGGL((k_backproject<T, kZRun>), grid, block, lds, s, g, views, cols, rl, vol,
                     partials);
  return hipGetLastError();
}

template hipError_t launch_backproject<float>(const GeomDev&, const ViewInfo*, const ColInfo*,
                                              const float*, float*, double*, int*, hipStream_t);
template hipError_t launch_backproject<__half>(const GeomDev&, const ViewInfo*, const ColInfo*,
                                               const __half*, __half*, double*, int*, hipStream_t);
template hipError_t launch_backproject<__hip_bfloat16>(const GeomDev&, const ViewInfo*,
                                                       const ColInfo*, const __hip_bfloat16*,
                                                       __hip_bfloat16*, double*, int*, hipStream_t);

}  // namespace tfcb
