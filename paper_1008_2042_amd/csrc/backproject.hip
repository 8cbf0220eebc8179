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

template <typename T>
__global__ __launch_bounds__(256) void k_backproject(GeomDev g, const ViewInfo* __restrict__ views,
                                                     const ColInfo* __restrict__ cols,
                                                     const T* __restrict__ rl,
                                                     T* __restrict__ vol,
                                                     double* __restrict__ partials) {
  __shared__ double red[4];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  const bool active = i < g.nx && j < g.ny;
  double part = 0.0;
  if (active) {
    const float xc = 0.5f * (float)(g.nx - 1), yc = 0.5f * (float)(g.ny - 1);
    const float zc = 0.5f * (float)(g.nz - 1), rc = 0.5f * (float)(g.nv - 1);
    const float cu = 0.5f * (float)(g.nu - 1);
    const float inv_du = 1.f / g.du;
    const float kf = (float)k;
    const float X = ((float)i - xc) * g.dx, Y = ((float)j - yc) * g.dy;
    float acc = 0.f;
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
      // detector column of a point: u = sdd (-x sn + y cs) / (sad - (x cs + y sn))
      const float ua = g.sdd * (-Xa * vi.sn + Ya * vi.cs) / (g.sad - (Xa * vi.cs + Ya * vi.sn));
      const float ub = g.sdd * (-Xb * vi.sn + Yb * vi.cs) / (g.sad - (Xb * vi.cs + Yb * vi.sn));
      const float ca = fmaf(ua, inv_du, cu), cb = fmaf(ub, inv_du, cu);
      const int clo = max(0, (int)floorf(fminf(ca, cb)));
      const int chi = min(g.nu - 1, (int)ceilf(fmaxf(ca, cb)));
      const ColInfo* __restrict__ cview = cols + (size_t)view * g.nu;
      const T* __restrict__ rview = rl + (size_t)view * g.nv * g.nu;
      const float fp = (float)p;
      for (int c = clo; c <= chi; ++c) {
        const ColInfo ci = cview[c];
        if (p < ci.p_lo || p > ci.p_hi) continue;
        const float th = fmaf(fp, ci.dt, ci.t0);
        const float wt = 1.f - fabsf(th - (float)t);
        if (wt <= 0.f) continue;
        const float tau = fmaf(fp, ci.dtau, ci.tau0);
        const float inv_s = 1.f / (tau * g.dvdz);
        const int rlo = max(0, (int)floorf(fmaf(kf - 1.f - zc, inv_s, rc)));
        const int rhi = min(g.nv - 1, (int)ceilf(fmaf(kf + 1.f - zc, inv_s, rc)));
        float a = 0.f;
        for (int r = rlo; r <= rhi; ++r) {
          const float vz = ((float)r - rc) * g.dvdz;
          const float zh = fmaf(tau, vz, zc);
          const float wz = fmaxf(0.f, 1.f - fabsf(zh - kf));
          a = fmaf(wz, ld(rview + (size_t)r * g.nu + c), a);
        }
        acc = fmaf(wt, a, acc);
      }
    }
    const size_t o = ((size_t)k * g.ny + j) * g.nx + i;
    st(vol + o, acc);
    if (partials) {
      const float sv = ld(vol + o);
      part = (double)sv * (double)sv;
    }
  }
  if (partials) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

int backproject_num_blocks(const GeomDev& g) {
  return ((g.nx + 63) / 64) * ((g.ny + 3) / 4) * g.nz;
}

template <typename T>
hipError_t launch_backproject(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                              const T* rl, T* vol, double* partials, int* n_partials,
                              hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL((k_backproject<T>), grid, block, 0, s, g, views, cols, rl, vol, partials);
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
