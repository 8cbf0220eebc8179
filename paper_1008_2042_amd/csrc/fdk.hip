// FDK, the comparison baseline of the paper's experiments (section 3; the
// paper names it without details): the textbook Feldkamp-Davis-Kress
// reconstruction for an equally spaced full circular orbit and a flat
// detector.  Detector coordinates are scaled to the rotation axis,
// p = u SAD / SDD, zeta = v SAD / SDD, pitch dp = du SAD / SDD.
//
// k_fdk_filter: one block per detector row.  The row, weighted by
// SDD / sqrt(SDD^2 + u^2 + v^2), and the Ram-Lak kernel's odd taps
// (-1 / (pi n dp)^2; even taps are 0, the centre tap 1 / (4 dp^2)) are
// staged in LDS; each output pixel is dp times the linear convolution of
// the row with the kernel (zero outside the row), accumulated in FP32.
//
// k_fdk_backproject: one thread per z-run of kFdkRun voxels of one (x, y)
// column.  Per view the depth U = SAD - x.s_hat, the detector column and
// the weight (SAD / U)^2 are the run's; each voxel adds the filtered
// projections interpolated bilinearly at its detector position (taps off
// the detector read 0).  The sum is scaled by pi / n_views.
#include "tfcb_internal.h"

namespace tfcb {

constexpr int kFdkRun = 8;
constexpr int kFdkMaxRow = 8192;  // detector columns one LDS row holds (48 KB)

template <typename T>
__global__ __launch_bounds__(256) void k_fdk_filter(GeomDev g, const T* __restrict__ proj,
                                                    float* __restrict__ q, float dp) {
  extern __shared__ float lds[];
  float* w = lds;              // the weighted row, nu values
  float* h = lds + g.nu;       // h[m] = kernel tap at lag 2m + 1, m < nu / 2 + 1
  const int row = blockIdx.x;  // view * nv + r
  const int r = row % g.nv;
  const float v = ((float)r - 0.5f * (float)(g.nv - 1)) * g.dv;
  const float sdd2v2 = fmaf(g.sdd, g.sdd, v * v);
  const T* __restrict__ in = proj + (size_t)row * g.nu;
  for (int c = threadIdx.x; c < g.nu; c += 256) {
    const float u = ((float)c - 0.5f * (float)(g.nu - 1)) * g.du;
    w[c] = ld(in + c) * g.sdd * rsqrtf(fmaf(u, u, sdd2v2));
  }
  const float k_odd = -1.f / ((float)(M_PI * M_PI) * dp * dp);
  const int nh = g.nu / 2 + 1;
  for (int m = threadIdx.x; m < nh; m += 256) {
    const float n = (float)(2 * m + 1);
    h[m] = k_odd / (n * n);
  }
  __syncthreads();
  const float h0 = 0.25f / (dp * dp);
  float* __restrict__ out = q + (size_t)row * g.nu;
  for (int c = threadIdx.x; c < g.nu; c += 256) {
    float s = h0 * w[c];
    // odd lags n = 2m + 1 on both sides that stay inside the row
    for (int m = 0; m < nh; ++m) {
      const int n = 2 * m + 1;
      if (c - n < 0 && c + n >= g.nu) break;
      const float lo = c - n >= 0 ? w[c - n] : 0.f;
      const float hi = c + n < g.nu ? w[c + n] : 0.f;
      s = fmaf(h[m], lo + hi, s);
    }
    out[c] = dp * s;
  }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_fdk_backproject(GeomDev g,
                                                         const ViewInfo* __restrict__ views,
                                                         const float* __restrict__ q,
                                                         T* __restrict__ vol) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k0 = blockIdx.z * K;
  if (i >= g.nx || j >= g.ny) return;
  const float X = ((float)i - 0.5f * (float)(g.nx - 1)) * g.dx;
  const float Y = ((float)j - 0.5f * (float)(g.ny - 1)) * g.dy;
  const float zc = 0.5f * (float)(g.nz - 1);
  const float cu = 0.5f * (float)(g.nu - 1), cv = 0.5f * (float)(g.nv - 1);
  const float inv_du = 1.f / g.du, inv_dv = 1.f / g.dv;
  const size_t view_px = (size_t)g.nu * g.nv;
  float acc[K];
#pragma unroll
  for (int t = 0; t < K; ++t) acc[t] = 0.f;
  for (int view = 0; view < g.n_views; ++view) {
    const ViewInfo vi = views[view];
    const float U = g.sad - fmaf(X, vi.cs, Y * vi.sn);
    const float mag = g.sdd / U;
    const float uc = fmaf(mag * fmaf(-X, vi.sn, Y * vi.cs), inv_du, cu);
    const float wgt = (g.sad / U) * (g.sad / U);
    const int c0 = (int)floorf(uc);
    const float fc = uc - (float)c0;
    const bool in0 = c0 >= 0 && c0 < g.nu, in1 = c0 + 1 >= 0 && c0 + 1 < g.nu;
    const float* __restrict__ pv = q + view * view_px;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const float Zk = ((float)(k0 + t) - zc) * g.dz;
      const float vr = fmaf(mag * Zk, inv_dv, cv);
      const int r0 = (int)floorf(vr);
      const float fr = vr - (float)r0;
      float a = 0.f, b = 0.f;
      if (r0 >= 0 && r0 < g.nv) {
        const float* row = pv + (size_t)r0 * g.nu;
        a = fmaf(fc, (in1 ? row[c0 + 1] : 0.f) - (in0 ? row[c0] : 0.f), in0 ? row[c0] : 0.f);
      }
      if (r0 + 1 >= 0 && r0 + 1 < g.nv) {
        const float* row = pv + (size_t)(r0 + 1) * g.nu;
        b = fmaf(fc, (in1 ? row[c0 + 1] : 0.f) - (in0 ? row[c0] : 0.f), in0 ? row[c0] : 0.f);
      }
      acc[t] = fmaf(wgt, fmaf(fr, b - a, a), acc[t]);
    }
  }
  const float scale = (float)M_PI / (float)g.n_views;
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (k0 + t < g.nz) st(vol + ((size_t)(k0 + t) * g.ny + j) * g.nx + i, scale * acc[t]);
}

size_t fdk_lds_bytes(int nu) { return sizeof(float) * ((size_t)nu + nu / 2 + 1); }
bool fdk_supported(int nu) { return nu <= kFdkMaxRow; }

template <typename T>
hipError_t launch_fdk(const GeomDev& g, const ViewInfo* views, const T* proj, float* q, T* vol,
                      hipStream_t s) {
  const float dp = (float)((double)g.du * (double)g.sad / (double)g.sdd);
  hipLaunchKernelGGL((k_fdk_filter<T>), dim3((unsigned)g.n_views * g.nv), dim3(256),
                     fdk_lds_bytes(g.nu), s, g, proj, q, dp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, (g.nz + kFdkRun - 1) / kFdkRun);
  hipLaunchKernelGGL((k_fdk_backproject<T, kFdkRun>), grid, dim3(256), 0, s, g, views,
                     (const float*)q, vol);
  return hipGetLastError();
}

#define TFCB_INST_FDK(T)                                                                     \
  template hipError_t launch_fdk<T>(const GeomDev&, const ViewInfo*, const T*, float*, T*, \
                                    hipStream_t);
TFCB_INST_FDK(float)
TFCB_INST_FDK(__half)
TFCB_INST_FDK(__hip_bfloat16)

}  // namespace tfcb
