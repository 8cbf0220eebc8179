// CGLS vector steps (Appendix 1), device-side scalar logic, layout
// transposes, casts, and the multigrid transfer operators (section 2.2.3).
// Every kernel here is HBM-bound: coalesced row access, LDS tiles where a
// transpose is involved, deterministic FP64 reductions without atomics.
#include "tfcb_internal.h"

namespace tfcb {

// ------------------------------------------------------------- reductions
__global__ __launch_bounds__(kReduceThreads) void k_finalize(const double* __restrict__ partials,
                                                             int n, int mode,
                                                             CglsScalars* __restrict__ sc,
                                                             double nvox) {
  __shared__ double red[kReduceThreads / 64];
  // four independent partial sums per thread keep four loads in flight; the
  // order is fixed, so the result is the same on every call
  constexpr int T = kReduceThreads;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * T < n; i += 4 * T) {
    v0 += partials[i];
    v1 += partials[i + T];
    v2 += partials[i + 2 * T];
    v3 += partials[i + 3 * T];
  }
  for (; i < n; i += T) v0 += partials[i];
  const double sum = wave_block_sum((v0 + v1) + (v2 + v3), red);
  if (threadIdx.x != 0) return;
  const double tiny = 1e-300;
  switch (mode) {
    case FIN_GAMMA_INIT: {
      // s = P^T r of a new CGLS call; the first direction is s / sigma
      sc->gamma = sum;
      sc->stopped = 0;
      sc->alpha = 0.0;
      sc->beta_sigma = 0.0;
      const double sig = sqrt(sum / nvox);
      sc->sigma = sig > 0.0 ? sig : 1.0;
      sc->inv_sigma = 1.0 / sc->sigma;
      break;
    }
    case FIN_ALPHA: {
      // sum = ||qn||^2; ||q||^2 = sigma^2 ||qn||^2
      const double delta = sc->sigma * sc->sigma * sum;
      sc->delta = delta;
      if (sc->stopped || sc->gamma <= tiny || delta <= tiny) {
        if (!sc->stopped) sc->breakdowns += 1;
        sc->stopped = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = sc->gamma / (sc->sigma * sum);
      }
      break;
    }
    case FIN_BETA: {
      // sum = ||s'||^2: beta = gamma' / gamma, pn' = (s' + beta sigma pn) / sigma'
      if (sc->stopped) {
        sc->beta_sigma = 0.0;
        sc->inv_sigma = 1.0 / sc->sigma;
      } else {
        // with sigma' = rms(s') the two terms of pn' = s'/sigma' +
        // (sigma'/sigma) pn are both O(1): beta sigma / sigma' = sigma'/sigma
        const double beta = sum / sc->gamma;
        sc->beta_sigma = beta * sc->sigma;
        const double sig = sqrt(sum / nvox);
        sc->sigma = sig > 0.0 ? sig : 1.0;
        sc->inv_sigma = 1.0 / sc->sigma;
        sc->gamma = sum;
      }
      break;
    }
    default:
      sc->resid2 = sum;
      break;
  }
}

hipError_t launch_finalize(const double* partials, int n, int mode, CglsScalars* sc,
                           double nvox, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kReduceThreads), 0, s, partials, n, mode, sc,
                     nvox);
  return hipGetLastError();
}

__global__ void k_cgls_reset(CglsScalars* sc) {
  if (threadIdx.x == 0) {
    sc->gamma = 0.0;
    sc->delta = 0.0;
    sc->sigma = 1.0;
    sc->alpha = 0.0;
    sc->beta_sigma = 0.0;
    sc->inv_sigma = 1.0;
    sc->resid2 = 0.0;
    sc->stopped = 0;
    sc->breakdowns = 0;
  }
}

hipError_t launch_cgls_reset(CglsScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_reset, dim3(1), dim3(64), 0, s, sc);
  return hipGetLastError();
}

// ------------------------------------------------- x / p updates + transpose
// Tiles of 32 (x) x 32 (y) of one z slice; 256 threads, 4 rows each.  The
// [z][x][y] copy of p is written through an LDS tile so both layouts are
// written with full rows.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_xp_update(int nx, int ny, T* __restrict__ x,
                                                   T* __restrict__ pN, T* __restrict__ pT,
                                                   const T* __restrict__ s,
                                                   const CglsScalars* __restrict__ sc) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const bool stopped = sc->stopped != 0;
  const float alpha = (float)sc->alpha, beta_sigma = (float)sc->beta_sigma;
  const float inv_sigma = (float)sc->inv_sigma;
  const size_t zoff = (size_t)z * nx * ny;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int yy = y0 + ty + 8 * rr, xx = x0 + tx;
    if (xx < nx && yy < ny) {
      const size_t o = zoff + (size_t)yy * nx + xx;
      const int on = pad_index(ny, nx, z, yy, xx);
      float pn;
      if (MODE == 0) {
        pn = ld(s + o) * inv_sigma;
      } else {
        const float pv = ld(pN + on);
        if (!stopped) st(x + o, fmaf(alpha, pv, ld(x + o)));
        pn = (MODE == 1) ? fmaf(beta_sigma, pv, ld(s + o)) * inv_sigma : pv;
      }
      if (MODE != 2) {
        st(pN + on, pn);
        tile[ty + 8 * rr][tx] = ld(pN + on);
      }
    }
  }
  if (MODE == 2) return;
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int xx = x0 + ty + 8 * rr, yy = y0 + tx;
    if (xx < nx && yy < ny) st(pT + pad_index(nx, ny, z, xx, yy), tile[tx][ty + 8 * rr]);
  }
}

// Interior of the padded native and transposed copies of a native volume.
template <typename T>
__global__ __launch_bounds__(256) void k_pad_copies(int nx, int ny, const T* __restrict__ in,
                                                    T* __restrict__ padN, T* __restrict__ padT) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const size_t zoff = (size_t)z * nx * ny;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int yy = y0 + ty + 8 * rr, xx = x0 + tx;
    if (xx < nx && yy < ny) {
      const float v = ld(in + zoff + (size_t)yy * nx + xx);
      st(padN + pad_index(ny, nx, z, yy, xx), v);
      tile[ty + 8 * rr][tx] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int xx = x0 + ty + 8 * rr, yy = y0 + tx;
    if (xx < nx && yy < ny) st(padT + pad_index(nx, ny, z, xx, yy), tile[tx][ty + 8 * rr]);
  }
}

template <typename T>
hipError_t launch_pad_copies(int nx, int ny, int nz, const T* in, T* padN, T* padT,
                             hipStream_t s) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz);
  hipLaunchKernelGGL((k_pad_copies<T>), grid, dim3(256), 0, s, nx, ny, in, padN, padT);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xp_update(int nx, int ny, int nz, int mode, T* x, T* p, T* pT, const T* s,
                            const CglsScalars* sc, hipStream_t st_) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz);
  if (mode == 0)
    hipLaunchKernelGGL((k_xp_update<T, 0>), grid, dim3(256), 0, st_, nx, ny, x, p, pT, s, sc);
  else if (mode == 1)
    hipLaunchKernelGGL((k_xp_update<T, 1>), grid, dim3(256), 0, st_, nx, ny, x, p, pT, s, sc);
  else
    hipLaunchKernelGGL((k_xp_update<T, 2>), grid, dim3(256), 0, st_, nx, ny, x, p, pT, s, sc);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_transpose_xy(int nx, int ny, const T* __restrict__ in,
                                                      T* __restrict__ out) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const size_t zoff = (size_t)z * nx * ny;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int yy = y0 + ty + 8 * rr, xx = x0 + tx;
    if (xx < nx && yy < ny) tile[ty + 8 * rr][tx] = ld(in + zoff + (size_t)yy * nx + xx);
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int xx = x0 + ty + 8 * rr, yy = y0 + tx;
    if (xx < nx && yy < ny) st(out + zoff + (size_t)xx * ny + yy, tile[tx][ty + 8 * rr]);
  }
}

template <typename T>
hipError_t launch_transpose_xy(int nx, int ny, int nz, const T* in, T* out, hipStream_t s) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz);
  hipLaunchKernelGGL((k_transpose_xy<T>), grid, dim3(256), 0, s, nx, ny, in, out);
  return hipGetLastError();
}

// ---------------------------------------------------------- element-wise
template <typename T>
__global__ __launch_bounds__(256) void k_copy(size_t n, const T* __restrict__ in,
                                              T* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    out[i] = in[i];
}
template <typename T>
__global__ __launch_bounds__(256) void k_fill(size_t n, float v, T* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    st(out + i, v);
}
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_cast(size_t n, const Tin* __restrict__ in,
                                              Tout* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    st(out + i, ld(in + i));
}
// One partial count of non-finite values per block; a single-block pass
// then folds them into flag[0] (no atomics).
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite_part(size_t n, const T* __restrict__ in,
                                                        double* __restrict__ part) {
  __shared__ double red[4];
  double bad = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float v = ld(in + i);
    bad += (v - v != 0.f) ? 1.0 : 0.0;  // NaN or +-inf
  }
  const double s = wave_block_sum(bad, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_nonfinite_fold(const double* __restrict__ part, int n,
                                                        int* __restrict__ flag) {
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  const double s = wave_block_sum(v, red);
  if (threadIdx.x == 0) flag[0] = s > 0.0 ? 1 : 0;
}

static unsigned elementwise_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

template <typename T>
hipError_t launch_copy(size_t n, const T* in, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), dim3(elementwise_blocks(n)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(size_t n, float v, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), dim3(elementwise_blocks(n)), dim3(256), 0, s, n, v, out);
  return hipGetLastError();
}
template <typename Tin, typename Tout>
hipError_t launch_cast(size_t n, const Tin* in, Tout* out, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(elementwise_blocks(n)), dim3(256), 0, s, n, in,
                     out);
  return hipGetLastError();
}
// `flag` points at an int followed (8-byte aligned) by room for 1024 doubles.
template <typename T>
hipError_t launch_nonfinite(size_t n, const T* in, int* flag, hipStream_t s) {
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(flag) + 8);
  unsigned nb = elementwise_blocks(n);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL((k_nonfinite_part<T>), dim3(nb), dim3(256), 0, s, n, in, part);
  hipLaunchKernelGGL(k_nonfinite_fold, dim3(1), dim3(256), 0, s, part, (int)nb, flag);
  return hipGetLastError();
}

// -------------------------------------------------------------- multigrid
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(int nu, int nv, int nuc, int nvc,
                                                  const T* __restrict__ in, T* __restrict__ out) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int view = blockIdx.z;
  if (c >= nuc || r >= nvc) return;
  const T* a = in + (size_t)view * nu * nv;
  float s = 0.f;
  int cnt = 0;
  for (int dr = 0; dr < 2; ++dr)
    for (int dc = 0; dc < 2; ++dc) {
      const int rr = 2 * r + dr, cc = 2 * c + dc;
      if (rr < nv && cc < nu) {
        s += ld(a + (size_t)rr * nu + cc);
        ++cnt;
      }
    }
  st(out + ((size_t)view * nvc + r) * nuc + c, s / (float)cnt);
}

template <typename T>
hipError_t launch_restrict(int n_views, int nu, int nv, const T* in, T* out, hipStream_t s) {
  const int nuc = (nu + 1) / 2, nvc = (nv + 1) / 2;
  dim3 grid((nuc + 63) / 64, (nvc + 3) / 4, n_views);
  hipLaunchKernelGGL((k_restrict<T>), grid, dim3(256), 0, s, nu, nv, nuc, nvc, in, out);
  return hipGetLastError();
}

struct ProlongAxis {
  float df, dc;  // fine and coarse voxel sizes
  int nf, nc;
};

__device__ __forceinline__ void prolong_index(const ProlongAxis& a, int i, int& i0, int& i1,
                                              float& w1) {
  const float pos = ((float)i - 0.5f * (float)(a.nf - 1)) * a.df;
  float t = pos / a.dc + 0.5f * (float)(a.nc - 1);
  t = fminf(fmaxf(t, 0.f), (float)(a.nc - 1));
  int b = (int)floorf(t);
  b = b > a.nc - 1 ? a.nc - 1 : b;
  i0 = b;
  i1 = b + 1 < a.nc ? b + 1 : a.nc - 1;
  w1 = t - (float)b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong(ProlongAxis ax, ProlongAxis ay, ProlongAxis az,
                                                 const T* __restrict__ in, T* __restrict__ out) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= ax.nf || j >= ay.nf) return;
  int x0, x1, y0, y1, z0, z1;
  float wx, wy, wz;
  prolong_index(ax, i, x0, x1, wx);
  prolong_index(ay, j, y0, y1, wy);
  prolong_index(az, k, z0, z1, wz);
  const int ncx = ax.nc, ncy = ay.nc;
  auto at = [&](int z, int y, int x) { return ld(in + ((size_t)z * ncy + y) * ncx + x); };
  const float c00 = fmaf(wx, at(z0, y0, x1) - at(z0, y0, x0), at(z0, y0, x0));
  const float c01 = fmaf(wx, at(z0, y1, x1) - at(z0, y1, x0), at(z0, y1, x0));
  const float c10 = fmaf(wx, at(z1, y0, x1) - at(z1, y0, x0), at(z1, y0, x0));
  const float c11 = fmaf(wx, at(z1, y1, x1) - at(z1, y1, x0), at(z1, y1, x0));
  const float c0 = fmaf(wy, c01 - c00, c00), c1 = fmaf(wy, c11 - c10, c10);
  st(out + ((size_t)k * ay.nf + j) * ax.nf + i, fmaf(wz, c1 - c0, c0));
}

template <typename T>
hipError_t launch_prolong(const tfcb_geometry& co, const tfcb_geometry& fi, const T* in, T* out,
                          hipStream_t s) {
  ProlongAxis ax{(float)fi.dx, (float)co.dx, fi.nx, co.nx};
  ProlongAxis ay{(float)fi.dy, (float)co.dy, fi.ny, co.ny};
  ProlongAxis az{(float)fi.dz, (float)co.dz, fi.nz, co.nz};
  dim3 grid((fi.nx + 63) / 64, (fi.ny + 3) / 4, fi.nz);
  hipLaunchKernelGGL((k_prolong<T>), grid, dim3(256), 0, s, ax, ay, az, in, out);
  return hipGetLastError();
}

#define TFCB_INST(T)                                                                            \
  template hipError_t launch_xp_update<T>(int, int, int, int, T*, T*, T*, const T*,             \
                                          const CglsScalars*, hipStream_t);                    \
  template hipError_t launch_transpose_xy<T>(int, int, int, const T*, T*, hipStream_t);          \
  template hipError_t launch_pad_copies<T>(int, int, int, const T*, T*, T*, hipStream_t);         \
  template hipError_t launch_copy<T>(size_t, const T*, T*, hipStream_t);                        \
  template hipError_t launch_fill<T>(size_t, float, T*, hipStream_t);                           \
  template hipError_t launch_nonfinite<T>(size_t, const T*, int*, hipStream_t);                 \
  template hipError_t launch_restrict<T>(int, int, int, const T*, T*, hipStream_t);             \
  template hipError_t launch_prolong<T>(const tfcb_geometry&, const tfcb_geometry&, const T*,    \
                                        T*, hipStream_t);
TFCB_INST(float)
TFCB_INST(__half)
TFCB_INST(__hip_bfloat16)
#undef TFCB_INST
template hipError_t launch_cast<float, float>(size_t, const float*, float*, hipStream_t);
template hipError_t launch_cast<float, __half>(size_t, const float*, __half*, hipStream_t);
template hipError_t launch_cast<__half, float>(size_t, const __half*, float*, hipStream_t);
template hipError_t launch_cast<float, __hip_bfloat16>(size_t, const float*, __hip_bfloat16*,
                                                       hipStream_t);
template hipError_t launch_cast<__hip_bfloat16, float>(size_t, const __hip_bfloat16*, float*,
                                                       hipStream_t);

}  // namespace tfcb
