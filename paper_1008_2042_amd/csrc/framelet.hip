// Fused tight-frame regulariser: out = H(W^T T_lambda W in), then the next
// momentum point (section 2.1: the 27 tensor-product filters
// h_l(x) h_m(y) h_n(z) of h0 = [1,2,1]/4, h1 = sqrt(2)/4 [1,0,-1],
// h2 = [-1,2,-1]/4; the vector shrinkage of Eq. (2); positivity H;
// Algorithm A2 steps 3-4 and step 1 of the next iteration).  The 27 bands
// never reach HBM.
//
// Boundary: W convolves the half-sample symmetric extension of the volume.
// The coefficients computed from that extension at a position just outside
// the grid equal (+-) the coefficients at the mirrored inside position, with
// the sign of the band's filter symmetry, and the shrink factor is the same
// there.  So evaluating analysis + shrink on a halo of d voxels around the
// tile (from reflected input) and synthesising from those positions gives
// exactly the adjoint W^T of the reflected convolution, with no special edge
// code.
//
// Evaluation.  The filter bank's 3 x 3 matrix H[l][m] = h_l[m] has
// orthogonal columns: sum_l h_l[m] h_l[k] = c_m [m == k] with c = (1/4, 1/2,
// 1/4), which is h0 itself.  Two exact consequences follow for the
// tensor-product bank, with K the separable [1,2,1]/4 smoothing (taps -d, 0,
// +d on every axis) and s(p) the shrink factor at coefficient position p:
//   * sum over all 27 bands of W_b^T (s W_b f) = f K(s), so that
//     W^T T W f = f K(s) + K(L - s alpha_0), where alpha_0 = K f is the low
//     band and L the value T keeps for it (alpha_0 itself, or the coarser
//     level's result with two levels);
//   * sum over all 27 bands of (W_b f)(p)^2 = K(f^2)(p).
// The kernel evaluates these forms, with the high-band energy of a position
// written as sums of squares (no cancellation): per slice, the xy energy of
// the 8 bands other than the xy low band is the weighted variance
// E = sum_k w_k (f_k - b0)^2 over the 3 x 3 neighbourhood (w = [1,2,1]/4 in
// x times in y, b0 = the xy low band), and
//   ||alpha_high||^2 = (E(z - d) + 2 E(z) + E(z + d)) / 4 + a01^2 + a02^2
// with a01, a02 the two z-high bands of b0.  The result equals the
// 27-band analysis, shrink and synthesis up to rounding.
//
// Mapping: a block owns an HX x HY tile of (x, y) positions (one thread
// each) = the output tile plus a halo of d, and marches along z over a chunk
// of output slices, one chain per residue of z modulo d (with dilation d the
// slices a coefficient or an output reads are d apart, so the residue
// classes never mix).  Per step of a chain (staged slice zs) a thread
//   1. reads the 3 x 3 neighbourhood of its position in slice zs from LDS and
//      forms b0 and E there;
//   2. from b0 and E of slices za - d, za, za + d (za = zs - d, held in
//      registers) forms the shrink factor s and R = L - s alpha_0 at za;
//   3. smooths s and R in z over za - 2d, za - d, za and writes the two sums
//      for slice zo = za - d to LDS, and stages the next slice;
//   4. after the step's one barrier, smooths the two in x and y and writes
//      f K(s) + K(R) at (x, y, zo), with H and the momentum epilogue.
// The staged slices and the smoothed pairs are double-buffered in LDS, so a
// step needs one barrier.
#include "tfcb_internal.h"

namespace tfcb {

namespace {

constexpr float kH1 = 0.35355339059327373f;  // sqrt(2) / 4

__device__ __forceinline__ int reflect_idx(int j, int n) {
  while (j < 0 || j >= n) j = (j < 0) ? -1 - j : 2 * n - 1 - j;
  return j;
}

}  // namespace

template <typename T, int D, int HX, int HY, bool HAS_LOW, bool MOM>
__global__ __launch_bounds__(HX* HY) void k_framelet(int nx, int ny, int nz, int zchunk,
                                                      float lambda, int positivity,
                                                      const T* __restrict__ in,
                                                      const T* __restrict__ low,
                                                      T* __restrict__ out,
                                                      const T* __restrict__ fcur,
                                                      T* __restrict__ vnext, float mom) {
  constexpr int FX = HX + 2 * D, FY = HY + 2 * D;
  constexpr int NT = HX * HY;
  constexpr int NS = (FX * FY + NT - 1) / NT;  // staged elements per thread
  __shared__ float sbuf[2][FY][FX];
  __shared__ float kbuf[2][2][HY][HX];  // z-smoothed s and R, per step parity

  const int tx = threadIdx.x % HX, ty = threadIdx.x / HX;
  const int ox = blockIdx.x * (HX - 2 * D);  // first output x of the tile
  const int oy = blockIdx.y * (HY - 2 * D);
  const int z_begin = blockIdx.z * zchunk;
  const int z_end = min(nz, z_begin + zchunk);
  // this thread's position (may be a halo position outside the grid)
  const int px = ox + tx - D, py = oy + ty - D;
  const bool writer = tx >= D && tx < HX - D && ty >= D && ty < HY - D && px < nx && py < ny;
  const size_t plane = (size_t)nx * ny;
  const float lam2 = lambda * lambda;

  // staged elements of this thread: in-plane offsets (reflected) and LDS slots
  int soff[NS], sslot[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int e = threadIdx.x + k * NT;
    const int fx = e % FX, fy = e / FX;
    sslot[k] = e < FX * FY ? e : -1;
    const int gx = reflect_idx(ox - 2 * D + fx, nx);
    const int gy = reflect_idx(oy - 2 * D + min(fy, FY - 1), ny);
    soff[k] = gy * nx + gx;
  }
  const int lowoff = reflect_idx(px, nx) + nx * reflect_idx(py, ny);
  float* const sflat0 = &sbuf[0][0][0];
  float* const sflat1 = &sbuf[1][0][0];

  for (int cls = 0; cls < D; ++cls) {
    const int z0 = z_begin + cls;
    if (z0 >= z_end) break;
    const int z1 = z0 + ((z_end - 1 - z0) / D) * D;  // last output slice of the chain
    // staged slices zs_i = z0 - 2d + i d, i = 0 .. last
    const int last = (z1 - z0) / D + 4;
    float nxt[NS];
    auto load_slice = [&](int i) {
      const size_t zoff = (size_t)reflect_idx(z0 - 2 * D + i * D, nz) * plane;
#pragma unroll
      for (int k = 0; k < NS; ++k) nxt[k] = sslot[k] >= 0 ? ld(in + zoff + soff[k]) : 0.f;
    };
    auto store_slice = [&](int i) {
      float* const dst = (i & 1) ? sflat1 : sflat0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (sslot[k] >= 0) dst[sslot[k]] = nxt[k];
    };
    load_slice(0);
    store_slice(0);
    load_slice(1);
    __syncthreads();
    // rolling values, oldest first: b0 and E of slices zs - 2d, zs - d, zs;
    // f at this position for zs - 2d, zs - d, zs; s and R of za - 2d, za - d, za
    float b0o = 0.f, b0m = 0.f, b0n = 0.f, eo = 0.f, em = 0.f, en = 0.f;
    float fco = 0.f, fcm = 0.f, fcn = 0.f;
    float sho = 0.f, shm = 0.f, shn = 0.f, ro = 0.f, rm = 0.f, rn = 0.f;
    for (int i = 0; i <= last; ++i) {
      const int zs = z0 - 2 * D + i * D;
      const int za = zs - D, zo = za - D;
      float lowv = 0.f;
      if (HAS_LOW && i >= 2) lowv = ld(low + (size_t)reflect_idx(za, nz) * plane + lowoff);
      // ---- 1. xy low band and xy high-band energy of slice zs
      {
        const float (&sl)[FY][FX] = sbuf[i & 1];
        float f[3][3];
#pragma unroll
        for (int ry = 0; ry < 3; ++ry)
#pragma unroll
          for (int rx = 0; rx < 3; ++rx) f[ry][rx] = sl[ty + ry * D][tx + rx * D];
        float r[3];
#pragma unroll
        for (int ry = 0; ry < 3; ++ry) r[ry] = fmaf(0.25f, f[ry][0] + f[ry][2], 0.5f * f[ry][1]);
        const float b0 = fmaf(0.25f, r[0] + r[2], 0.5f * r[1]);
        float dv[3][3];
#pragma unroll
        for (int ry = 0; ry < 3; ++ry)
#pragma unroll
          for (int rx = 0; rx < 3; ++rx) dv[ry][rx] = f[ry][rx] - b0;
        const float corner = fmaf(dv[0][0], dv[0][0], fmaf(dv[0][2], dv[0][2],
                             fmaf(dv[2][0], dv[2][0], dv[2][2] * dv[2][2])));
        const float edge = fmaf(dv[0][1], dv[0][1], fmaf(dv[1][0], dv[1][0],
                           fmaf(dv[1][2], dv[1][2], dv[2][1] * dv[2][1])));
        const float e = fmaf(0.0625f, corner, fmaf(0.125f, edge, 0.25f * (dv[1][1] * dv[1][1])));
        b0o = b0m; b0m = b0n; b0n = b0;
        eo = em; em = en; en = e;
        fco = fcm; fcm = fcn; fcn = f[1][1];
      }
      // ---- 2. shrink factor and low-band remainder at za
      if (i >= 2) {
        const float a00 = fmaf(0.25f, b0o + b0n, 0.5f * b0m);
        const float a01 = kH1 * (b0n - b0o);
        const float a02 = fmaf(-0.25f, b0o + b0n, 0.5f * b0m);
        const float n2 = fmaf(0.25f, eo + en, fmaf(0.5f, em, fmaf(a01, a01, a02 * a02)));
        // s = max(1 - lambda / ||alpha_h||, 0), with the hardware reciprocal
        // square root (1 ulp); the clamp keeps it finite for lambda = 0
        const float sh = n2 <= lam2 ? 0.f
                                    : 1.f - lambda * __builtin_amdgcn_rsqf(fmaxf(n2, 1e-30f));
        const float L = HAS_LOW ? lowv : a00;
        sho = shm; shm = shn; shn = sh;
        ro = rm; rm = rn; rn = fmaf(-sh, a00, L);
      }
      // ---- 3. z sums for slice zo, and the next slice into the other buffer
      const bool emit = i >= 4;
      if (emit) {
        kbuf[i & 1][0][ty][tx] = fmaf(0.25f, sho + shn, 0.5f * shm);
        kbuf[i & 1][1][ty][tx] = fmaf(0.25f, ro + rn, 0.5f * rm);
      }
      if (i < last) {
        store_slice(i + 1);
        if (i + 2 <= last) load_slice(i + 2);
      }
      __syncthreads();
      // ---- 4. xy sums and the output voxel
      if (emit && writer) {
        float ks[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          float r[3];
#pragma unroll
          for (int ry = 0; ry < 3; ++ry) {
            const float* row = &kbuf[i & 1][w][ty + (ry - 1) * D][tx];
            r[ry] = fmaf(0.25f, row[-D] + row[D], 0.5f * row[0]);
          }
          ks[w] = fmaf(0.25f, r[0] + r[2], 0.5f * r[1]);
        }
        float v = fmaf(fco, ks[0], ks[1]);
        // H: negative voxels to zero; a NaN stays NaN (fmaxf would map it to
        // 0 and hide a failed reconstruction from the non-finite check)
        if (positivity) v = v < 0.f ? 0.f : v;
        const size_t o = (size_t)zo * plane + (size_t)py * nx + px;
        st(out + o, v);
        if (MOM) {
          const float fn = as_stored<T>(v);
          st(vnext + o, fmaf(mom, fn - ld(fcur + o), fn));
        }
      }
    }
    __syncthreads();  // the next chain restages both buffers
  }
}

// Blocks resident per CU for a kernel, and the CU count, cached per kernel.
template <typename K>
static int resident_slots(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return 1024;
  return max(1, cus * per_cu);
}

template <typename T, int D, int HX, int HY, bool HAS_LOW, bool MOM>
static hipError_t launch_fw1(int nx, int ny, int nz, float lambda, int positivity, const T* in,
                             const T* low, T* out, const T* fcur, T* vnext, float mom,
                             hipStream_t s) {
  auto kern = k_framelet<T, D, HX, HY, HAS_LOW, MOM>;
  static const int slots = resident_slots(kern, HX * HY);
  const int tox = HX - 2 * D, toy = HY - 2 * D;
  const long gx = (nx + tox - 1) / tox, gy = (ny + toy - 1) / toy;
  // Split z into chunks: a chunk costs its slices plus 4 d steps of halo, and
  // the launch takes ceil(blocks / resident slots) rounds; pick the split
  // with the least rounds x steps (the fewest chunks on a tie).
  int zchunk = nz;
  long best = -1;
  for (int chunks = 1; chunks <= nz; ++chunks) {
    const int zc = (nz + chunks - 1) / chunks;
    if (chunks > 1 && zc < 4 * D) break;
    const long nb = gx * gy * ((nz + zc - 1) / zc);
    const long cost = ((nb + slots - 1) / slots) * (long)(zc + 4 * D);
    if (best < 0 || cost < best) {
      best = cost;
      zchunk = zc;
    }
  }
  dim3 grid((unsigned)gx, (unsigned)gy, (nz + zchunk - 1) / zchunk);
  hipLaunchKernelGGL(kern, grid, dim3(HX * HY), 0, s, nx, ny, nz, zchunk, lambda, positivity, in,
                     low, out, fcur, vnext, mom);
  return hipGetLastError();
}

template <typename T, int D, int HX, int HY>
static hipError_t launch_fw(int nx, int ny, int nz, float lambda, int positivity, const T* in,
                            const T* low, T* out, const T* fcur, T* vnext, float mom,
                            hipStream_t s) {
  if (low) {
    if (vnext)
      return launch_fw1<T, D, HX, HY, true, true>(nx, ny, nz, lambda, positivity, in, low, out,
                                                  fcur, vnext, mom, s);
    return launch_fw1<T, D, HX, HY, true, false>(nx, ny, nz, lambda, positivity, in, low, out,
                                                 fcur, vnext, mom, s);
  }
  if (vnext)
    return launch_fw1<T, D, HX, HY, false, true>(nx, ny, nz, lambda, positivity, in, low, out,
                                                 fcur, vnext, mom, s);
  return launch_fw1<T, D, HX, HY, false, false>(nx, ny, nz, lambda, positivity, in, low, out,
                                                fcur, vnext, mom, s);
}

template <typename T>
hipError_t launch_framelet(int nx, int ny, int nz, int dil, float lambda, int positivity,
                           const T* in, const T* low, T* out, const T* fcur, T* vnext, float mom,
                           hipStream_t s) {
  if (dil == 1)
    return launch_fw<T, 1, 32, 16>(nx, ny, nz, lambda, positivity, in, low, out, fcur, vnext, mom,
                                   s);
  return launch_fw<T, 2, 32, 16>(nx, ny, nz, lambda, positivity, in, low, out, fcur, vnext, mom,
                                 s);
}

// low = A0^3 in: the level-1 low band (h0 in x, y, z; reflected edges).
template <typename T>
__global__ __launch_bounds__(256) void k_lowpass(int nx, int ny, int nz, const T* __restrict__ in,
                                                 T* __restrict__ low) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= nx || j >= ny) return;
  const float w[3] = {0.25f, 0.5f, 0.25f};
  float acc = 0.f;
  for (int c = -1; c <= 1; ++c) {
    const int zz = reflect_idx(k - c, nz);
    float sy = 0.f;
    for (int b = -1; b <= 1; ++b) {
      const int yy = reflect_idx(j - b, ny);
      const T* row = in + ((size_t)zz * ny + yy) * nx;
      float sx = 0.f;
      for (int a = -1; a <= 1; ++a) sx = fmaf(w[a + 1], ld(row + reflect_idx(i - a, nx)), sx);
      sy = fmaf(w[b + 1], sx, sy);
    }
    acc = fmaf(w[c + 1], sy, acc);
  }
  st(low + ((size_t)k * ny + j) * nx + i, acc);
}

template <typename T>
hipError_t launch_lowpass(int nx, int ny, int nz, const T* in, T* low, hipStream_t s) {
  dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz);
  hipLaunchKernelGGL((k_lowpass<T>), grid, dim3(256), 0, s, nx, ny, nz, in, low);
  return hipGetLastError();
}

#define TFCB_INST(T)                                                                          \
  template hipError_t launch_framelet<T>(int, int, int, int, float, int, const T*, const T*,   \
                                         T*, const T*, T*, float, hipStream_t);               \
  template hipError_t launch_lowpass<T>(int, int, int, const T*, T*, hipStream_t);
TFCB_INST(float)
TFCB_INST(__half)
TFCB_INST(__hip_bfloat16)
#undef TFCB_INST

}  // namespace tfcb
