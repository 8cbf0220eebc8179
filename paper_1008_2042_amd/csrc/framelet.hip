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
// there.  So running analysis + shrink on a halo of d voxels around the tile
// (from reflected input) and then correlating with the filters gives exactly
// the adjoint W^T of the reflected convolution, with no special edge code.
//
// Mapping: a block owns an HX x HY tile of (x, y) positions (one thread
// each) = the output tile plus a halo of d, and marches along z over a chunk
// of output slices.  Per step za it
//   1. stages input slice za + d (tile + 2d halo, reflected indices) into an
//      LDS ring of 2d+1 slices;
//   2. computes the 27 coefficients at (x, y, za) separably from the ring,
//      shrinks the 26 high bands by max(1 - lambda/||alpha_h||, 0);
//   3. folds them along z into 9 partial sums c_lm for output slices
//      za - d, za, za + d (an LDS ring of accumulators, one per position);
//   4. when slice za - d is complete, correlates its 9 partial sums in x and y
//      for the interior positions and writes the voxel, with H and the
//      momentum epilogue.
#include "tfcb_internal.h"

namespace tfcb {

namespace {

constexpr float kH1 = 0.35355339059327373f;  // sqrt(2) / 4

__device__ __forceinline__ int reflect_idx(int j, int n) {
  while (j < 0 || j >= n) j = (j < 0) ? -1 - j : 2 * n - 1 - j;
  return j;
}

// Convolution of a triple (f[n-d], f[n], f[n+d]) with h0, h1, h2.
// (A_l f)[n] = sum_m h_l[m] f[n - m d], h listed as h[-1], h[0], h[+1].
__device__ __forceinline__ void conv3(float fm, float f0, float fp, float& o0, float& o1,
                                      float& o2) {
  const float s = fp + fm;
  o0 = fmaf(0.25f, s, 0.5f * f0);
  o1 = kH1 * (fp - fm);
  o2 = fmaf(-0.25f, s, 0.5f * f0);
}

// Correlation sum_m h_l[m] c[n + m d] for one filter l, values at n-d, n, n+d.
__device__ __forceinline__ float corr3(int l, float cm, float c0, float cp) {
  if (l == 0) return fmaf(0.25f, cm + cp, 0.5f * c0);
  if (l == 1) return kH1 * (cm - cp);
  return fmaf(-0.25f, cm + cp, 0.5f * c0);
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
  constexpr int M = 2 * D + 1;          // ring depth
  constexpr int FX = HX + 2 * D, FY = HY + 2 * D;
  constexpr int NT = HX * HY;
  __shared__ float fring[M][FY][FX];
  __shared__ float cacc[M][9][HY][HX];

  const int tx = threadIdx.x % HX, ty = threadIdx.x / HX;
  const int ox = blockIdx.x * (HX - 2 * D);  // first output x of the tile
  const int oy = blockIdx.y * (HY - 2 * D);
  const int z_begin = blockIdx.z * zchunk;
  const int z_end = min(nz, z_begin + zchunk);
  // this thread's position (may be a halo position outside the grid)
  const int px = ox + tx - D, py = oy + ty - D;

  auto stage = [&](int zs) {
    const int slot = ((zs % M) + M) % M;
    const int zr = reflect_idx(zs, nz);
    for (int e = threadIdx.x; e < FX * FY; e += NT) {
      const int fx = e % FX, fy = e / FX;
      const int gx = reflect_idx(ox - 2 * D + fx, nx);
      const int gy = reflect_idx(oy - 2 * D + fy, ny);
      fring[slot][fy][fx] = ld(in + ((size_t)zr * ny + gy) * nx + gx);
    }
  };
  for (int s = 0; s < M; ++s)
    for (int q = 0; q < 9; ++q) cacc[s][q][ty][tx] = 0.f;
  for (int zs = z_begin - 2 * D; zs < z_begin; ++zs) stage(zs);

  for (int za = z_begin - D; za < z_end + D; ++za) {
    stage(za + D);
    __syncthreads();
    // ---- analysis at (px, py, za): b_lm on the three slices za - d, za, za + d
    float b[3][9];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int zs = za + (sl - 1) * D;  // sl = 0: za - d (f[n - d]), 2: za + d
      const int slot = ((zs % M) + M) % M;
      float a[3][3];  // a[row][l]: x-filtered rows y - d, y, y + d
#pragma unroll
      for (int ry = 0; ry < 3; ++ry) {
        const int fy = ty + D + (ry - 1) * D;
        const float fm = fring[slot][fy][tx], f0 = fring[slot][fy][tx + D],
                    fp = fring[slot][fy][tx + 2 * D];
        conv3(fm, f0, fp, a[ry][0], a[ry][1], a[ry][2]);
      }
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        float o0, o1, o2;
        conv3(a[0][l], a[1][l], a[2][l], o0, o1, o2);
        b[sl][0 * 3 + l] = o0;  // index 3m + l
        b[sl][1 * 3 + l] = o1;
        b[sl][2 * 3 + l] = o2;
      }
    }
    float alpha[27];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      float o0, o1, o2;
      conv3(b[0][q], b[1][q], b[2][q], o0, o1, o2);
      alpha[q] = o0;       // n = 0
      alpha[9 + q] = o1;   // n = 1
      alpha[18 + q] = o2;  // n = 2
    }
    // ---- shrink (Eq. (2))
    float n2 = 0.f;
#pragma unroll
    for (int q = 1; q < 27; ++q) n2 = fmaf(alpha[q], alpha[q], n2);
    const float nrm = sqrtf(n2);
    const float sh = nrm <= lambda ? 0.f : 1.f - lambda / nrm;
#pragma unroll
    for (int q = 1; q < 27; ++q) alpha[q] *= sh;
    if (HAS_LOW) {
      const int gx = reflect_idx(px, nx), gy = reflect_idx(py, ny), gz = reflect_idx(za, nz);
      alpha[0] = ld(low + ((size_t)gz * ny + gy) * nx + gx);
    }
    // ---- fold along z into the accumulators of output slices za+d, za, za-d
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float a0 = alpha[q], a1 = alpha[9 + q], a2 = alpha[18 + q];
      const float up = fmaf(0.25f, a0 - a2, kH1 * a1);    // to zo = za + d (tap m = -1)
      const float mid = 0.5f * (a0 + a2);                 // to zo = za
      const float dn = fmaf(0.25f, a0 - a2, -kH1 * a1);   // to zo = za - d (tap m = +1)
      const int zu = za + D, zd = za - D;
      if (zu >= z_begin && zu < z_end) cacc[zu % M][q][ty][tx] += up;
      if (za >= z_begin && za < z_end) cacc[za % M][q][ty][tx] += mid;
      if (zd >= z_begin && zd < z_end) cacc[zd % M][q][ty][tx] += dn;
    }
    __syncthreads();
    // ---- output slice zo = za - d is complete
    const int zo = za - D;
    if (zo >= z_begin && zo < z_end) {
      const int slot = zo % M;
      const bool interior = tx >= D && tx < HX - D && ty >= D && ty < HY - D;
      if (interior && px < nx && py < ny) {
        float v = 0.f;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          float col[3];  // y-correlated sums at x - d, x, x + d
#pragma unroll
          for (int cx = 0; cx < 3; ++cx) {
            const int xx = tx + (cx - 1) * D;
            float s = 0.f;
#pragma unroll
            for (int m = 0; m < 3; ++m)
              s += corr3(m, cacc[slot][3 * m + l][ty - D][xx], cacc[slot][3 * m + l][ty][xx],
                         cacc[slot][3 * m + l][ty + D][xx]);
            col[cx] = s;
          }
          v += corr3(l, col[0], col[1], col[2]);
        }
        // H: negative voxels to zero; a NaN stays NaN (fmaxf would map it to 0
        // and hide a failed reconstruction from the non-finite check)
        if (positivity) v = v < 0.f ? 0.f : v;
        const size_t o = ((size_t)zo * ny + py) * nx + px;
        st(out + o, v);
        if (MOM) {
          const float fn = ld(out + o);
          st(vnext + o, fmaf(mom, fn - ld(fcur + o), fn));
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 9; ++q) cacc[slot][q][ty][tx] = 0.f;
    }
  }
}

template <typename T, int D, int HX, int HY>
static hipError_t launch_fw(int nx, int ny, int nz, float lambda, int positivity, const T* in,
                            const T* low, T* out, const T* fcur, T* vnext, float mom,
                            hipStream_t s) {
  const int tox = HX - 2 * D, toy = HY - 2 * D;
  const int gx = (nx + tox - 1) / tox, gy = (ny + toy - 1) / toy;
  // split z so the launch has enough blocks to fill the chip
  int chunks = 1;
  while ((long)gx * gy * chunks < 1024 && nz / (chunks * 2) >= 8 * D) chunks *= 2;
  const int zchunk = (nz + chunks - 1) / chunks;
  dim3 grid(gx, gy, (nz + zchunk - 1) / zchunk);
  dim3 block(HX * HY);
  if (low) {
    if (vnext)
      hipLaunchKernelGGL((k_framelet<T, D, HX, HY, true, true>), grid, block, 0, s, nx, ny, nz,
                         zchunk, lambda, positivity, in, low, out, fcur, vnext, mom);
    else
      hipLaunchKernelGGL((k_framelet<T, D, HX, HY, true, false>), grid, block, 0, s, nx, ny, nz,
                         zchunk, lambda, positivity, in, low, out, fcur, vnext, mom);
  } else {
    if (vnext)
      hipLaunchKernelGGL((k_framelet<T, D, HX, HY, false, true>), grid, block, 0, s, nx, ny, nz,
                         zchunk, lambda, positivity, in, low, out, fcur, vnext, mom);
    else
      hipLaunchKernelGGL((k_framelet<T, D, HX, HY, false, false>), grid, block, 0, s, nx, ny, nz,
                         zchunk, lambda, positivity, in, low, out, fcur, vnext, mom);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_framelet(int nx, int ny, int nz, int dil, float lambda, int positivity,
                           const T* in, const T* low, T* out, const T* fcur, T* vnext, float mom,
                           hipStream_t s) {
  if (dil == 1)
    return launch_fw<T, 1, 32, 16>(nx, ny, nz, lambda, positivity, in, low, out, fcur, vnext, mom,
                                   s);
  // dilation 2 keeps five slices in flight: a 32 x 8 tile keeps LDS at 55 KB
  return launch_fw<T, 2, 32, 8>(nx, ny, nz, lambda, positivity, in, low, out, fcur, vnext, mom,
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
