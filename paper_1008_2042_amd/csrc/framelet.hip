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
// of output slices, one chain per residue of z modulo d (with dilation d the
// three slices a coefficient or an output reads are d apart, so the residue
// classes never mix).  Per step of a chain (slice zs = za + d) a thread
//   1. filters the staged slice zs in x and y at its position (9 LDS reads),
//      giving the 9 xy bands b_lm of that slice;
//   2. filters in z the b of slices za - d, za, za + d held in registers,
//      giving the 27 coefficients at (x, y, za), and shrinks the 26 high bands
//      by max(1 - lambda/||alpha_h||, 0);
//   3. folds them along z into register accumulators c_lm of output slices
//      za - d, za, za + d, after which slice za - d is complete;
//   4. writes the next slice (loaded into registers at the start of the step)
//      to the other LDS buffer, and, when za - d is an output slice,
//      correlates its c_lm in y (27 LDS reads) and then in x (9 reads) for the
//      interior positions and writes the voxel, with H and the momentum
//      epilogue.
// b and c rotate through three register sets (the loop is unrolled three
// times), so nothing moves between registers; a step costs two barriers.
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

// The xy bands of one staged slice at (tx, ty): x filter of rows y - d, y,
// y + d, then y filter; b[3m + l] = h_m (y) h_l (x).
template <int D, int FX, int FY>
__device__ __forceinline__ void xy_bands(const float (&sl)[FY][FX], int tx, int ty, float (&b)[9]) {
  float a[3][3];  // a[row][l]: x-filtered rows y - d, y, y + d
#pragma unroll
  for (int ry = 0; ry < 3; ++ry) {
    const int fy = ty + D + (ry - 1) * D;
    conv3(sl[fy][tx], sl[fy][tx + D], sl[fy][tx + 2 * D], a[ry][0], a[ry][1], a[ry][2]);
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) conv3(a[0][l], a[1][l], a[2][l], b[l], b[3 + l], b[6 + l]);
}

template <typename T, int D, int HX, int HY, bool HAS_LOW, bool MOM>
__global__ __launch_bounds__(HX* HY, HAS_LOW ? 3 : 4) void k_framelet(int nx, int ny, int nz, int zchunk,
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
  __shared__ float cbuf[9][HY][HX];
  __shared__ float colbuf[3][HY][HX];

  const int tx = threadIdx.x % HX, ty = threadIdx.x / HX;
  const int ox = blockIdx.x * (HX - 2 * D);  // first output x of the tile
  const int oy = blockIdx.y * (HY - 2 * D);
  const int z_begin = blockIdx.z * zchunk;
  const int z_end = min(nz, z_begin + zchunk);
  // this thread's position (may be a halo position outside the grid)
  const int px = ox + tx - D, py = oy + ty - D;
  const bool interior = tx >= D && tx < HX - D && ty >= D && ty < HY - D;
  const bool ycorr = ty >= D && ty < HY - D;
  const bool writer = interior && px < nx && py < ny;
  const size_t plane = (size_t)nx * ny;

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
    // slices zs_i = z0 - 2d + i d, i = 0 .. last
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
    float b0[9], b1[9], b2[9], c0[9], c1[9], c2[9];
    // prologue: slices 0 and 1 give the xy bands of za - d and za for the
    // first coefficient slice za = z0 - d
    load_slice(0);
    store_slice(0);
    load_slice(1);
    __syncthreads();
    xy_bands<D>(sbuf[0], tx, ty, b0);
    store_slice(1);
    load_slice(2);
    __syncthreads();
    xy_bands<D>(sbuf[1], tx, ty, b1);
    store_slice(2);
    if (last >= 3) load_slice(3);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 9; ++q) c0[q] = c1[q] = 0.f;

    // Step i (2 <= i <= last): slice i is staged in buffer i & 1 and slice
    // i + 1 is in registers.  bo, bm = xy bands of za - d, za (za = zs_i - d);
    // bn receives those of za + d.  cx, cy, cz = accumulators of za - d, za,
    // za + d (cz is set here: za + d has no earlier contribution).  Returns
    // true after the last step.
    auto step = [&](int i, float (&bo)[9], float (&bm)[9], float (&bn)[9], float (&cx)[9],
                    float (&cy)[9], float (&cz)[9]) -> bool {
      const int za = z0 - D + (i - 2) * D;
      xy_bands<D>(sbuf[i & 1], tx, ty, bn);
      float low0 = 0.f;
      if (HAS_LOW) low0 = ld(low + (size_t)reflect_idx(za, nz) * plane + lowoff);
      // ---- analysis in z: alpha[9n + q] = h_n (z) b_q
      float alpha[27];
#pragma unroll
      for (int q = 0; q < 9; ++q) conv3(bo[q], bm[q], bn[q], alpha[q], alpha[9 + q], alpha[18 + q]);
      // ---- shrink (Eq. (2))
      float n2 = 0.f;
#pragma unroll
      for (int q = 1; q < 27; ++q) n2 = fmaf(alpha[q], alpha[q], n2);
      const float nrm = sqrtf(n2);
      const float sh = nrm <= lambda ? 0.f : 1.f - lambda / nrm;
#pragma unroll
      for (int q = 1; q < 27; ++q) alpha[q] *= sh;
      if (HAS_LOW) alpha[0] = low0;
      // ---- fold along z into the accumulators of za + d, za, za - d
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const float a0 = alpha[q], a1 = alpha[9 + q], a2 = alpha[18 + q];
        cz[q] = fmaf(0.25f, a0 - a2, kH1 * a1);        // tap m = -1
        cy[q] += 0.5f * (a0 + a2);                      // tap m = 0
        cx[q] += fmaf(0.25f, a0 - a2, -kH1 * a1);       // tap m = +1
      }
      // ---- stage the next slice, and publish it and (below) slice za - d
      const int zo = za - D;
      const bool emit = i >= 4;
      if (emit) {
#pragma unroll
        for (int q = 0; q < 9; ++q) cbuf[q][ty][tx] = cx[q];
      }
      if (i < last) {
        store_slice(i + 1);
        if (i + 2 <= last) load_slice(i + 2);
      }
      __syncthreads();
      if (emit) {
        // y correlation of the 9 partial sums, for the rows the x
        // correlation reads
        if (ycorr) {
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            float sy = 0.f;
#pragma unroll
            for (int m = 0; m < 3; ++m)
              sy += corr3(m, cbuf[3 * m + l][ty - D][tx], cbuf[3 * m + l][ty][tx],
                          cbuf[3 * m + l][ty + D][tx]);
            colbuf[l][ty][tx] = sy;
          }
        }
        __syncthreads();
        if (writer) {
          float v = 0.f;
#pragma unroll
          for (int l = 0; l < 3; ++l)
            v += corr3(l, colbuf[l][ty][tx - D], colbuf[l][ty][tx], colbuf[l][ty][tx + D]);
          // H: negative voxels to zero; a NaN stays NaN (fmaxf would map it to
          // 0 and hide a failed reconstruction from the non-finite check)
          if (positivity) v = v < 0.f ? 0.f : v;
          const size_t o = (size_t)zo * plane + (size_t)py * nx + px;
          st(out + o, v);
          if (MOM) {
            const float fn = ld(out + o);
            st(vnext + o, fmaf(mom, fn - ld(fcur + o), fn));
          }
        }
      }
      return i >= last;
    };
    // the accumulator of za - d is complete after its step; its registers
    // become the accumulator of za + 2d, which the next step sets
    for (int i = 2;; i += 3) {
      if (step(i, b0, b1, b2, c0, c1, c2)) break;
      if (step(i + 1, b1, b2, b0, c1, c2, c0)) break;
      if (step(i + 2, b2, b0, b1, c2, c0, c1)) break;
    }
    __syncthreads();  // the next chain restages both buffers
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
