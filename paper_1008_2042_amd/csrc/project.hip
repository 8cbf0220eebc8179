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
#include <type_traits>

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
// floor(x) as an int in one conversion (v_cvt_flr_i32_f32), |x| < 2^31
__device__ __forceinline__ int floor_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
// x clamped to [LO, hi] in one instruction (LO a small constant, hi uniform)
template <int LO>
__device__ __forceinline__ int clamp_int(int x, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "n"(LO), "s"(hi));
  return r;
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

// Levels that rows j..RPT-1 can still use, counted from row j's lower
// level: the host's row plan keeps the rows' z span within
// (RPT - 1) rs + 0.05 <= NL - 2 slices, so rows j..RPT-1 span at most
// (RPT - 1 - j) (NL - 2.05) / (RPT - 1) slices, and floor(zh_k) -
// floor(zh_j) is at most the ceiling of that.
template <int RPT, int NL>
__host__ __device__ constexpr int levels_needed(int j) {
  return RPT == 1 ? 2
                  : 2 + ((RPT - 1 - j) * (100 * NL - 205) + 100 * (RPT - 1) - 1) /
                            (100 * (RPT - 1));
}

// Row j's bilinear sample from the trans-interpolated levels: the two levels
// around its z index, d_j = floor(zh_j) - floor(zh_0) and d_j + 1, weighted
// by the fraction fr_j = zh_j - floor(zh_j).  The rows' z indices rise with j
// by more than 0 and less than one slice per row, so d_j is d_{j-1} or
// d_{j-1} + 1, and it is d_{j-1} + 1 exactly where the fraction wraps,
// fr_j < fr_{j-1}: the pair is carried along as a shift register of the
// levels, which moves on there.  At row j only the levels_needed(j) entries
// that later rows can reach move.
template <int RPT, int NL>
__device__ __forceinline__ void rows_from_levels(const float (&lev)[NL], const float (&fr)[RPT],
                                                 float (&acc)[RPT]) {
  float win[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) win[l] = lev[l];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    if (j > 0 && fr[j] < fr[j - 1]) {
#pragma unroll
      for (int l = 0; l + 1 < NL; ++l)
        if (l < levels_needed<RPT, NL>(j)) win[l] = win[l + 1];
    }
    acc[j] += fmaf(fr[j], win[1] - win[0], win[0]);
  }
}
static_assert(levels_needed<16, 6>(0) == 6 && levels_needed<16, 6>(15) == 2 &&
                  levels_needed<8, 7>(0) == 7 && levels_needed<4, 4>(3) == 2,
              "level window");

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
  float fr[RPT];  // z fractions, v_fract (the hardware's x - floor(x))
#pragma unroll
  for (int j = 0; j < RPT; ++j) fr[j] = __builtin_amdgcn_fractf(z_index(ci, p, vz[j], zc));
  const int iz0 = min(max((int)floorf(z_index(ci, p, vz[0], zc)), -kZPad), nz - 1);
  const T* __restrict__ q = vb + ((iz0 * ns + p) * ntp + it);
  float lev[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const float v0 = ld(q + l * zs), v1 = ld(q + l * zs + 1);
    lev[l] = fmaf(wt, v1 - v0, v0);
  }
  rows_from_levels<RPT, NL>(lev, fr, acc);
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
    const int ntp = pad_row(nt), zs = ns * ntp;
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
        const float rs = as_stored<T>(res);  // the stored (rounded) residual
        st(rl + o, ell * rs);
        part += (double)rs * (double)rs;
      } else {
        st(out + o, val);
        const float qs = as_stored<T>(val);
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

// ------------------------------------------------------------- staged P
// The same samples, with each plane's volume data staged in LDS per block.
// A block (64 columns x 4 RPT rows) walks the union of its threads' plane
// windows.  For every plane the box of levels and trans positions its
// threads can touch follows from the block's corner rays (the trans index is
// monotone in the column, the z index in the column and the row), widened by
// 0.01 for rounding: z levels from the lowest row's floor to the stack top of
// the last wave's first row, trans positions from the lower corner's floor
// down to a 4-element boundary up to the upper corner's floor + 1.  The box's
// level rows are loaded two planes ahead with aligned 4-element vector loads
// (each needed line once per block and plane) into registers, and stored
// into one of two LDS buffers while the threads sample the other one, so a
// plane costs one barrier.  A block whose box can exceed the buffers on any
// of its planes takes the direct path of k_project instead.
constexpr int kStageF4 = 32;    // 4-element vectors per staged level row
constexpr int kStageRows = 24;  // level rows per staged plane
constexpr int kStageRegs = (kStageRows * kStageF4 + 255) / 256;
constexpr int kStageBoxes = 512;  // planes whose boxes a block tabulates in LDS (8 KB; 4 KB packed)

// Four consecutive stored elements, loaded as they are stored (a float4, or
// 8 bytes of FP16/BF16) and widened to FP32 only when written to LDS, so
// that the loads of the next plane stay in flight while this plane is
// sampled.
template <typename T> struct Raw4 { using type = uint2; };
template <> struct Raw4<float> { using type = float4; };
template <typename T>
__device__ __forceinline__ typename Raw4<T>::type ld_raw4(const T* p) {
  return *reinterpret_cast<const typename Raw4<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ typename Raw4<T>::type raw4_zero() {
  return typename Raw4<T>::type{};
}
template <typename T> __device__ __forceinline__ float4 widen4(typename Raw4<T>::type u);
template <> __device__ __forceinline__ float4 widen4<float>(float4 u) { return u; }
template <> __device__ __forceinline__ float4 widen4<__half>(uint2 u) {
  __half_raw h0, h1, h2, h3;
  h0.x = (unsigned short)(u.x & 0xffffu);
  h1.x = (unsigned short)(u.x >> 16);
  h2.x = (unsigned short)(u.y & 0xffffu);
  h3.x = (unsigned short)(u.y >> 16);
  return make_float4(__half2float(__half(h0)), __half2float(__half(h1)),
                     __half2float(__half(h2)), __half2float(__half(h3)));
}
template <> __device__ __forceinline__ float4 widen4<__hip_bfloat16>(uint2 u) {
  // a bfloat16 is the upper half of the float with the same bits
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
}

struct StageBox {
  int zl, nzr;  // first level row and level-row count
  int tl4, nf4; // first trans element (a multiple of 4) and vector count
};

__device__ __forceinline__ StageBox stage_box(const ColInfo& cA, const ColInfo& cB, float vzA,
                                              float vzB, int p, float zc, int nt, int nz, int nl) {
  const float tA = trans_index(cA, p), tB = trans_index(cB, p);
  const int tlo = max((int)floorf(fminf(tA, tB) - 0.01f), -1);
  const int thi = min((int)floorf(fmaxf(tA, tB) + 0.01f) + 1, nt);
  const float z1 = z_index(cA, p, vzA, zc), z2 = z_index(cB, p, vzA, zc);
  const float z3 = z_index(cA, p, vzB, zc), z4 = z_index(cB, p, vzB, zc);
  StageBox b;
  b.zl = max((int)floorf(fminf(z1, z2) - 0.01f), -kZPad);
  const int ztop = min((int)floorf(fmaxf(z3, z4) + 0.01f), nz - 1) + nl - 1;
  b.nzr = max(ztop - b.zl + 1, 0);
  b.tl4 = tlo & ~3;
  b.nf4 = thi >= tlo ? ((thi - b.tl4) >> 2) + 1 : 0;
  return b;
}

// The samples of plane p for the RPT rows of one column, from the staged box
// `tile` (level row z - b.zl, element i - b.tl4, rows of 4 kStageF4).  Same
// arithmetic as sample_rows.
template <int RPT, int NL>
__device__ __forceinline__ void sample_rows_lds(const float* __restrict__ tile, const StageBox& b,
                                                const ColInfo& ci, int p, const float (&vz)[RPT],
                                                float zc, int nt, int nz, float (&acc)[RPT]) {
  const float th = trans_index(ci, p);
  const float tf = floorf(th);
  const int it = clamp_int<-1>((int)tf, nt - 1);
  const float wt = th - tf;
  float fr[RPT];  // z fractions, v_fract (the hardware's x - floor(x))
#pragma unroll
  for (int j = 0; j < RPT; ++j) fr[j] = __builtin_amdgcn_fractf(z_index(ci, p, vz[j], zc));
  const int iz0 = clamp_int<-kZPad>(floor_int(z_index(ci, p, vz[0], zc)), nz - 1);
  const float* __restrict__ q = tile + (iz0 - b.zl) * (4 * kStageF4) + (it - b.tl4);
  float lev[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const float v0 = q[l * 4 * kStageF4], v1 = q[l * 4 * kStageF4 + 1];
    lev[l] = fmaf(wt, v1 - v0, v0);
  }
  rows_from_levels<RPT, NL>(lev, fr, acc);
}

// XCD-aware order of the projector's blocks.  The chip dispatches the
// workgroups of a launch to its 8 XCDs in turn (workgroup n to XCD n mod 8),
// and each XCD has its own L2.  When the volume's padded copy is larger than
// the 256 MB Infinity Cache, every view's sweep of it comes from HBM, and the
// 1-D launch is remapped: XCD x takes the x-th contiguous chunk of a logical
// order in which groups of `group` adjacent views of the same 64-column x
// 4 RPT-row detector tile are consecutive, then the tiles of a row of the
// detector, then the rows.  The blocks resident on one XCD at a time then
// sweep nearly the same region of the volume at nearly the same planes
// (adjacent views of a dense orbit are a fraction of a degree apart), so the
// L2 serves most of their staging loads.  Logical slots past the last view of
// the last group are empty.  group = 0 keeps the plain order (tile x fastest,
// then row tile, then view, round-robin over the XCDs), which measured
// faster where the copy stays in the Infinity Cache.
struct BlockMap {
  int gx, gy, gz;  // column tiles, row tiles, views
  int group;       // adjacent views per group; 0 = the plain order
  int n_logical;   // group * gx * gy * ceil(gz / group) (gx * gy * gz for 0)
  int per_xcd;     // slots of each XCD: ceil(n_logical / 8)
};

// (column tile, row tile, view) of this workgroup, or false for an empty slot.
__device__ __forceinline__ bool map_block(const BlockMap& m, int& bx, int& by, int& bz) {
  const int n = blockIdx.x;
  if (m.group == 0) {
    if (n >= m.n_logical) return false;
    bx = n % m.gx;
    by = (n / m.gx) % m.gy;
    bz = n / (m.gx * m.gy);
    return true;
  }
  const int l = (n & 7) * m.per_xcd + (n >> 3);
  if (l >= m.n_logical) return false;
  const int vin = l % m.group;
  int rest = l / m.group;
  bx = rest % m.gx;
  rest /= m.gx;
  by = rest % m.gy;
  bz = (rest / m.gy) * m.group + vin;
  return bz < m.gz;
}

template <typename T, int MODE, int RPT, int NL>
// Every plan fits 128 VGPRs (the rows' z factors, uniform over a wave, sit in
// scalar registers): at least four waves per SIMD, four blocks per CU within
// LDS.
__global__ __launch_bounds__(256, 4) void k_project_staged(GeomDev g, BlockMap bm, const ViewInfo* __restrict__ views,
                                                        const ColInfo* __restrict__ cols,
                                                        const T* __restrict__ padN,
                                                        const T* __restrict__ padT,
                                                        const T* __restrict__ gin,
                                                        T* __restrict__ out, T* __restrict__ rl,
                                                        double* __restrict__ partials) {
  static_assert(NL >= 2 && NL <= kZPad + 1 && RPT > 1, "level stack");
  __shared__ double red[4];
  __shared__ int srange[8];
  __shared__ float4 tile[2][kStageRows * kStageF4];
  // the box table: packed into two ints per plane where the box is moved to
  // scalar registers (plans of at most 8 rows: (zl << 8 | nzr, tl4 << 8 |
  // nf4), the counts being at most kStageRows and kStageF4 on every plane
  // of a staged block), four ints otherwise
  constexpr bool kScalarBox = RPT <= 8;
  static_assert(kStageRows < 256 && kStageF4 < 256, "box counts packed in 8 bits");
  __shared__ std::conditional_t<kScalarBox, int2, int4> boxes[kStageBoxes];
  int bx, by, bz;
  if (!map_block(bm, bx, by, bz)) return;  // the whole block: before any barrier
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cblk = bx * 64, rblk = by * 4 * RPT;
  const int c = cblk + lane;
  const int r0 = rblk + wave * RPT;
  const int view = bz;
  const ViewInfo vi = views[view];
  const int nt = vi.step_x ? g.ny : g.nx;
  const int ns = vi.step_x ? g.nx : g.ny;
  const int nz = g.nz;
  const T* __restrict__ base = vi.step_x ? padT : padN;
  const float zc = 0.5f * (float)(nz - 1);
  const bool active = c < g.nu && r0 < g.nv;
  const ColInfo* __restrict__ cview = cols + (size_t)view * g.nu;
  const ColInfo ci = cview[min(c, g.nu - 1)];
  float vz[RPT];
  int lo = ns, hi = -1;  // union of the rows' windows
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    // uniform over the wave: kept in a scalar register
    vz[j] = __int_as_float(__builtin_amdgcn_readfirstlane(
        __float_as_int(((float)(r0 + j) - 0.5f * (float)(g.nv - 1)) * g.dvdz)));
    if (active && r0 + j < g.nv) {
      int l, h;
      plane_range(ci, vz[j], zc, nt, nz, l, h);
      if (l <= h) {
        lo = min(lo, l);
        hi = max(hi, h);
      }
    }
  }
  // the block's plane range
  int mlo = lo, mhi = hi;
  for (int off = 32; off > 0; off >>= 1) {
    mlo = min(mlo, __shfl_xor(mlo, off, 64));
    mhi = max(mhi, __shfl_xor(mhi, off, 64));
  }
  if (lane == 0) {
    srange[wave] = mlo;
    srange[4 + wave] = mhi;
  }
  __syncthreads();
  const int LO = min(min(srange[0], srange[1]), min(srange[2], srange[3]));
  const int HI = max(max(srange[4], srange[5]), max(srange[6], srange[7]));
  // corner rays: the block's first and last column, its first row and the
  // first row of its last wave
  const ColInfo cA = cview[cblk], cB = cview[min(cblk + 63, g.nu - 1)];
  const float vzA = ((float)rblk - 0.5f * (float)(g.nv - 1)) * g.dvdz;
  const float vzB = ((float)min(rblk + 3 * RPT, g.nv - 1) - 0.5f * (float)(g.nv - 1)) * g.dvdz;
  bool staged = LO <= HI;
  if (staged) {
    // Bounds of the box over all planes: the z span between the corner rays
    // (max of two linear functions minus min of two) and the trans width
    // |tB - tA| are convex in p, so their largest values over [LO, HI] are
    // at the ends; the floors, the 0.01 widenings, the stack height and the
    // 4-element alignment add at most the constants below.
    float span = 0.f, width = 0.f;
    for (int e = 0; e < 2; ++e) {
      const int pe = e ? HI : LO;
      const float z1 = z_index(cA, pe, vzA, zc), z2 = z_index(cB, pe, vzA, zc);
      const float z3 = z_index(cA, pe, vzB, zc), z4 = z_index(cB, pe, vzB, zc);
      span = fmaxf(span, fmaxf(z3, z4) - fminf(z1, z2));
      width = fmaxf(width, fabsf(trans_index(cB, pe) - trans_index(cA, pe)));
    }
    const int max_rows = (int)floorf(span + 0.02f) + NL + 1;
    const int max_f4 = (((int)floorf(width + 0.02f) + 5) >> 2) + 1;
    staged = max_rows <= kStageRows && max_f4 <= kStageF4;
  }
  float acc0[RPT], acc1[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) acc0[j] = acc1[j] = 0.f;
  if (staged) {
    // the boxes of all the block's planes, computed once (up to
    // kStageBoxes planes; beyond that each thread computes them itself)
    const bool table = HI - LO < kStageBoxes;
    if (table)
      for (int i = threadIdx.x; i <= HI - LO; i += 256) {
        const StageBox b = stage_box(cA, cB, vzA, vzB, LO + i, zc, nt, nz, NL);
        if constexpr (kScalarBox)
          boxes[i] = make_int2(b.zl * 256 + b.nzr, b.tl4 * 256 + b.nf4);
        else
          boxes[i] = make_int4(b.zl, b.nzr, b.tl4, b.nf4);
      }
    __syncthreads();
    auto get_box = [&](int p) {
      StageBox b;
      if constexpr (kScalarBox) {
        // the same for every thread: moved to scalar registers, so that
        // the staging addresses are computed on the scalar unit
        int x, y;
        if (table) {
          const int2 v = boxes[p - LO];
          x = v.x;
          y = v.y;
        } else {
          const StageBox c = stage_box(cA, cB, vzA, vzB, p, zc, nt, nz, NL);
          x = c.zl * 256 + c.nzr;
          y = c.tl4 * 256 + c.nf4;
        }
        x = __builtin_amdgcn_readfirstlane(x);
        y = __builtin_amdgcn_readfirstlane(y);
        b.zl = x >> 8;
        b.nzr = x & 0xff;
        b.tl4 = y >> 8;
        b.nf4 = y & 0xff;
      } else if (table) {
        const int4 v = boxes[p - LO];
        b.zl = v.x;
        b.nzr = v.y;
        b.tl4 = v.z;
        b.nf4 = v.w;
      } else {
        b = stage_box(cA, cB, vzA, vzB, p, zc, nt, nz, NL);
      }
      return b;
    };
    // this thread's (level row, vector) slots of the box and their offsets
    // from the box's first element; per plane only the first element moves
    const int zs = ns * pad_row(nt);
    int srow[kStageRegs], sq4[kStageRegs], soff[kStageRegs];
#pragma unroll
    for (int k = 0; k < kStageRegs; ++k) {
      const int e = threadIdx.x + 256 * k;
      srow[k] = e / kStageF4;
      sq4[k] = e % kStageF4;
      soff[k] = srow[k] * zs + 4 * sq4[k];
    }
    // Two register sets, so that a plane's loads are issued two planes
    // before its data go to LDS: iteration p issues plane p + 2's loads into
    // one set, samples plane p and stores plane p + 1 (loaded an iteration
    // earlier) from the other set into the tile buffer plane p - 1 used.
    using Raw = typename Raw4<T>::type;
    auto stage_load = [&](Raw (&r)[kStageRegs], int p) {
      const StageBox b = get_box(p);
      // the box's first vector; a non-empty box lies in the buffer, and the
      // clamp keeps an empty one's there too
      const int zl = min(max(b.zl, -kZPad), nz + kZPad - 1);
      const int tl4 = min(max(b.tl4, -4), pad_row(nt) - 4);
      const T* __restrict__ first = base + pad_index(ns, nt, zl, p, tl4);
      // a slot outside the box loads the box's first vector instead (in
      // bounds; the samples read only inside the box), so no load is
      // conditional
#pragma unroll
      for (int k = 0; k < kStageRegs; ++k) {
        const bool in = srow[k] < b.nzr && sq4[k] < b.nf4;
        if constexpr (kScalarBox)  // a 32-bit byte offset from the scalar first element
          r[k] = ld_raw4(reinterpret_cast<const T*>(reinterpret_cast<const char*>(first) +
                                                    (in ? (unsigned)soff[k] * sizeof(T) : 0u)));
        else
          r[k] = ld_raw4(first + (in ? soff[k] : 0));
      }
    };
    auto stage_store = [&](const Raw (&r)[kStageRegs], int buf) {
#pragma unroll
      for (int k = 0; k < kStageRegs; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e < kStageRows * kStageF4) tile[buf][e] = widen4<T>(r[k]);
      }
    };
    Raw regA[kStageRegs], regB[kStageRegs];
    stage_load(regA, LO);
    stage_store(regA, 0);
    stage_load(regB, min(LO + 1, HI));
    __syncthreads();
    // Loads and stores are unconditional (past HI the last plane is loaded
    // again and stored into the buffer no later plane reads), so that no
    // branch separates them and only the older set's loads are waited for.
    auto step = [&](int p, Raw (&ld_set)[kStageRegs], const Raw (&st_set)[kStageRegs]) {
      const int cur = (p - LO) & 1;
      stage_load(ld_set, min(p + 2, HI));
      if (p >= lo && p <= hi)
        sample_rows_lds<RPT, NL>(reinterpret_cast<const float*>(tile[cur]), get_box(p), ci, p, vz,
                                 zc, nt, nz, acc0);
      stage_store(st_set, cur ^ 1);
      __syncthreads();
    };
    for (int p = LO; p <= HI; p += 2) {
      step(p, regA, regB);
      if (p + 1 <= HI) step(p + 1, regB, regA);
    }
  } else if (active) {
    const int ntp = pad_row(nt), zs = ns * ntp;
    const T* __restrict__ vb = base + pad_index(ns, nt, 0, 0, 0);
    int p = lo;
    for (; p < hi; p += 2) {
      sample_rows<T, RPT, NL>(vb, ci, p, vz, zc, nt, nz, ns, ntp, zs, acc0);
      sample_rows<T, RPT, NL>(vb, ci, p + 1, vz, zc, nt, nz, ns, ntp, zs, acc1);
    }
    if (p == hi) sample_rows<T, RPT, NL>(vb, ci, p, vz, zc, nt, nz, ns, ntp, zs, acc0);
  }
  double part = 0.0;
  if (active) {
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
        const float rs = as_stored<T>(res);  // the stored (rounded) residual
        st(rl + o, ell * rs);
        part += (double)rs * (double)rs;
      } else {
        st(out + o, val);
        const float qs = as_stored<T>(val);
        part += (double)qs * (double)qs;
      }
    }
  }
  if (MODE != 0) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0) partials[((size_t)bz * bm.gy + by) * bm.gx + bx] = s;
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
  const RowPlan cand[] = {{16, 6}, {8, 4}, {8, 6}, {8, 7}, {4, 3}, {4, 4}, {2, 3}};
  // 16 rows per thread only when its grid fills the chip a few times over
  // (about 768 blocks run at once); a smaller grid (the coarse level of the
  // multigrid) takes the first 8-row plan that fits, twice the blocks
  const long blocks16 = (long)((g.nu + 63) / 64) * ((g.nv + 63) / 64) * g.n_views;
  const bool small = blocks16 < 1536;
  for (const RowPlan& c : cand)
    if (std::ceil((c.rpt - 1) * row_span + 0.05) + 2.0 <= (double)c.nl && !(small && c.rpt > 8))
      return c;
  return {1, 2};
}

// Adjacent views per XCD group of the staged projector's launch: 16 when a
// padded copy exceeds 100 MB (it cannot stay in the 256 MB Infinity Cache
// with the rest of the working set), else the plain order.  Per call with
// its padded copies, at 512x512x256 with 360 views (283 MB copies): 44.7 ms
// in the plain order, 42.3 with contiguous chunks per XCD and no grouping,
// 38.3 with groups of 4 or 8, 37.3-37.9 with 16; at 512x512x70 (87 MB):
// 1.69 ms in the plain order, 1.69-1.71 with groups of 1-8, 1.86 with 16.
static int xcd_view_group(const GeomDev& g, size_t elem_bytes) {
  const double copy_bytes = (double)pad_elems_vol(g.nx, g.ny, g.nz) * (double)elem_bytes;
  return copy_bytes > 100e6 ? 16 : 0;
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
  if (RPT > 1) {
    BlockMap bm;
    bm.gx = (int)grid.x;
    bm.gy = (int)grid.y;
    bm.gz = (int)grid.z;
    bm.group = xcd_view_group(g, sizeof(T));
    bm.n_logical = bm.group == 0
                       ? bm.gx * bm.gy * bm.gz
                       : bm.group * bm.gx * bm.gy * ((bm.gz + bm.group - 1) / bm.group);
    bm.per_xcd = (bm.n_logical + 7) / 8;
    hipLaunchKernelGGL((k_project_staged<T, MODE, (RPT > 1 ? RPT : 2), NL>),
                       dim3((unsigned)(8 * bm.per_xcd)), block, 0, s, g, bm, views, cols, padN,
                       padT, gin, out, rl, partials);
  } else
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
  else if (rp.rpt == 8 && rp.nl == 6)
    launch_project_rows<T, MODE, 8, 6>(g, views, cols, padN, padT, gin, out, rl, partials,
                                       n_partials, s);
  else if (rp.rpt == 8)
    launch_project_rows<T, MODE, 8, 7>(g, views, cols, padN, padT, gin, out, rl, partials,
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
constexpr int kResRows = 4;  // row groups per block of the residual update

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
  const int view = blockIdx.z;
  double part = 0.0;
  if (c < g.nu) {
    // a wave takes one row of 64 columns, the block kResRows groups of 4 rows
    const ViewInfo vi = views[view];
    const ColInfo ci = cols[(size_t)view * g.nu + c];
    const bool stopped = sc->stopped != 0;
    const float alpha = (float)sc->alpha;
#pragma unroll
    for (int k = 0; k < kResRows; ++k) {
      const int row = blockIdx.y * 4 * kResRows + 4 * k + (threadIdx.x >> 6);
      if (row < g.nv) {
        const size_t o = ((size_t)view * g.nv + row) * g.nu + c;
        float rv = ld(r + o);
        if (!stopped) {
          rv = rv - alpha * ld(q + o);
          st(r + o, rv);
          rv = as_stored<T>(rv);
        }
        st(rl + o, ray_length(g, vi, ci, row) * rv);
        part += (double)rv * (double)rv;
      }
    }
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
  dim3 grid((g.nu + 63) / 64, (g.nv + 4 * kResRows - 1) / (4 * kResRows), g.n_views);
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
