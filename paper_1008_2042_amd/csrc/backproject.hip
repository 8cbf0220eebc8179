// Backprojector P^T: the exact transpose of the Joseph projector, evaluated
// as a gather, one thread per voxel run, no atomics (the paper's section
// 2.2.2 motivates a voxel-driven P^T by the write conflicts of a ray-driven
// one; here the voxel-driven form is the exact matrix transpose rather than
// the continuous closed form of Eq. (3)).
//
// For voxel (i, j, k) and a view stepping along axis s, the voxel lies on
// plane p (its index along s) at trans index t.  Ray (c, r) weights it by
// l(c,r) * hat(t_p(c) - t) * hat(z_p(c,r) - k), with the projector's FP32
// expressions for t_p and z_p (same table entries, same FMAs).  The columns
// with hat(t_p(c) - t) > 0 are those whose detector coordinate lies between
// the projections of the trans neighbours t - 1 and t + 1 on plane p; for
// each such column the rows follow from the z index of the row.  The
// projections are prescaled by l (rl = l * g) once per application.
//
// Mapping: 256-thread blocks of kBX (x) x kBY (y) voxel columns; each thread
// accumulates a run of K voxels along z.  Per view the block first stages
// its whole detector footprint (the bounding box of the projection of its
// voxel box grown by one voxel, the support of the hat weights) into LDS as
// running sums down each detector column (coalesced row loads), so that a z
// segment's two sums are two differences of staged values and no row is
// visited per voxel; a view whose footprint does not fit is read from global
// memory row by row instead.
// Within a column the footprint rows are split into z segments (rows whose
// z index lies between two voxel centres); the segment sums of g and fr * g
// give both tent weights.
#include "tfcb_internal.h"

namespace tfcb {

constexpr int kZRun = 8;        // voxels per thread along z
constexpr int kPrefTile = 4096; // LDS float pairs for one view's staged footprint (32 KB)
constexpr int kChunks = 1;      // 64-column chunks of the four-wave scan
constexpr int kPrefCols = 1;    // bracket columns whose table records are fetched before the scan
constexpr int kQuarterRows = 16; // footprint rows per wave in the four-wave scan
// voxel columns of a block: 16 x 16 keeps the footprint of a view smaller
// than 64 x 4 would (about half the area at the paper's geometry, and at
// most 60 detector columns at the 512 x 512 x 256 geometry, so one 64-column
// chunk of the scan)
constexpr int kBX = 16, kBY = 16;
static_assert(kBX * kBY == 256 && 64 % kBX == 0, "block shape");

// One detector column's contribution to the K voxels of a z-run, with trans
// weight wt, in second-difference form.  Segment m = 0..K holds the rows
// whose z index zh_r lies in [k0 - 1 + m, k0 + m); they give (1 - fr) of
// their value to voxel k0 - 1 + m and fr to voxel k0 + m,
// fr = zh_r - (k0 - 1 + m).  With zh_r = zh_rm + zstep (r - rm) (zh_rm the
// projector's expression for a reference row rm, zstep = tau dv/dz) and the
// column's prefix sums X(e) = sum_{r < e} g_r, Y(e) = sum_{r < e} (r - rm) g_r
// taken at the segment bounds e_{-1} < e_0 <= ... <= e_K, segment m has
// S_m = X(e_m) - X(e_{m-1}) and sum fr g = coef_m S_m + zstep (Y(e_m) -
// Y(e_{m-1})), coef_m = zh_rm - (k0 - 1 + m).  Voxel q then receives
//   B_{q-1} - 2 B_q + B_{q+1},   B_m = (1 - coef_m) X(e_m) - zstep Y(e_m),
// (the tent's second difference of the integrated column).  That is linear
// in B, so the run keeps bsum_m = sum over views and columns of wt B_m
// (m = -1..K) and forms the voxels once at the end; a constant added to X or
// Y (another origin of the sums) changes B by a linear function of m, which
// the second difference removes.  Bounds: e_m is the first row of z index
// >= k0 + m, ceil((k0 + m - zc) / zstep + rc), clamped to the rows present;
// a row misplaced by rounding at a bound has fr within an ulp of 0 or 1.
//
// This form reads the rows from global memory (row r at col[r * stride]),
// summing them once from the first bound on.
template <int K, typename P>
__device__ __forceinline__ void column_to_run(const P* __restrict__ col, int stride, int r0,
                                              int r1, int rm, float a, float inv_s, float aw,
                                              float wt, float bw, float (&bsum)[K + 2]) {
  int r = min(r1 + 1, max(r0, (int)ceilf(a)));
  float X = 0.f, Y = 0.f, w = (float)(r - rm);
  // bsum[0] gets aw * 0 + bw * 0 at the first bound
  aw += wt;
#pragma unroll
  for (int m = 0; m <= K; ++m) {
    a += inv_s;
    const int e = min(r1 + 1, max(r, (int)ceilf(a)));
    for (; r < e; ++r) {
      const float g = ld(col + (size_t)r * stride);
      X += g;
      Y = fmaf(w, g, Y);
      w += 1.f;
    }
    bsum[m + 1] = fmaf(aw, X, bsum[m + 1]);
    bsum[m + 1] = fmaf(bw, Y, bsum[m + 1]);
    aw += wt;
  }
}

// -ceil(a) as floor(-a), in one conversion
__device__ __forceinline__ int neg_ceil(float a) {
  int r;
  asm("v_cvt_flr_i32_f32_e64 %0, -%1" : "=v"(r) : "v"(a));
  return r;
}
// x clamped to [lo, hi]
__device__ __forceinline__ int clamp3(int x, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}
// b - 8 f for |f| < 2^23
__device__ __forceinline__ int minus8_add(int f, int b) {
  int r;
  asm("v_mad_i32_i24 %0, %1, -8, %2" : "=v"(r) : "v"(f), "v"(b));
  return r;
}

// The same from the column's prefix sums staged in LDS: entry e of the
// column (byte offset colb + 8 e, e = r0..r1 + 1) holds (X(e), Y(e)) summed
// from the footprint's first row r0.  Bounds are handled as f = -e, so that
// the clamp and the address take one instruction each.
template <int K>
__device__ __forceinline__ void column_to_run_prefix(const float2* __restrict__ pre, int colb,
                                                     int nlo, int nhi, float a, float inv_s,
                                                     float aw, float wt, float bw,
                                                     float (&bsum)[K + 2]) {
  const char* __restrict__ base = reinterpret_cast<const char*>(pre);
#pragma unroll
  for (int m = -1; m <= K; ++m) {
    if (m >= 0) a += inv_s;
    const float2 pe =
        *reinterpret_cast<const float2*>(base + minus8_add(clamp3(neg_ceil(a), nlo, nhi), colb));
    bsum[m + 1] = fmaf(aw, pe.x, bsum[m + 1]);
    bsum[m + 1] = fmaf(bw, pe.y, bsum[m + 1]);
    aw += wt;
  }
}

template <typename T, int K>
__global__ __launch_bounds__(256, 4) void k_backproject(GeomDev g, const ViewInfo* __restrict__ views,
                                                     const ColInfo* __restrict__ cols,
                                                     const T* __restrict__ rl,
                                                     T* __restrict__ vol,
                                                     double* __restrict__ partials) {
  __shared__ double red[4];
  __shared__ float2 pre[kPrefTile];
  // group totals of the four-wave scan: 3 x 64 (quarters) or 7 x 32 (halves)
  __shared__ float2 qtot[256];
  __shared__ float cbox[2][2][8];  // projected corner columns / rows, two views
  const float rc = 0.5f * (float)(g.nv - 1);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * kBX + (int)(threadIdx.x % kBX);
  const int j = blockIdx.y * kBY + (int)(threadIdx.x / kBX);
  const int k0 = blockIdx.z * K;
  const bool active = i < g.nx && j < g.ny;
  const float xc = 0.5f * (float)(g.nx - 1), yc = 0.5f * (float)(g.ny - 1);
  const float zc = 0.5f * (float)(g.nz - 1);
  const float cu = 0.5f * (float)(g.nu - 1);
  const float inv_du = 1.f / g.du, inv_dv = 1.f / g.dv;
  const float X = ((float)i - xc) * g.dx, Y = ((float)j - yc) * g.dy;
  // the block's voxel box grown by one voxel on every side (mm); signed
  // arithmetic: the first block's lower bound is index -1
  const int bi = (int)blockIdx.x * kBX, bj = (int)blockIdx.y * kBY;
  const float bx0 = ((float)(bi - 1) - xc) * g.dx;
  const float bx1 = ((float)min(g.nx, bi + kBX) - xc) * g.dx;
  const float by0 = ((float)(bj - 1) - yc) * g.dy;
  const float by1 = ((float)min(g.ny, bj + kBY) - yc) * g.dy;
  const float bz0 = ((float)(k0 - 1) - zc) * g.dz;
  const float bz1 = ((float)(min(g.nz, k0 + K)) - zc) * g.dz;

  // second-difference accumulators of the run (bounds k0 - 1 .. k0 + K)
  float bsum[K + 2];
#pragma unroll
  for (int q = 0; q < K + 2; ++q) bsum[q] = 0.f;

  // footprint box of a view: the 8 corners of the grown voxel box
  // projected to (column, row), one corner per thread
  auto corners = [&](int view, int buf) {
    if (threadIdx.x < 8) {
      const ViewInfo vc = views[view];
      const float cx = (threadIdx.x & 1) ? bx1 : bx0;
      const float cy = (threadIdx.x & 2) ? by1 : by0;
      const float cz = (threadIdx.x & 4) ? bz1 : bz0;
      const float den = __builtin_amdgcn_rcpf(g.sad - (cx * vc.cs + cy * vc.sn));
      cbox[buf][0][threadIdx.x] = fmaf(g.sdd * (-cx * vc.sn + cy * vc.cs) * den, inv_du, cu);
      cbox[buf][1][threadIdx.x] = fmaf(g.sdd * cz * den, inv_dv, rc);
    }
  };
  corners(0, 0);
  __syncthreads();
  // wave index as a scalar, so that the scan's row bounds are uniform branches
  const int wv = __builtin_amdgcn_readfirstlane(wave);

  // Per view, two barriers: B1 (the previous view's reads of the tile are
  // done, the quarter totals are visible) and B2 (the tile is complete).
  // The next view's corners are projected between them into the other
  // half of cbox.
  for (int view = 0; view < g.n_views; ++view) {
    const ViewInfo vi = views[view];
    const T* __restrict__ rview = rl + (size_t)view * g.nv * g.nu;
    const int cb = view & 1;
    float umin = cbox[cb][0][0], umax = umin, vmin = cbox[cb][1][0], vmax = vmin;
#pragma unroll
    for (int e = 1; e < 8; ++e) {
      umin = fminf(umin, cbox[cb][0][e]);
      umax = fmaxf(umax, cbox[cb][0][e]);
      vmin = fminf(vmin, cbox[cb][1][e]);
      vmax = fmaxf(vmax, cbox[cb][1][e]);
    }
    // the same in every lane: held as scalars
    const int c0 = __builtin_amdgcn_readfirstlane(max(0, (int)floorf(umin) - 1));
    const int c1 = __builtin_amdgcn_readfirstlane(min(g.nu - 1, (int)ceilf(umax) + 1));
    const int r0 = __builtin_amdgcn_readfirstlane(max(0, (int)floorf(vmin) - 1));
    const int r1 = __builtin_amdgcn_readfirstlane(min(g.nv - 1, (int)ceilf(vmax) + 1));
    const int W = c1 - c0 + 1, H = r1 - r0 + 1;
    const int rm = r0 + (H >> 1);
    // Column-major prefix sums with an odd column stride Hp (adjacent columns
    // in different banks).  Four-wave scan of footprints up to 128 x 64:
    // wave w takes footprint rows [16 w, 16 w + 16) of both 64-column
    // chunks, and Hp = 16 ceil(H / 16) + 1 leaves room for the last
    // quarter's rows past H, so every quarter loads and writes 16 rows
    // without per-row conditions (rows past H load row r1 again and land in
    // the column's padding, which is never read; no later quarter uses that
    // wave's totals).  Other footprints: stride (H + 1) | 1, scanned a
    // column per lane.
    const int Hq = 16 * ((H + 15) >> 4) + 1;
    const bool quarters = W > 0 && H > 0 && W <= kChunks * 64 && H <= 4 * kQuarterRows &&
                          W * Hq <= kPrefTile;
    const int Hp = quarters ? Hq : ((H + 1) | 1);
    const bool staged = quarters || (W > 0 && H > 0 && W * Hp <= kPrefTile);
    // Footprints at most 32 columns wide are scanned in halves: each wave
    // takes two groups of 8 rows, one per half-wave (lanes 0-31 rows
    // [16 w, 16 w + 8), lanes 32-63 rows [16 w + 8, 16 w + 16)), so a lane
    // sums 8 rows instead of 16.  The scalar row pointer then steps without
    // the clamp at r1 (the upper half reads 8 rows below it): rows past the
    // footprint land, as before, in groups no later group reads and in the
    // column's padding.  An active group starts above row H, so the rows
    // read reach r1 + 7 at most; those must lie in the buffer, which holds
    // for every view but the bottom rows of the last one (such a view takes
    // the quarter scan).
    const bool halves = quarters && W <= 32 && r1 + 7 < (g.n_views - view) * g.nv;
    const int hsel = halves ? (lane >> 5) : 0;
    const int grp = halves ? 2 * wv + hsel : wv;  // this lane's row group
    const int cl = halves ? (lane & 31) : lane;   // this lane's footprint column
    const int q0 = (halves ? 8 : kQuarterRows) * grp;
    const bool qrows = quarters && q0 < H;  // this lane's group has rows to scan
    const float wq = (float)(r0 + q0 - rm);  // row offset of the group's first row
    float qv[kChunks][kQuarterRows];
    if (qrows) {
      if (halves) {
        // a scalar row pointer stepped down 8 rows from row 16 w, a 32-bit
        // offset per lane (its column, and 8 rows for the upper half)
        const uint32_t cb = (uint32_t)((min(cl, W - 1) + hsel * 8 * g.nu) * (int)sizeof(T));
        const T* __restrict__ rp = rview + (size_t)(r0 + kQuarterRows * wv) * g.nu + c0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          qv[0][u] = ld(reinterpret_cast<const T*>(reinterpret_cast<const char*>(rp) + cb));
          rp += g.nu;
        }
      } else {
#pragma unroll
        for (int h = 0; h < kChunks; ++h) {
          if (h == 1 && W <= 64) break;
          // a scalar row pointer stepped down the rows, a 32-bit column offset per lane
          const uint32_t cb = (uint32_t)(min(lane + 64 * h, W - 1) * sizeof(T));
          const T* __restrict__ rp = rview + (size_t)(r0 + q0) * g.nu + c0;
          int row = r0 + q0;
#pragma unroll
          for (int u = 0; u < kQuarterRows; ++u) {
            qv[h][u] = ld(reinterpret_cast<const T*>(reinterpret_cast<const char*>(rp) + cb));
            const bool step = row < r1;
            rp += step ? g.nu : 0;
            row += step ? 1 : 0;
          }
        }
      }
    }
    // This thread's plane, trans index and bracket of columns, and their
    // table records, loaded before the tile is built so that their latency
    // overlaps it.
    int p, t;
    float Xa, Ya, Xb, Yb;  // the trans neighbours t - 1 and t + 1 on plane p
    if (vi.step_x) {
      p = i;
      t = j;
      Xa = X;
      Xb = X;
      Ya = Y - g.dy;
      Yb = Y + g.dy;
    } else {
      p = j;
      t = i;
      Ya = Y;
      Yb = Y;
      Xa = X - g.dx;
      Xb = X + g.dx;
    }
    // detector column of a point: u = sdd (-x sn + y cs) / (sad - (x cs + y sn));
    // the hardware reciprocal is accurate to ~1e-4 column here
    const float ua = g.sdd * (-Xa * vi.sn + Ya * vi.cs) *
                     __builtin_amdgcn_rcpf(g.sad - (Xa * vi.cs + Ya * vi.sn));
    const float ub = g.sdd * (-Xb * vi.sn + Yb * vi.cs) *
                     __builtin_amdgcn_rcpf(g.sad - (Xb * vi.cs + Yb * vi.sn));
    const float ca = fmaf(ua, inv_du, cu), cbc = fmaf(ub, inv_du, cu);
    // a column has a non-zero trans weight only strictly between ca and cbc
    // (the margin covers the reciprocal's error); all of them lie inside
    // the footprint box
    const int clo = !active ? 1 : max(c0, (int)floorf(fminf(ca, cbc) - 1e-3f) + 1);
    const int chi = !active ? 0 : min(c1, (int)ceilf(fmaxf(ca, cbc) + 1e-3f) - 1);
    const ColInfo* __restrict__ cview = cols + (size_t)view * g.nu;
    float4 pf0[kPrefCols];
    int4 pf1[kPrefCols];
#pragma unroll
    for (int q = 0; q < kPrefCols; ++q) {
      const int c = min(clo + q, g.nu - 1);
      if (clo + q <= chi) {
        pf0[q] = reinterpret_cast<const float4*>(cview + c)[0];
        pf1[q] = reinterpret_cast<const int4*>(cview + c)[1];
      }
    }
    if (halves) {
      // sum (wq + u) v = wq sum v + sum u v
      if (qrows && grp < 7 && cl < W) {
        float s0 = 0.f, su = 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          s0 += qv[0][u];
          su = fmaf((float)u, qv[0][u], su);
        }
        qtot[grp * 32 + cl] = make_float2(s0, fmaf(wq, s0, su));
      }
    } else if (qrows && wv < 3) {
#pragma unroll
      for (int h = 0; h < kChunks; ++h) {
        if (h == 1 && W <= 64) break;
        // sum (wq + u) v = wq sum v + sum u v
        float s0 = 0.f, su = 0.f;
#pragma unroll
        for (int u = 0; u < kQuarterRows; ++u) {
          s0 += qv[h][u];
          su = fmaf((float)u, qv[h][u], su);
        }
        const int cc = lane + 64 * h;
        if (cc < W) qtot[wv * 64 + cc] = make_float2(s0, fmaf(wq, s0, su));
      }
    }
    __syncthreads();  // B1
    if (view + 1 < g.n_views) corners(view + 1, cb ^ 1);
    if (qrows && halves) {
      if (cl < W) {
        float s0 = 0.f, s1 = 0.f, w = wq;
        for (int k = 0; k < grp; ++k) {
          const float2 qt = qtot[k * 32 + cl];
          s0 += qt.x;
          s1 += qt.y;
        }
        float2* __restrict__ dst = pre + cl * Hp + q0 + 1;
        if (grp == 0) dst[-1] = make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          s0 += qv[0][u];
          s1 = fmaf(w, qv[0][u], s1);
          w += 1.f;
          dst[u] = make_float2(s0, s1);
        }
      }
    } else if (qrows) {
#pragma unroll
      for (int h = 0; h < kChunks; ++h) {
        if (h == 1 && W <= 64) break;
        const int cc = lane + 64 * h;
        if (cc < W) {
          float s0 = 0.f, s1 = 0.f, w = wq;
          for (int k = 0; k < wv; ++k) {
            const float2 qt = qtot[k * 64 + cc];
            s0 += qt.x;
            s1 += qt.y;
          }
          float2* __restrict__ dst = pre + cc * Hp + q0 + 1;
          if (wv == 0) dst[-1] = make_float2(0.f, 0.f);
#pragma unroll
          for (int u = 0; u < kQuarterRows; ++u) {
            s0 += qv[h][u];
            s1 = fmaf(w, qv[h][u], s1);
            w += 1.f;
            dst[u] = make_float2(s0, s1);
          }
        }
      }
    } else if (staged) {
      // a wave scans 64 columns down the footprint's rows with coalesced
      // loads, 8 rows in flight per lane
      for (int chunk = wave * 64; chunk < W; chunk += 256) {
        const int cc = chunk + lane;
        const bool own = cc < W;
        const T* __restrict__ src = rview + (size_t)r0 * g.nu + (c0 + min(cc, W - 1));
        float2* __restrict__ dst = pre + cc * Hp;
        float s0 = 0.f, s1 = 0.f;
        if (own) dst[0] = make_float2(0.f, 0.f);
        for (int rr = 0; rr < H; rr += 8) {
          float w8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) w8[u] = rr + u < H ? ld(src + (size_t)(rr + u) * g.nu) : 0.f;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (rr + u < H) {
              s0 += w8[u];
              s1 = fmaf((float)(r0 + rr + u - rm), w8[u], s1);
              if (own) dst[rr + u + 1] = make_float2(s0, s1);
            }
          }
        }
      }
    }
    __syncthreads();  // B2
    if (!active || W <= 0 || H <= 0) continue;
    const float fp = (float)p;
    // per column: a = the argument of the first bound's ceiling, and the
    // weights of X and Y in wt B_m, aw = wt (1 - coef_m) from m = -1 on and
    // bw = -wt zstep
    const float kz = (float)(k0 - 1) - zc;
    const float vzm = ((float)rm - rc) * g.dvdz;  // the projector's vz for row rm
    if (staged) {
      // Every column of the bracket is evaluated; one whose plane lies
      // outside 0 < tau < 1 or with no trans weight gets weight 0 (its table
      // entries are finite and its bounds are clamped into the tile).
      const int nlo = -(r1 + 1), nhi = -r0;
      auto column = [&](int c, const float4& h0, const int4& h1) {
        const float th = fmaf(fp, h0.y, h0.x);
        float wt = 1.f - fabsf(th - (float)t);
        wt = (p >= h1.z && p <= h1.w && wt > 0.f) ? wt : 0.f;
        const float tau = fmaf(fp, h0.w, h0.z);
        const float zstep = tau * g.dvdz;
        const float inv_s = __builtin_amdgcn_rcpf(zstep);
        const float coef0 = fmaf(tau, vzm, zc) - (float)(k0 - 1);
        const int colb = ((c - c0) * Hp - r0) * (int)sizeof(float2);
        column_to_run_prefix<K>(pre, colb, nlo, nhi, fmaf(kz, inv_s, rc), inv_s, -wt * coef0, wt,
                                -wt * zstep, bsum);
      };
#pragma unroll
      for (int q = 0; q < kPrefCols; ++q)
        if (clo + q <= chi) column(clo + q, pf0[q], pf1[q]);
      for (int c = clo + kPrefCols; c <= chi; ++c)
        column(c, reinterpret_cast<const float4*>(cview + c)[0],
               reinterpret_cast<const int4*>(cview + c)[1]);
    } else {
      for (int c = clo; c <= chi; ++c) {
        const float4 h0 = reinterpret_cast<const float4*>(cview + c)[0];
        const int4 h1 = reinterpret_cast<const int4*>(cview + c)[1];
        const float th = fmaf(fp, h0.y, h0.x);
        const float wt = 1.f - fabsf(th - (float)t);
        // plane outside 0 < tau < 1, or no trans weight
        if (p < h1.z || p > h1.w || !(wt > 0.f)) continue;
        const float tau = fmaf(fp, h0.w, h0.z);
        const float zstep = tau * g.dvdz;
        const float inv_s = __builtin_amdgcn_rcpf(zstep);
        const float coef0 = fmaf(tau, vzm, zc) - (float)(k0 - 1);
        column_to_run<K>(rview + c, g.nu, r0, r1, rm, fmaf(kz, inv_s, rc), inv_s, -wt * coef0,
                         wt, -wt * zstep, bsum);
      }
    }
  }

  double part = 0.0;
  if (active) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (k0 + q < g.nz) {
        const size_t o = ((size_t)(k0 + q) * g.ny + j) * g.nx + i;
        st(vol + o, fmaf(-2.f, bsum[q + 1], bsum[q] + bsum[q + 2]));
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
  return ((g.nx + kBX - 1) / kBX) * ((g.ny + kBY - 1) / kBY) * ((g.nz + kZRun - 1) / kZRun);
}

template <typename T>
hipError_t launch_backproject(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                              const T* rl, T* vol, double* partials, int* n_partials,
                              hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, (g.nz + kZRun - 1) / kZRun);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL((k_backproject<T, kZRun>), grid, block, 0, s, g, views, cols, rl, vol,
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
