// The paper's own operator pair: Siddon's ray-tracing projector (section
// 2.2.1) and the closed-form voxel-driven backprojection of Eq. (3)
// (section 2.2.2, Appendix 2).  The two are not transposes of each other
// (the paper measures their adjoint mismatch at under 1 %); CGLS uses the
// second in place of P^T, as the paper does.
//
// Siddon P: one thread per ray.  Voxels are boxes of size dx dy dz around
// the voxel centres (half-open along each axis), and the ray's value is the
// sum over the voxels it crosses of the value times the length inside the
// box.  The traversal is the incremental form (Jacobs et al.): per moving
// axis the parameter of the next face crossing, the piece up to the nearest
// one belongs to the current voxel, and the axes whose face is reached move
// on.  Every face parameter of an axis comes from one expression,
// (face position - source) / a, also for the ray's entry and exit, so the
// walk never leaves the volume and ends after at most nx + ny + nz + 3
// steps.  It reads the zero-padded volume copies that the CGLS keeps for P
// (the one whose fastest axis is the view's trans axis).
//
// Eq. (3) P^T: one thread per z-run of K voxels of one (x, y) column; per
// view the in-plane part of the projection (magnification, detector column
// and its bilinear weights, in-plane distances) is shared by the run, and
// each voxel adds L^3 / (L0 l^2) times the bilinear interpolation of the
// projection at its hit point (taps off the detector read zero).
#include <cmath>

#include "tfcb_internal.h"

namespace tfcb {

constexpr int kEq3Run = 8;  // voxels per thread along z (the P^T grid shape)

struct SiddonAxis {
  float s, lo, d, inv;  // face b sits at lo + b d, crossed at alpha = (lo + b d - s) inv
  int n;
  int dir;    // +1 / -1: direction of travel along the axis; 0: parallel to its faces
  int fixed;  // voxel index along a non-moving axis (-1: outside the volume)
};

// Axis set-up for a ray s + alpha a, alpha in [0, 1], against n boxes of
// size d starting at lo.
__device__ __forceinline__ SiddonAxis siddon_axis(float s, float a, float lo, float d, int n) {
  SiddonAxis ax;
  ax.s = s;
  ax.lo = lo;
  ax.d = d;
  ax.n = n;
  ax.fixed = 0;
  if (fabsf(a) < 1e-30f) {  // parallel to the faces (also keeps 1 / a finite)
    ax.dir = 0;
    ax.inv = 0.f;
    // half-open boxes [lo + i d, lo + (i + 1) d)
    const float t = floorf((s - lo) / d);
    ax.fixed = (t >= 0.f && t < (float)n) ? (int)t : -1;
    return ax;
  }
  ax.dir = a > 0.f ? 1 : -1;
  ax.inv = 1.f / a;
  return ax;
}

// Crossing parameter of face b (the face position first, so a ray almost
// parallel to the faces keeps its precision).
__device__ __forceinline__ float face_alpha(const SiddonAxis& ax, int b) {
  return (fmaf((float)b, ax.d, ax.lo) - ax.s) * ax.inv;
}
// The m-th face the ray crosses along this axis (m = 0..n).
__device__ __forceinline__ int face_of(const SiddonAxis& ax, int m) {
  return ax.dir > 0 ? m : ax.n - m;
}

// Number m of this axis's faces crossed at or before amin, 1 <= m <= n
// (the ray enters the volume at amin, at or after this axis's first face,
// and leaves it after amin, at or before its last face).
__device__ __forceinline__ int faces_before(const SiddonAxis& ax, float a, float amin) {
  const float b = floorf((fmaf(amin, a, ax.s) - ax.lo) / ax.d);  // voxel at the entry point
  int m = ax.dir > 0 ? (int)b + 1 : ax.n - (int)b;
  m = min(max(m, 1), ax.n);
  while (m > 1 && face_alpha(ax, face_of(ax, m - 1)) > amin) --m;
  while (m < ax.n && face_alpha(ax, face_of(ax, m)) <= amin) ++m;
  return m;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_project_siddon(GeomDev g, const ViewInfo* __restrict__ views,
                                                        const T* __restrict__ padN,
                                                        const T* __restrict__ padT,
                                                        const T* __restrict__ gin,
                                                        T* __restrict__ out,
                                                        double* __restrict__ partials) {
  __shared__ double red[4];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int view = blockIdx.z;
  double part = 0.0;
  if (c < g.nu && r < g.nv) {
    const ViewInfo vi = views[view];
    const float uc = ((float)c - 0.5f * (float)(g.nu - 1)) * g.du;
    const float vr = ((float)r - 0.5f * (float)(g.nv - 1)) * g.dv;
    const float ax_ = fmaf(-g.sdd, vi.cs, -uc * vi.sn);
    const float ay_ = fmaf(-g.sdd, vi.sn, uc * vi.cs);
    const float az_ = vr;
    const float lox = -0.5f * (float)g.nx * g.dx, loy = -0.5f * (float)g.ny * g.dy;
    const float loz = -0.5f * (float)g.nz * g.dz;
    const SiddonAxis X = siddon_axis(vi.sx, ax_, lox, g.dx, g.nx);
    const SiddonAxis Y = siddon_axis(vi.sy, ay_, loy, g.dy, g.ny);
    const SiddonAxis Z = siddon_axis(0.f, az_, loz, g.dz, g.nz);
    // the part of [0, 1] inside the volume: after every moving axis's first
    // face, before every one's last
    float amin = 0.f, amax = 1.f;
    const bool hit = X.fixed >= 0 && Y.fixed >= 0 && Z.fixed >= 0;
    if (X.dir) {
      amin = fmaxf(amin, face_alpha(X, face_of(X, 0)));
      amax = fminf(amax, face_alpha(X, face_of(X, g.nx)));
    }
    if (Y.dir) {
      amin = fmaxf(amin, face_alpha(Y, face_of(Y, 0)));
      amax = fminf(amax, face_alpha(Y, face_of(Y, g.ny)));
    }
    if (Z.dir) {
      amin = fmaxf(amin, face_alpha(Z, face_of(Z, 0)));
      amax = fminf(amax, face_alpha(Z, face_of(Z, g.nz)));
    }
    float sum = 0.f;
    if (hit && amax > amin) {
      // per moving axis: index bx of the next face to cross and its
      // parameter; the voxel lies behind that face
      int ix = X.fixed, iy = Y.fixed, iz = Z.fixed;
      int bx = 0, by = 0, bz = 0;
      float nxa = INFINITY, nya = INFINITY, nza = INFINITY;
      if (X.dir) {
        bx = face_of(X, faces_before(X, ax_, amin));
        ix = X.dir > 0 ? bx - 1 : bx;
        nxa = face_alpha(X, bx);
      }
      if (Y.dir) {
        by = face_of(Y, faces_before(Y, ay_, amin));
        iy = Y.dir > 0 ? by - 1 : by;
        nya = face_alpha(Y, by);
      }
      if (Z.dir) {
        bz = face_of(Z, faces_before(Z, az_, amin));
        iz = Z.dir > 0 ? bz - 1 : bz;
        nza = face_alpha(Z, bz);
      }
      // Offsets in a padded copy: views stepping along y read the native
      // copy [nz + 2 kZPad][ny][pad_row(nx)], those stepping along x the
      // transposed one [nz + 2 kZPad][nx][pad_row(ny)], so that adjacent detector
      // columns (lanes) walk adjacent addresses of the fastest axis.
      const T* __restrict__ vb;
      int o, ox, oy, oz;
      if (vi.step_x) {
        const int rowp = pad_row(g.ny), slab = g.nx * rowp;
        vb = padT + pad_index(g.nx, g.ny, 0, 0, 0);
        o = (iz * g.nx + ix) * rowp + iy;
        ox = X.dir * rowp;
        oy = Y.dir;
        oz = Z.dir * slab;
      } else {
        const int rowp = pad_row(g.nx), slab = g.ny * rowp;
        vb = padN + pad_index(g.ny, g.nx, 0, 0, 0);
        o = (iz * g.ny + iy) * rowp + ix;
        ox = X.dir;
        oy = Y.dir * rowp;
        oz = Z.dir * slab;
      }
      float alpha = amin;
      // every step moves at least one axis past a face or reaches amax, and
      // an axis passes at most n + 1 faces: at most nx + ny + nz + 3 steps
      const int max_steps = g.nx + g.ny + g.nz + 3;
      for (int step = 0; alpha < amax && step < max_steps; ++step) {
        const float an = fminf(fminf(nxa, nya), fminf(nza, amax));
        sum = fmaf(ld(vb + o), an - alpha, sum);
        alpha = an;
        if (nxa == an) {
          bx += X.dir;
          o += ox;
          nxa = face_alpha(X, bx);
        }
        if (nya == an) {
          by += Y.dir;
          o += oy;
          nya = face_alpha(Y, by);
        }
        if (nza == an) {
          bz += Z.dir;
          o += oz;
          nza = face_alpha(Z, bz);
        }
      }
      sum *= sqrtf(fmaf(ax_, ax_, fmaf(ay_, ay_, az_ * az_)));
    }
    const size_t o = ((size_t)view * g.nv + r) * g.nu + c;
    if (MODE == 0) {
      st(out + o, sum);
    } else if (MODE == 1) {
      const float res = ld(gin + o) - sum;
      st(out + o, res);
      const float rs = as_stored<T>(res);  // the stored (rounded) residual
      part = (double)rs * (double)rs;
    } else {
      st(out + o, sum);
      const float qs = as_stored<T>(sum);
      part = (double)qs * (double)qs;
    }
  }
  if (MODE != 0) {
    const double s = wave_block_sum(part, red);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

template <typename T>
hipError_t launch_project_siddon(const GeomDev& g, const ViewInfo* views, const T* padN,
                                 const T* padT, int mode, const T* gin, T* out, double* partials,
                                 int* n_partials, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nu + 63) / 64, (g.nv + 3) / 4, g.n_views);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  if (mode == 0)
    hipLaunchKernelGGL((k_project_siddon<T, 0>), grid, block, 0, s, g, views, padN, padT, gin,
                       out, partials);
  else if (mode == 1)
    hipLaunchKernelGGL((k_project_siddon<T, 1>), grid, block, 0, s, g, views, padN, padT, gin,
                       out, partials);
  else
    hipLaunchKernelGGL((k_project_siddon<T, 2>), grid, block, 0, s, g, views, padN, padT, gin,
                       out, partials);
  return hipGetLastError();
}

// Bilinear taps of one detector axis at fractional index f: the two loaded
// pixels q0 = clamp(floor f, 0, n - 2) and q1 = q0 + 1 (both inside the
// detector), weighted by the hat of their distance to f, so a tap that
// falls off the detector gets weight 0.  n = 1: the single pixel.
struct Taps {
  int q0, q1;
  float w0, w1;
};
__device__ __forceinline__ Taps axis_taps(float f, int n) {
  Taps t;
  const int q = (int)floorf(f);
  t.q0 = min(max(q, 0), max(n - 2, 0));
  t.q1 = min(t.q0 + 1, n - 1);
  t.w0 = fmaxf(0.f, 1.f - fabsf(f - (float)t.q0));
  t.w1 = t.q1 != t.q0 ? fmaxf(0.f, 1.f - fabsf(f - (float)(t.q0 + 1))) : 0.f;
  return t;
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_backproject_eq3(GeomDev g, const ViewInfo* __restrict__ views,
                                                         const T* __restrict__ proj,
                                                         T* __restrict__ vol,
                                                         double* __restrict__ partials) {
  __shared__ double red[4];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k0 = blockIdx.z * K;
  const bool active = i < g.nx && j < g.ny;
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.f;
  if (active) {
    const float X = ((float)i - 0.5f * (float)(g.nx - 1)) * g.dx;
    const float Y = ((float)j - 0.5f * (float)(g.ny - 1)) * g.dy;
    const float zc = 0.5f * (float)(g.nz - 1);
    const float cu = 0.5f * (float)(g.nu - 1), cv = 0.5f * (float)(g.nv - 1);
    const float inv_du = 1.f / g.du, inv_dv = 1.f / g.dv;
    const float inv_sdd = 1.f / g.sdd;
    const size_t view_px = (size_t)g.nu * g.nv;
    for (int view = 0; view < g.n_views; ++view) {
      const ViewInfo vi = views[view];
      // distance from the source to the voxel column along the central ray
      const float w = g.sad - fmaf(X, vi.cs, Y * vi.sn);
      if (!(w > 0.f)) continue;
      const float mag = g.sdd / w;
      const float us = mag * fmaf(-X, vi.sn, Y * vi.cs);
      const Taps tc = axis_taps(fmaf(us, inv_du, cu), g.nu);
      const float dxs = X - vi.sx, dys = Y - vi.sy;
      const float l2xy = fmaf(dxs, dxs, dys * dys);
      const float L2xy = fmaf(g.sdd, g.sdd, us * us);
      const T* __restrict__ pv = proj + view * view_px;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const float Zk = ((float)(k0 + q) - zc) * g.dz;
        const float vs = mag * Zk;
        const Taps tr = axis_taps(fmaf(vs, inv_dv, cv), g.nv);
        const T* r0p = pv + (size_t)tr.q0 * g.nu;
        const T* r1p = pv + (size_t)tr.q1 * g.nu;
        const float a = fmaf(tc.w1, ld(r0p + tc.q1), tc.w0 * ld(r0p + tc.q0));
        const float b = fmaf(tc.w1, ld(r1p + tc.q1), tc.w0 * ld(r1p + tc.q0));
        const float gv = fmaf(tr.w1, b, tr.w0 * a);
        const float L2 = fmaf(vs, vs, L2xy), l2 = fmaf(Zk, Zk, l2xy);
        // L^3 / (L0 l^2)
        acc[q] = fmaf(L2 * sqrtf(L2) * inv_sdd / l2, gv, acc[q]);
      }
    }
  }
  const float pref = g.dx * g.dy * g.dz / (g.du * g.dv);
  double part = 0.0;
  if (active) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (k0 + q < g.nz) {
        const size_t o = ((size_t)(k0 + q) * g.ny + j) * g.nx + i;
        st(vol + o, pref * acc[q]);
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

template <typename T>
hipError_t launch_backproject_eq3(const GeomDev& g, const ViewInfo* views, const T* proj, T* vol,
                                  double* partials, int* n_partials, hipStream_t s) {
  dim3 block(256);
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, (g.nz + kEq3Run - 1) / kEq3Run);
  if (n_partials) *n_partials = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL((k_backproject_eq3<T, kEq3Run>), grid, block, 0, s, g, views, proj, vol,
                     partials);
  return hipGetLastError();
}

#define TFCB_INST(T)                                                                              \
  template hipError_t launch_project_siddon<T>(const GeomDev&, const ViewInfo*, const T*, const T*, \
                                               int, const T*, T*, double*, int*, hipStream_t);     \
  template hipError_t launch_backproject_eq3<T>(const GeomDev&, const ViewInfo*, const T*, T*,     \
                                                double*, int*, hipStream_t);
TFCB_INST(float)
TFCB_INST(__half)
TFCB_INST(__hip_bfloat16)
#undef TFCB_INST

}  // namespace tfcb
