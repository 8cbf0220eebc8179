// Internal declarations of the tfcb HIP library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>

#include "../../include/tfcb.h"

namespace tfcb {

// ---------------------------------------------------------------- storage
// Volumes and projections are stored as T; every load widens to FP32 and
// every store rounds to nearest even.
template <typename T> __device__ __forceinline__ float ld(const T* p);
template <> __device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<__half>(const __half* p) { return __half2float(*p); }
template <> __device__ __forceinline__ float ld<__hip_bfloat16>(const __hip_bfloat16* p) {
  return __bfloat162float(*p);
}
template <typename T> __device__ __forceinline__ void st(T* p, float v);
template <> __device__ __forceinline__ void st<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void st<__half>(__half* p, float v) { *p = __float2half(v); }
template <> __device__ __forceinline__ void st<__hip_bfloat16>(__hip_bfloat16* p, float v) {
  *p = __float2bfloat16(v);
}

// st then ld of the same element, without the memory round trip: the value
// as stored (rounded to nearest even for FP16 and BF16)
template <typename T> __device__ __forceinline__ float as_stored(float v);
template <> __device__ __forceinline__ float as_stored<float>(float v) { return v; }
template <> __device__ __forceinline__ float as_stored<__half>(float v) {
  return __half2float(__float2half(v));
}
template <> __device__ __forceinline__ float as_stored<__hip_bfloat16>(float v) {
  return __bfloat162float(__float2bfloat16(v));
}

inline size_t dtype_size(tfcb_dtype dt) { return dt == TFCB_F32 ? 4 : 2; }

// ------------------------------------------------------- padded copies
// The projector reads a volume through zero-padded copies laid out
// [nz + 2 kZPad][ns][pad_row(nt)] (kZPad zero slices below and above in z,
// zero columns after every trans row up to a multiple of 4 elements) behind
// 4 leading zero elements, so every row starts on a 4-element boundary.
// Element (k, p, i) with k in [-kZPad, nz + kZPad), p in [0, ns), i in
// [-4, pad_row(nt) - 1] sits at 4 + ((k + kZPad) ns + p) pad_row(nt) + i.
// A thread that samples several detector rows of one column loads a stack
// of up to kZPad + 1 consecutive slices per plane; the pads make every such
// stack of a plane where any of its rows is inside the volume lie inside the
// buffer, and the taps that fall off the grid read exact zeros: no compares
// in the loop.  "native" copy: ns = ny, nt = nx (y-stepping views);
// "transposed" copy: ns = nx, nt = ny (x-stepping views).  Only the interior
// is ever written; the pads are cleared once per call.
constexpr int kZPad = 6;
constexpr int kPadLead = 4;
__host__ __device__ __forceinline__ int pad_row(int nt) { return (nt + 1 + 3) & ~3; }
inline size_t pad_elems(int ns, int nt, int nz) {
  return kPadLead + (size_t)(nz + 2 * kZPad) * (size_t)ns * (size_t)pad_row(nt);
}
inline size_t pad_elems_vol(int nx, int ny, int nz) {
  // the larger of the two copies' sizes
  const size_t a = pad_elems(ny, nx, nz), b = pad_elems(nx, ny, nz);
  return a > b ? a : b;
}
__host__ __device__ __forceinline__ int pad_index(int ns, int nt, int k, int p, int i) {
  return kPadLead + ((k + kZPad) * ns + p) * pad_row(nt) + i;
}

// ------------------------------------------------------------- geometry
// A view is processed in its own frame: "step" is the axis whose voxel-centre
// planes the rays cross (x or y), "trans" the other in-plane axis.  For
// step = y the native volume [z][y][x] is read; for step = x a copy laid out
// [z][x][y] is read, so in both cases the trans index is the fastest one and
// a wavefront of adjacent detector columns reads adjacent addresses.
struct ViewInfo {
  int32_t step_x;      // 1: planes x = const (reads the [z][x][y] copy)
  int32_t pad;
  float cs, sn;        // cos, sin of the view angle
  float sx, sy;        // source position (mm)
  float pad2[2];
};

// Per (view, detector column): everything a ray needs that does not depend
// on the detector row.  Plane p of the stepping axis is crossed at ray
// parameter tau_p = tau0 + p * dtau (0 < tau_p < 1 for p_lo <= p <= p_hi),
// at fractional trans index t_p = t0 + p * dt.  The fractional z index of
// row r is tau_p * vz_r + (nz - 1) / 2 with vz_r = (r - (nv-1)/2) dv / dz.
// The path length between planes is l = d_step * sqrt(a2 + v_r^2) * inv_astep.
struct alignas(16) ColInfo {
  float t0, dt;
  float tau0, dtau;
  float a2, inv_astep;
  int32_t p_lo, p_hi;
};
static_assert(sizeof(ColInfo) == 32, "ColInfo is read as two 16-byte vectors");

struct GeomDev {
  int32_t nx, ny, nz, nu, nv, n_views;
  float dx, dy, dz, du, dv, sad, sdd;
  float dvdz;  // dv / dz
};

inline GeomDev make_geom_dev(const tfcb_geometry& g) {
  GeomDev d;
  d.nx = g.nx; d.ny = g.ny; d.nz = g.nz; d.nu = g.nu; d.nv = g.nv; d.n_views = g.n_views;
  d.dx = (float)g.dx; d.dy = (float)g.dy; d.dz = (float)g.dz;
  d.du = (float)g.du; d.dv = (float)g.dv;
  d.sad = (float)g.sad; d.sdd = (float)g.sdd;
  d.dvdz = (float)(g.dv / g.dz);
  return d;
}

// ------------------------------------------------------- device scalars
// CGLS state kept on the device so no iteration needs a host round trip.
//
// The search direction is stored normalised, pn = p / sigma with sigma the
// rms of the latest s = P^T r, so P pn stays O(planes) whatever the scale of
// the data (FP16 storage would otherwise overflow).  CGLS is invariant to
// that scaling: with qn = P pn, alpha p = (gamma / (sigma ||qn||^2)) pn and
// alpha q = the same factor times qn, and the next direction is
// pn' = (s' + beta sigma pn) / sigma'.
struct CglsScalars {
  double gamma;      // ||s||^2 of the current direction
  double delta;      // ||q||^2 = sigma^2 ||qn||^2
  double sigma;      // scale of the stored direction
  double alpha;      // step applied to pn and qn: gamma / (sigma ||qn||^2)
  double beta_sigma; // beta * sigma, the weight of the old pn in the new one
  double inv_sigma;  // 1 / sigma of the new direction
  double resid2;     // latest ||r||^2
  int32_t stopped;     // breakdown guard fired in this CGLS call
  int32_t breakdowns;  // number of CGLS calls stopped so far
};

constexpr int kReduceThreads = 1024;

// Deterministic block sum of one FP64 value per thread (blockDim a multiple
// of 64): wavefront butterfly, then the wave sums in order by thread 0.
// The result is valid in thread 0 only.
__device__ __forceinline__ double wave_block_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += lds[w];
  return r;
}

__device__ __forceinline__ float ray_length(const GeomDev& g, const ViewInfo& vi,
                                            const ColInfo& ci, int r) {
  const float vr = ((float)r - 0.5f * (float)(g.nv - 1)) * g.dv;
  const float ds = vi.step_x ? g.dx : g.dy;
  return ds * sqrtf(ci.a2 + vr * vr) * ci.inv_astep;
}



// ------------------------------------------------------------ launchers
// All return hipGetLastError() of the launch.
// Per-view and per-column tables of g; the view angles (g.angles, a host
// array, or NULL for 2 pi k / n_views) are passed by value in the launches'
// arguments, so the host array may be released as soon as this returns.
hipError_t launch_geom_tables(const tfcb_geometry& g, ViewInfo* views, ColInfo* cols,
                              hipStream_t s);

// P of a volume given as its two zero-padded copies (padN native, padT
// transposed).  mode 0: out = P vol.  mode 1: r = g - P vol, rl = l * r,
// partial ||r||^2.  mode 2: out = P vol, partial ||out||^2.
template <typename T>
hipError_t launch_project(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                          const T* padN, const T* padT, int mode, const T* gin, T* out, T* rl,
                          double* partials, int* n_partials, hipStream_t s);
// Interior of both padded copies from a native [z][y][x] volume.
template <typename T>
hipError_t launch_pad_copies(int nx, int ny, int nz, const T* in, T* padN, T* padT,
                             hipStream_t s);
int project_num_blocks(const GeomDev& g);

// P^T of the length-prescaled projections rl (= l * g).  Writes vol and,
// when partials != nullptr, per-block partial sums of vol^2.
template <typename T>
hipError_t launch_backproject(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                              const T* rl, T* vol, double* partials, int* n_partials,
                              hipStream_t s);
int backproject_num_blocks(const GeomDev& g);

// The paper's operator pair.  Siddon P of the volume given as its two
// padded copies, modes as launch_project (mode 1 writes no rl).  Eq. (3)
// backprojection of plain projections (no length prescale); partials as
// launch_backproject, on the same grid (backproject_num_blocks).
template <typename T>
hipError_t launch_project_siddon(const GeomDev& g, const ViewInfo* views, const T* padN,
                                 const T* padT, int mode, const T* gin, T* out, double* partials,
                                 int* n_partials, hipStream_t s);
template <typename T>
hipError_t launch_backproject_eq3(const GeomDev& g, const ViewInfo* views, const T* proj, T* vol,
                                  double* partials, int* n_partials, hipStream_t s);

// rl = l * g for every ray (prescale before P^T).
template <typename T>
hipError_t launch_prescale(const GeomDev& g, const ColInfo* cols, const ViewInfo* views,
                           const T* in, T* out, hipStream_t s);

// out[z][x][y] = in[z][y][x].
template <typename T>
hipError_t launch_transpose_xy(int nx, int ny, int nz, const T* in, T* out, hipStream_t s);

// Framelet: out = H(W^T T_lambda W in) for one level with dilation dil;
// when low != nullptr the low band of W in is replaced by low (2-level use).
// Epilogue: fnew = (positivity ? max(v,0) : v); when vnext != nullptr also
// vnext = fnew + mom * (fnew - fcur).
template <typename T>
hipError_t launch_framelet(int nx, int ny, int nz, int dil, float lambda, int positivity,
                           const T* in, const T* low, T* out, const T* fcur, T* vnext, float mom,
                           hipStream_t s);
// low = A0^3 in (the level-1 low band, reflect edges, dilation 1).
template <typename T>
hipError_t launch_lowpass(int nx, int ny, int nz, const T* in, T* low, hipStream_t s);

// CGLS vector kernels.
enum FinalizeMode { FIN_GAMMA_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RESID = 3 };
// nvox: voxel count of the grid (sigma = sqrt(gamma / nvox)).
hipError_t launch_finalize(const double* partials, int n, int mode, CglsScalars* sc,
                           double nvox, hipStream_t s);
template <typename T>
hipError_t launch_residual_update(const GeomDev& g, const ViewInfo* views, const ColInfo* cols,
                                  T* r, const T* q, T* rl, const CglsScalars* sc,
                                  double* partials, int* n_partials, hipStream_t s);
// Normalised direction pn (see CglsScalars), kept only as its two padded
// copies pN (native) and pT (transposed).  mode 0: pn = s / sigma.
// mode 1: x += alpha pn; pn = (s + beta_sigma pn) / sigma'.  mode 2:
// x += alpha pn only.
template <typename T>
hipError_t launch_xp_update(int nx, int ny, int nz, int mode, T* x, T* pN, T* pT, const T* s,
                            const CglsScalars* sc, hipStream_t s_);
hipError_t launch_cgls_reset(CglsScalars* sc, hipStream_t s);

// Element-wise helpers.
template <typename T>
hipError_t launch_copy(size_t n, const T* in, T* out, hipStream_t s);
template <typename T>
hipError_t launch_fill(size_t n, float v, T* out, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_cast(size_t n, const Tin* in, Tout* out, hipStream_t s);
// flag[0] = 1 if any element is non-finite (flag must be zeroed first).
template <typename T>
hipError_t launch_nonfinite(size_t n, const T* in, int* flag, hipStream_t s);

// The ROF sub-problem of the TV comparison method (section 2.3): f from
// x by gradient descent with an adaptive step (see tv.hip), then H when
// positivity is set.  g: float volume scratch; state: rof_state_bytes();
// partials: rof_num_partials() doubles.  Synchronises `s` between chunks
// of attempts to read the stop flag; *steps_host = accepted steps.
template <typename T>
hipError_t launch_rof(int nx, int ny, int nz, float mu, float eps, double tol, int max_steps,
                      int positivity, const T* x, T* f, float* g, void* state, double* partials,
                      int* steps_host, hipStream_t s);
int rof_num_partials(int nx, int ny, int nz);
size_t rof_state_bytes();

// FDK (the comparison baseline): q = cosine-weighted, Ram-Lak-filtered
// projections (FP32 scratch, n_views * nv * nu), then the weighted
// backprojection into vol.  Needs nu <= 8192 (fdk_supported) and equally
// spaced views (the tables of views hold their angles).
template <typename T>
hipError_t launch_fdk(const GeomDev& g, const ViewInfo* views, const T* proj, float* q, T* vol,
                      hipStream_t s);
bool fdk_supported(int nu);

// Multigrid.
template <typename T>
hipError_t launch_restrict(int n_views, int nu, int nv, const T* in, T* out, hipStream_t s);
template <typename T>
hipError_t launch_prolong(const tfcb_geometry& co, const tfcb_geometry& fi, const T* in, T* out,
                          hipStream_t s);

}  // namespace tfcb
