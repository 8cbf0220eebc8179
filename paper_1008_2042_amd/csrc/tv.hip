// The TV comparison method (section 2.3): after the CGLS step, the ROF
// sub-problem argmin_f ||f - x||^2 + mu TV(f) is solved by gradient descent
// with an adaptive step, then positivity.  TV(f) is the l1 norm of the
// gradient, with forward differences in index units, each |d| smoothed to
// sqrt(d^2 + eps^2) so that the energy is differentiable.
//
// Every step of the descent runs on the device with its scalars in FP64:
// the gradient (k_tv_grad), the energy of the trial point f - s grad
// (k_tv_trial, per-block FP64 partial sums), the decision (k_tv_decide, one
// block: accept and double s up to 1/2, or halve s and retry; stop below the
// relative decrease tol or at the step cap) and the update (k_tv_apply).
// Once the state says stopped, every kernel returns at once, so the host
// enqueues attempts in chunks and reads the flag back only between chunks.
// The kernels are stencils bound by HBM and L2: 64 x 4 threads per block
// over x and y of one z slice, coalesced along x.
#include "tfcb_internal.h"

namespace tfcb {

struct RofState {
  double E;       // energy of the current f
  double s;       // step of the next trial
  double s_used;  // step of the accepted trial (for k_tv_apply)
  int32_t accepted;   // the last decision accepted its trial
  int32_t need_grad;  // f changed since the gradient was taken
  int32_t stopped;
  int32_t steps;      // accepted steps
  int32_t halvings;   // consecutive rejected trials
  int32_t phase;      // 0: the next decision records E(f) (s = 0 trial)
};

struct TvParams {
  int nx, ny, nz;
  float mu, e2;  // mu_TV, eps^2
};

// d / sqrt(d^2 + eps^2), the derivative of the smoothed |d|
__device__ __forceinline__ float tv_psi(float d, float e2) { return d * rsqrtf(fmaf(d, d, e2)); }

template <typename T>
__global__ __launch_bounds__(256) void k_tv_grad(TvParams p, const T* __restrict__ x,
                                                 const T* __restrict__ f,
                                                 float* __restrict__ g,
                                                 const RofState* __restrict__ st) {
  if (st->stopped || !st->need_grad) return;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= p.nx || j >= p.ny) return;
  const size_t sy = p.nx, sz = (size_t)p.nx * p.ny;
  const size_t q = k * sz + j * sy + i;
  const float fq = ld(f + q);
  float t = 0.f;
  if (i + 1 < p.nx) t -= tv_psi(ld(f + q + 1) - fq, p.e2);
  if (i > 0) t += tv_psi(fq - ld(f + q - 1), p.e2);
  if (j + 1 < p.ny) t -= tv_psi(ld(f + q + sy) - fq, p.e2);
  if (j > 0) t += tv_psi(fq - ld(f + q - sy), p.e2);
  if (k + 1 < p.nz) t -= tv_psi(ld(f + q + sz) - fq, p.e2);
  if (k > 0) t += tv_psi(fq - ld(f + q - sz), p.e2);
  g[q] = fmaf(p.mu, t, 2.f * (fq - ld(x + q)));
}

// The trial point's value at q: f - s g, evaluated exactly as k_tv_apply
// stores it (the starting point's energy reads f alone: no gradient yet).
template <typename T>
__device__ __forceinline__ float trial_value(const T* __restrict__ f, const float* __restrict__ g,
                                             size_t q, float s, bool start = false) {
  return start ? ld(f + q) : fmaf(-s, g[q], ld(f + q));
}

template <typename T>
__global__ __launch_bounds__(256) void k_tv_trial(TvParams p, const T* __restrict__ x,
                                                  const T* __restrict__ f,
                                                  const float* __restrict__ g,
                                                  const RofState* __restrict__ st,
                                                  double* __restrict__ partials) {
  __shared__ double red[4];
  if (st->stopped) return;
  const bool start = st->phase == 0;
  const float s = (float)st->s;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  double e = 0.0;
  if (i < p.nx && j < p.ny) {
    const size_t sy = p.nx, sz = (size_t)p.nx * p.ny;
    const size_t q = k * sz + j * sy + i;
    const float fq = trial_value(f, g, q, s, start);
    const float r = fq - ld(x + q);
    float tv = 0.f;
    if (i + 1 < p.nx) {
      const float d = trial_value(f, g, q + 1, s, start) - fq;
      tv += sqrtf(fmaf(d, d, p.e2));
    }
    if (j + 1 < p.ny) {
      const float d = trial_value(f, g, q + sy, s, start) - fq;
      tv += sqrtf(fmaf(d, d, p.e2));
    }
    if (k + 1 < p.nz) {
      const float d = trial_value(f, g, q + sz, s, start) - fq;
      tv += sqrtf(fmaf(d, d, p.e2));
    }
    e = (double)r * (double)r + (double)p.mu * (double)tv;
  }
  const double sum = wave_block_sum(e, red);
  if (threadIdx.x == 0)
    partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = sum;
}

__global__ __launch_bounds__(kReduceThreads) void k_tv_decide(const double* __restrict__ partials,
                                                              int n, double tol, int max_steps,
                                                              RofState* __restrict__ st) {
  __shared__ double red[kReduceThreads / 64];
  if (st->stopped) {
    // attempts enqueued after the stop: nothing to apply
    if (threadIdx.x == 0) st->accepted = 0;
    return;
  }
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
  const double Et = wave_block_sum((v0 + v1) + (v2 + v3), red);
  if (threadIdx.x != 0) return;
  if (st->phase == 0) {
    // the energy of the starting point f = x
    st->E = Et;
    st->s = 0.5;
    st->phase = 1;
    st->accepted = 0;
    st->need_grad = 1;
    st->stopped = !(Et > 0.0) || max_steps <= 0;
    return;
  }
  if (Et < st->E) {
    const double rel = (st->E - Et) / st->E;
    st->E = Et;
    st->s_used = st->s;
    st->s = fmin(2.0 * st->s, 0.5);
    st->accepted = 1;
    st->need_grad = 1;
    st->halvings = 0;
    st->steps += 1;
    st->stopped = rel < tol || st->steps >= max_steps;
  } else {
    st->accepted = 0;
    st->need_grad = 0;
    st->s *= 0.5;
    st->halvings += 1;
    if (st->halvings > 40) st->stopped = 1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tv_apply(TvParams p, T* __restrict__ f,
                                                  const float* __restrict__ g,
                                                  const RofState* __restrict__ rs) {
  // an accepted trial is applied even by the decision that set stopped
  if (!rs->accepted) return;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= p.nx || j >= p.ny) return;
  const size_t q = (size_t)k * p.nx * p.ny + (size_t)j * p.nx + i;
  st(f + q, trial_value(f, g, q, (float)rs->s_used));
}

__global__ void k_tv_reset(RofState* st) {
  if (threadIdx.x == 0) {
    st->E = 0.0;
    st->s = 0.0;
    st->s_used = 0.0;
    st->accepted = 0;
    st->need_grad = 1;
    st->stopped = 0;
    st->steps = 0;
    st->halvings = 0;
    st->phase = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_nonneg(size_t n, T* __restrict__ f) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const float v = ld(f + i);
    if (v < 0.f) st(f + i, 0.f);
  }
}

static dim3 tv_grid(int nx, int ny, int nz) { return dim3((nx + 63) / 64, (ny + 3) / 4, nz); }

// Two pinned host copies of the descent state per host thread (the stop
// flag read back between chunks), allocated on first use and kept for the
// life of the process.
static hipError_t rof_pinned_state(RofState** out) {
  static thread_local RofState* pinned = nullptr;
  if (!pinned) {
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, 2 * sizeof(RofState), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    pinned = static_cast<RofState*>(p);
  }
  *out = pinned;
  return hipSuccess;
}

int rof_num_partials(int nx, int ny, int nz) {
  const dim3 gr = tv_grid(nx, ny, nz);
  return (int)(gr.x * gr.y * gr.z);
}

size_t rof_state_bytes() { return sizeof(RofState); }

// One ROF attempt: gradient (if f moved), trial energy, decision, update.
template <typename T>
static hipError_t rof_attempt(const TvParams& p, const T* x, T* f, float* g, RofState* st,
                              double* partials, double tol, int max_steps, hipStream_t s) {
  const dim3 gr = tv_grid(p.nx, p.ny, p.nz);
  const int np = (int)(gr.x * gr.y * gr.z);
  hipLaunchKernelGGL((k_tv_grad<T>), gr, dim3(256), 0, s, p, x, (const T*)f, g,
                     (const RofState*)st);
  hipLaunchKernelGGL((k_tv_trial<T>), gr, dim3(256), 0, s, p, x, (const T*)f, (const float*)g,
                     (const RofState*)st, partials);
  hipLaunchKernelGGL(k_tv_decide, dim3(1), dim3(kReduceThreads), 0, s, (const double*)partials,
                     np, tol, max_steps, st);
  hipLaunchKernelGGL((k_tv_apply<T>), gr, dim3(256), 0, s, p, f, (const float*)g,
                     (const RofState*)st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rof(int nx, int ny, int nz, float mu, float eps, double tol, int max_steps,
                      int positivity, const T* x, T* f, float* g, void* state, double* partials,
                      int* steps_host, hipStream_t s) {
  TvParams p{nx, ny, nz, mu, eps * eps};
  RofState* st = static_cast<RofState*>(state);
  const size_t V = (size_t)nx * ny * nz;
  hipError_t e;
  if ((e = launch_copy(V, x, f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tv_reset, dim3(1), dim3(64), 0, s, st);
  // phase 0: the energy of f = x
  const dim3 gr = tv_grid(nx, ny, nz);
  const int np = (int)(gr.x * gr.y * gr.z);
  hipLaunchKernelGGL((k_tv_trial<T>), gr, dim3(256), 0, s, p, x, (const T*)f, (const float*)g,
                     (const RofState*)st, partials);
  hipLaunchKernelGGL(k_tv_decide, dim3(1), dim3(kReduceThreads), 0, s, (const double*)partials,
                     np, tol, max_steps, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Attempts in chunks, two chunks in flight: after enqueueing chunk c the
  // host waits for chunk c - 1 and reads the state it copied to pinned host
  // memory, so the device never idles on the host's decision; the chunk
  // enqueued past the stop only runs kernels that return at once.
  constexpr int kChunk = 4;
  const int max_attempts = max_steps * 42 + 1;  // each step: at most 41 trials
  RofState* pinned = nullptr;
  if ((e = rof_pinned_state(&pinned)) != hipSuccess) return e;
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (int b = 0; b < 2; ++b)
    if ((e = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming)) != hipSuccess) return e;
  int last = -1;
  RofState host{};
  for (int c = 0; c * kChunk < max_attempts; ++c) {
    for (int a = 0; a < kChunk; ++a)
      if ((e = rof_attempt<T>(p, x, f, g, st, partials, tol, max_steps, s)) != hipSuccess)
        break;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&pinned[c & 1], st, sizeof(RofState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(ev[c & 1], s);
    if (e != hipSuccess) break;
    last = c;
    if (c > 0) {
      if ((e = hipEventSynchronize(ev[(c - 1) & 1])) != hipSuccess) break;
      host = pinned[(c - 1) & 1];
      if (host.stopped) break;
    }
  }
  // the newest chunk's copy is still in flight: wait for it before the
  // pinned words are reused
  if (e == hipSuccess && last >= 0) {
    e = hipEventSynchronize(ev[last & 1]);
    if (e == hipSuccess) host = pinned[last & 1];
  }
  for (int b = 0; b < 2; ++b) (void)hipEventDestroy(ev[b]);
  if (e != hipSuccess) return e;
  if (steps_host) *steps_host = host.steps;
  if (positivity) {
    hipLaunchKernelGGL((k_nonneg<T>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, V, f);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

#define TFCB_INST_ROF(T)                                                                    \
  template hipError_t launch_rof<T>(int, int, int, float, float, double, int, int, const T*, \
                                    T*, float*, void*, double*, int*, hipStream_t);
TFCB_INST_ROF(float)
TFCB_INST_ROF(__half)
TFCB_INST_ROF(__hip_bfloat16)

}  // namespace tfcb
