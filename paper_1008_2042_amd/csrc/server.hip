// Continuous-batching reconstruction server.
//
// Requests of mixed volume sizes and view counts are submitted at any time;
// each is admitted (FIFO) as soon as a slot is free and its whole workspace
// fits in the caller-owned HBM arena.  An admitted request keeps its entire
// solver state on the device (its own workspace inside the arena) and runs
// on its own stream; every server step enqueues the next outer iteration of
// every active request, so the work of concurrent requests overlaps on the
// GPU while new requests are admitted and finished ones retired.  The CGLS
// step of an iteration (some 25 launches) is captured as a graph per grid
// and iterate buffer the first time it runs and replayed after that; the
// framelet step, whose momentum coefficient changes every iteration, is
// launched directly.  A request runs exactly the kernels and launch shapes
// of tfcb_reconstruct on its own buffers, with deterministic reductions, so
// its result is bitwise the same alone or in any mix.
#include <chrono>
#include <deque>
#include <map>
#include <memory>

#include "driver.h"

struct tfcb_server;

namespace tfcb {
namespace {

double host_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  Arena(char* base, size_t size) : base_(base), size_(size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t next = it->first + n;
        free_.erase(it);
        if (rest) free_[next] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return base_; }
  size_t size() const { return size_; }

 private:
  char* base_;
  size_t size_;
  std::map<size_t, size_t> free_;
};

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_FAILED = 3, RQ_CANCELLED = 4 };

struct Request {
  uint64_t id = 0;
  tfcb_geometry geom{};
  std::vector<double> angles;
  tfcb_options opts{};
  const float* proj = nullptr;
  float* vol = nullptr;
  hipEvent_t ready_ev = nullptr;  // recorded on the producer stream at submit
  int state = RQ_QUEUED;
  tfcb_status result = TFCB_OK;
  size_t need = 0;          // arena bytes the request needs
  size_t off = 0, bytes = 0;  // its arena block while admitted (bytes 0 otherwise)
  Plan plan;
  int slot = -1;
  int grid = -1;  // current grid (0 = finest), -1 before the prologue
  int iter = 0;   // outer iterations done on the current grid
  std::vector<double> mom;
  void *f_cur = nullptr, *f_nxt = nullptr, *xa = nullptr, *xb = nullptr;
  bool enqueued_all = false;
  // the CGLS step of one outer iteration per grid and x buffer (x0 or x1 as
  // the iterate), captured on first use and replayed after that
  hipGraphExec_t cgls_graph[4][2] = {};
  hipEvent_t done_ev = nullptr;
  std::deque<hipEvent_t> inflight;
  double t_done = 0.0;
};

}  // namespace
}  // namespace tfcb

using namespace tfcb;

struct tfcb_server {
  explicit tfcb_server(char* base, size_t n) : arena(base, n) {}
  Arena arena;
  int max_slots = 0;
  std::vector<hipStream_t> streams;
  std::vector<int> slot_busy;
  int* flags = nullptr;  // pinned host: one non-finite flag per slot
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<hipEvent_t> pool;
  uint64_t next_id = 1;
  hipEvent_t ref_ev = nullptr;
  double t_ref = 0.0;
};

namespace tfcb {
namespace {

hipError_t get_event(tfcb_server* S, hipEvent_t* e) {
  if (!S->pool.empty()) {
    *e = S->pool.back();
    S->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreateWithFlags(e, hipEventDefault);
}

template <typename T>
tfcb_status prologue(tfcb_server* S, Request& R) {
  hipStream_t s = S->streams[R.slot];
  const Plan& P = R.plan;
  // the projections are read only after the caller's work that produced them
  TFCB_HIP(hipStreamWaitEvent(s, R.ready_ev, 0));
  TFCB_HIP(launch_cgls_reset(P.sc, s));
  const int ng = R.opts.n_grids;
  for (int l = 0; l < ng; ++l) TFCB_TRY(setup_grid<T>(P.grid[l], s));
  TFCB_HIP((launch_cast<float, T>(npix(R.geom), R.proj, static_cast<T*>(P.grid[0].g), s)));
  for (int l = 1; l < ng; ++l) {
    const GridBufs& f = P.grid[l - 1];
    const GridBufs& c = P.grid[l];
    if (R.opts.bin_coarse_detector)
      TFCB_HIP(launch_restrict(f.geom.n_views, f.geom.nu, f.geom.nv, static_cast<const T*>(f.g),
                               static_cast<T*>(c.g), s));
    else
      TFCB_HIP(launch_copy(npix(c.geom), static_cast<const T*>(f.g), static_cast<T*>(c.g), s));
  }
  return TFCB_OK;
}

// Starts grid l: f = 0 on the coarsest grid, else the prolonged result of
// the coarser grid; v_0 = f_0; t restarts at 1.
template <typename T>
tfcb_status start_grid(tfcb_server* S, Request& R, int l) {
  hipStream_t s = S->streams[R.slot];
  const GridBufs& b = R.plan.grid[l];
  const size_t V = nvox(b.geom);
  void* prev = R.f_cur;
  R.f_cur = b.f0;
  R.f_nxt = b.f1;
  R.xa = b.x0;
  R.xb = b.x1;
  if (l == R.opts.n_grids - 1)
    TFCB_HIP(launch_fill(V, 0.f, static_cast<T*>(R.f_cur), s));
  else
    TFCB_HIP(launch_prolong(R.plan.grid[l + 1].geom, b.geom, static_cast<const T*>(prev),
                            static_cast<T*>(R.f_cur), s));
  TFCB_HIP(launch_copy(V, static_cast<const T*>(R.f_cur), static_cast<T*>(R.xa), s));
  R.grid = l;
  R.iter = 0;
  R.mom = momentum_schedule(R.opts.iters[R.opts.n_grids - 1 - l], R.opts.momentum != 0);
  return TFCB_OK;
}

template <typename T>
tfcb_status finish(tfcb_server* S, Request& R) {
  hipStream_t s = S->streams[R.slot];
  const size_t V = nvox(R.geom);
  TFCB_HIP((launch_cast<T, float>(V, static_cast<const T*>(R.f_cur), R.vol, s)));
  TFCB_HIP(launch_nonfinite(V, (const float*)R.vol, R.plan.flag, s));
  TFCB_HIP(hipMemcpyAsync(&S->flags[R.slot], R.plan.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  TFCB_HIP(get_event(S, &R.done_ev));
  TFCB_HIP(hipEventRecord(R.done_ev, s));
  R.enqueued_all = true;
  return TFCB_OK;
}

// The CGLS step of R's current outer iteration.  Its launches depend only on
// the grid and on which x buffer holds the iterate, so each such pair is
// captured once as a graph (no memset nodes: every fill is a kernel) and
// replayed on every later iteration.
template <typename T>
tfcb_status cgls_step(tfcb_server* S, Request& R, const GridBufs& b, hipStream_t s) {
  hipGraphExec_t& exec = R.cgls_graph[R.grid][R.xa == b.x0 ? 0 : 1];
  if (!exec) {
    TFCB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const tfcb_status st = run_cgls<T>(b, R.plan.sc, static_cast<T*>(R.xa),
                                       static_cast<const T*>(b.g), R.opts.cgls_steps, s);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != TFCB_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    TFCB_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      exec = nullptr;
      return fail(TFCB_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
  }
  TFCB_HIP(hipGraphLaunch(exec, s));
  return TFCB_OK;
}

// Enqueues the next outer iteration of R (and any grid transition).
template <typename T>
tfcb_status advance(tfcb_server* S, Request& R) {
  hipStream_t s = S->streams[R.slot];
  const int ng = R.opts.n_grids;
  if (R.grid < 0) {
    TFCB_TRY(prologue<T>(S, R));
    TFCB_TRY(start_grid<T>(S, R, ng - 1));
  }
  // skip over grids whose iterations are done (including grids with 0)
  while (R.iter >= R.opts.iters[ng - 1 - R.grid]) {
    if (R.grid == 0) return finish<T>(S, R);
    TFCB_TRY(start_grid<T>(S, R, R.grid - 1));
  }
  const GridBufs& b = R.plan.grid[R.grid];
  TFCB_TRY(cgls_step<T>(S, R, b, s));
  TFCB_TRY(run_framelet<T>(b.geom, R.opts.framelet_levels, (float)R.opts.lambda,
                           R.opts.positivity, static_cast<const T*>(R.xa),
                           static_cast<T*>(R.f_nxt), static_cast<const T*>(R.f_cur),
                           static_cast<T*>(R.xb), (float)R.mom[R.iter + 1],
                           static_cast<T*>(b.s), static_cast<T*>(b.t2), s));
  std::swap(R.f_cur, R.f_nxt);
  std::swap(R.xa, R.xb);
  R.iter += 1;
  hipEvent_t e;
  TFCB_HIP(get_event(S, &e));
  TFCB_HIP(hipEventRecord(e, s));
  R.inflight.push_back(e);
  return TFCB_OK;
}

tfcb_status advance_any(tfcb_server* S, Request& R) {
  return dispatch(R.opts.storage, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    return advance<T>(S, R);
  });
}

void release_request(tfcb_server* S, Request& R) {
  for (auto& per_grid : R.cgls_graph)
    for (hipGraphExec_t& e : per_grid)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
  if (R.ready_ev) {
    S->pool.push_back(R.ready_ev);
    R.ready_ev = nullptr;
  }
  for (hipEvent_t e : R.inflight) S->pool.push_back(e);
  R.inflight.clear();
  if (R.done_ev) {
    S->pool.push_back(R.done_ev);
    R.done_ev = nullptr;
  }
  if (R.slot >= 0) {
    S->slot_busy[R.slot] = 0;
    R.slot = -1;
  }
  if (R.bytes) {
    S->arena.release(R.off, R.bytes);
    R.bytes = 0;
  }
}

// Iterations a request may have queued on its stream ahead of the device.
constexpr size_t kMaxInflight = 2;

}  // namespace
}  // namespace tfcb

extern "C" {

tfcb_status tfcb_request_bytes(const tfcb_geometry* g, const tfcb_options* o, size_t* bytes) {
  return tfcb_workspace_size(g, o, bytes);
}

tfcb_status tfcb_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                               tfcb_server** out) {
  if (!out) return fail(TFCB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!arena || reinterpret_cast<uintptr_t>(arena) % 256 != 0)
    return fail(TFCB_EINVAL, "arena must be a 256-byte aligned device pointer");
  if (arena_bytes < 4096) return fail(TFCB_ENOMEM, "arena too small");
  if (max_slots < 1 || max_slots > 64) return fail(TFCB_EINVAL, "max_slots must be 1..64");
  std::unique_ptr<tfcb_server> S(new tfcb_server(static_cast<char*>(arena), arena_bytes));
  S->max_slots = max_slots;
  S->slot_busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st;
    TFCB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    S->streams.push_back(st);
  }
  TFCB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->flags), sizeof(int) * max_slots,
                         hipHostMallocDefault));
  std::memset(S->flags, 0, sizeof(int) * max_slots);
  TFCB_HIP(hipEventCreateWithFlags(&S->ref_ev, hipEventDefault));
  TFCB_HIP(hipEventRecord(S->ref_ev, S->streams[0]));
  TFCB_HIP(hipEventSynchronize(S->ref_ev));
  S->t_ref = host_now();
  *out = S.release();
  return TFCB_OK;
}

tfcb_status tfcb_server_submit(tfcb_server* S, const tfcb_geometry* g, const tfcb_options* o,
                               const float* proj, float* vol, void* stream, uint64_t* id) {
  if (!S || !id) return fail(TFCB_EINVAL, "server or id is NULL");
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_options(o));
  TFCB_TRY(validate_schedule(*g, *o));
  if (o->regulariser != 0)
    return fail(TFCB_EUNSUPPORTED, "the server runs the tight-frame method only (regulariser 0)");
  TFCB_TRY(check_ptr(proj, "proj", sizeof(float)));
  TFCB_TRY(check_ptr(vol, "vol", sizeof(float)));
  std::unique_ptr<Request> R(new Request());
  R->geom = *g;
  if (g->angles) {
    R->angles.assign(g->angles, g->angles + g->n_views);
    R->geom.angles = R->angles.data();
  }
  R->opts = *o;
  R->opts.profile = 0;
  R->proj = proj;
  R->vol = vol;
  Plan P;
  make_plan(R->geom, R->opts, nullptr, P);
  R->need = align_up(P.bytes);
  if (R->need > S->arena.size())
    return fail(TFCB_ENOMEM, "request needs %zu bytes, the arena holds %zu", R->need,
                S->arena.size());
  TFCB_HIP(get_event(S, &R->ready_ev));
  {
    const hipError_t e = hipEventRecord(R->ready_ev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
      S->pool.push_back(R->ready_ev);
      return fail(TFCB_EDEVICE, "hipEventRecord on the producer stream failed: %s",
                  hipGetErrorString(e));
    }
  }
  R->id = S->next_id++;
  *id = R->id;
  S->queue.push_back(R->id);
  S->reqs[R->id] = std::move(R);
  return TFCB_OK;
}

tfcb_status tfcb_server_step(tfcb_server* S, int32_t* n_active, int32_t* n_queued) {
  if (!S) return fail(TFCB_EINVAL, "server is NULL");
  // 1. retire requests whose last kernels have completed
  for (auto& kv : S->reqs) {
    Request& R = *kv.second;
    if (R.state != RQ_RUNNING || !R.enqueued_all) continue;
    hipError_t q = hipEventQuery(R.done_ev);
    if (q == hipErrorNotReady) continue;
    TFCB_HIP(q);
    float ms = 0.f;
    TFCB_HIP(hipEventElapsedTime(&ms, S->ref_ev, R.done_ev));
    R.t_done = S->t_ref + ms * 1e-3;
    const bool bad = S->flags[R.slot] != 0;
    R.state = bad ? RQ_FAILED : RQ_DONE;
    R.result = bad ? TFCB_ENUMERIC : TFCB_OK;
    release_request(S, R);
  }
  // 2. admit queued requests in arrival order while a slot and HBM are free
  while (!S->queue.empty()) {
    int slot = -1;
    for (int i = 0; i < S->max_slots; ++i)
      if (!S->slot_busy[i]) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    Request& R = *S->reqs[S->queue.front()];
    size_t off = 0;
    if (!S->arena.alloc(R.need, &off)) break;
    S->queue.pop_front();
    R.off = off;
    R.bytes = R.need;
    make_plan(R.geom, R.opts, S->arena.base() + off, R.plan);
    R.slot = slot;
    S->slot_busy[slot] = 1;
    S->flags[slot] = 0;
    R.state = RQ_RUNNING;
  }
  // 3. one more outer iteration for every active request not too far ahead
  int active = 0;
  for (auto& kv : S->reqs) {
    Request& R = *kv.second;
    if (R.state != RQ_RUNNING) continue;
    ++active;
    if (R.enqueued_all) continue;
    while (!R.inflight.empty() && hipEventQuery(R.inflight.front()) == hipSuccess) {
      S->pool.push_back(R.inflight.front());
      R.inflight.pop_front();
    }
    if (R.inflight.size() >= kMaxInflight) continue;
    const tfcb_status st = advance_any(S, R);
    if (st != TFCB_OK) {
      (void)hipStreamSynchronize(S->streams[R.slot]);
      R.state = RQ_FAILED;
      R.result = st;
      R.t_done = host_now();
      release_request(S, R);
      --active;
    }
  }
  if (n_active) *n_active = active;
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  return TFCB_OK;
}

tfcb_status tfcb_server_poll(tfcb_server* S, uint64_t id, int32_t* state, double* t_done,
                             tfcb_status* result) {
  if (!S) return fail(TFCB_EINVAL, "server is NULL");
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return fail(TFCB_EINVAL, "unknown request %llu", (unsigned long long)id);
  const Request& R = *it->second;
  if (state) *state = R.state;
  if (t_done) *t_done = R.t_done;
  if (result) *result = R.result;
  return TFCB_OK;
}

tfcb_status tfcb_server_cancel(tfcb_server* S, uint64_t id) {
  if (!S) return fail(TFCB_EINVAL, "server is NULL");
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return fail(TFCB_EINVAL, "unknown request %llu", (unsigned long long)id);
  Request& R = *it->second;
  if (R.state == RQ_QUEUED) {
    for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
      if (*q == id) {
        S->queue.erase(q);
        break;
      }
    release_request(S, R);  // holds only its producer event
  } else if (R.state == RQ_RUNNING) {
    TFCB_HIP(hipStreamSynchronize(S->streams[R.slot]));
    release_request(S, R);
  } else {
    return TFCB_OK;
  }
  R.state = RQ_CANCELLED;
  R.result = TFCB_OK;
  R.t_done = host_now();
  return TFCB_OK;
}

tfcb_status tfcb_server_destroy(tfcb_server* S) {
  if (!S) return TFCB_OK;
  tfcb_status st = TFCB_OK;
  for (hipStream_t s : S->streams)
    if (hipStreamSynchronize(s) != hipSuccess) st = fail(TFCB_EDEVICE, "stream sync failed");
  for (auto& kv : S->reqs) release_request(S, *kv.second);
  for (hipEvent_t e : S->pool) (void)hipEventDestroy(e);
  if (S->ref_ev) (void)hipEventDestroy(S->ref_ev);
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  if (S->flags) (void)hipHostFree(S->flags);
  delete S;
  return st;
}

}  // extern "C"
