/* tfcb.h — tight-frame regularised cone-beam CT reconstruction on MI355X.
 *
 * C-ABI of the HIP library libtfcb.so (gfx950).  The method is the TF
 * iteration of Jia, Dong, Lou & Jiang, "GPU-based Iterative Cone Beam CT
 * Reconstruction Using Tight Frame Regularization" (arXiv 1008.2042):
 * Algorithm A2 of section 2.1 (CGLS data step of Appendix 1, framelet
 * shrinkage of Eq. (2), positivity) inside the multigrid schedule of
 * section 2.2.3.
 *
 * General rules
 *  - Every function returns a tfcb_status; nothing throws or aborts across
 *    the ABI.  On failure tfcb_last_error() returns a thread-local detail
 *    string (valid until the next call on the same thread).
 *  - All arguments are validated before any work is enqueued.  A call that
 *    returns an error has enqueued nothing, unless it is TFCB_EDEVICE.
 *  - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *    data_ptr()); `stream` is a hipStream_t passed as void* (NULL = the
 *    null stream).  The library never allocates or frees device memory: the
 *    caller owns every buffer, including the workspace, which must be
 *    256-byte aligned and at least the size the matching *_workspace_size
 *    function reports.  Volume and projection buffers need only be aligned
 *    to their element size (4 bytes for FP32, 2 for FP16/BF16).  Caller
 *    pointers are not kept after a call returns.
 *  - Operator calls (project, backproject, framelet_shrink, restrict,
 *    prolong) are asynchronous on `stream`: they never synchronise it, and
 *    a host angle array is read before the call returns.  tfcb_cgls
 *    synchronises `stream` only when stats is non-NULL; tfcb_reconstruct
 *    synchronises `stream` before it returns.
 *  - Calls are reentrant when they use distinct workspaces and streams.
 *  - Geometry conventions (the paper leaves them open): source at
 *    (SAD cos t, SAD sin t, 0); flat detector through
 *    -(SDD - SAD)(cos t, sin t, 0) with u along (-sin t, cos t, 0) and v
 *    along +z; detector values are point samples at pixel centres
 *    u_c = (c - (nu-1)/2) du, v_r = (r - (nv-1)/2) dv; voxel centres
 *    x_i = (i - (nx-1)/2) dx (likewise y, z), so both grids are centred on
 *    the rotation axis.  Units: mm and radians.
 *  - Layouts: volume [nz][ny][nx] (x fastest); projections
 *    [n_views][nv][nu] (u fastest), post-log line integrals.
 */
#ifndef TFCB_H
#define TFCB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tfcb_status;
#define TFCB_OK 0
#define TFCB_EINVAL (-1)       /* bad argument (size, pointer, alignment, value) */
#define TFCB_ENOMEM (-2)       /* workspace or arena too small */
#define TFCB_EDEVICE (-3)      /* HIP runtime error; detail in tfcb_last_error */
#define TFCB_EUNSUPPORTED (-4) /* valid request this build does not handle */
#define TFCB_ENUMERIC (-5)     /* non-finite values in the result */
#define TFCB_EBUSY (-6)        /* resource in use */

typedef int32_t tfcb_dtype;
#define TFCB_F32 0  /* IEEE binary32 */
#define TFCB_F16 1  /* IEEE binary16, round-to-nearest-even on store */
#define TFCB_BF16 2 /* bfloat16, round-to-nearest-even on store */

/* Scan geometry (section 3: circular orbit, flat imager; Eq. (1)). */
typedef struct {
  int32_t nx, ny, nz;    /* volume voxels, each >= 1 */
  double dx, dy, dz;     /* voxel size (mm), > 0 */
  int32_t nu, nv;        /* detector pixels, each >= 1 */
  double du, dv;         /* pixel pitch (mm), > 0 */
  double sad, sdd;       /* source-axis and source-detector distances (mm) */
  int32_t n_views;       /* >= 1 */
  const double* angles;  /* HOST array of n_views view angles (rad), read
                            during the call only; NULL => 2 pi k / n_views */
} tfcb_geometry;

/* Reconstruction options (Algorithm A2 and section 2.2.3). */
typedef struct {
  double lambda;            /* shrink threshold (the paper's mu), >= 0, 1/mm */
  int32_t n_grids;          /* multigrid levels, 1..4; grid l+1 halves every
                               axis of grid l (ceil) and doubles the voxel */
  int32_t iters[4];         /* outer iterations per grid, coarsest first, >= 0 */
  int32_t cgls_steps;       /* CGLS products q = P p per outer iteration, 1..64 */
  int32_t framelet_levels;  /* 1 (the paper) or 2 */
  int32_t momentum;         /* 1 = Algorithm A2, 0 = Algorithm A1 */
  int32_t positivity;       /* 1 = apply H (negative voxels set to 0) */
  int32_t bin_coarse_detector; /* 1 = 2x2 detector binning (mean) per coarser grid */
  tfcb_dtype storage;       /* internal storage of volumes and projections;
                               arithmetic is FP32, reductions FP64 */
  int32_t profile;          /* 1 = time every P, P^T and framelet launch with
                               HIP events on `stream` (fills kernel_ms) */
  int32_t op_pair;          /* operators of the CGLS step: 0 = Joseph P with its
                               exact transpose (tfcb_project / tfcb_backproject);
                               1 = the paper's pair, Siddon P with the Eq. (3)
                               backprojection in place of P^T
                               (tfcb_project_siddon / tfcb_backproject_eq3) */
  int32_t regulariser;      /* step 2 of the outer iteration: 0 = the tight-frame
                               shrinkage (Algorithms A1/A2); 1 = the TV
                               comparison method of section 2.3: x = CGLS(f),
                               f = H(ROF(x)) with lambda as mu_TV (momentum and
                               framelet_levels unused); see tfcb_rof */
  double tv_eps;            /* TV: smoothing of |d|, > 0 (1/mm) */
  double tv_tol;            /* TV: stop the ROF descent at a relative energy
                               decrease below this (the paper's 0.1 %: 1e-3) */
  int32_t tv_max_steps;     /* TV: cap on accepted ROF steps, 0..100000 */
} tfcb_options;

typedef struct {
  double seconds_total;        /* device time of the whole schedule */
  double seconds_per_grid[4];  /* coarsest first */
  int32_t iters_done[4];
  double resid2_last;          /* ||g - P x||^2 after the last CGLS update (FP64) */
  int32_t cgls_breakdowns;     /* CGLS calls stopped by the 1e-300 guard */
  /* with options.profile: summed event-timed durations (ms) and launch
   * counts per kernel class, finest grid only: [0] P, [1] P^T, [2] framelet
   * regulariser; [3] the rest of the finest grid's time (vector updates,
   * transposes, reductions), launch count 0 */
  double kernel_ms[4];
  int32_t kernel_launches[4];
  int32_t rof_steps;           /* TV: accepted ROF steps over the schedule */
} tfcb_report;

const char* tfcb_status_str(tfcb_status s);
const char* tfcb_last_error(void);
/* Library version string, e.g. "tfcb 0.1 gfx950". */
const char* tfcb_version(void);

/* ---------------------------------------------------------------- sizes */
/* Workspace bytes for tfcb_reconstruct and tfcb_cgls with these options. */
tfcb_status tfcb_workspace_size(const tfcb_geometry* g, const tfcb_options* o, size_t* bytes);
/* Workspace bytes for tfcb_project / tfcb_backproject with storage dt. */
tfcb_status tfcb_operator_workspace_size(const tfcb_geometry* g, tfcb_dtype dt, size_t* bytes);
/* Workspace bytes for tfcb_framelet_shrink (0 for one level). */
tfcb_status tfcb_framelet_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t levels,
                                         tfcb_dtype dt, size_t* bytes);

/* ------------------------------------------------------------ operators */
/* proj = P vol: the line integral of Eq. (1) (section 2.1) discretised by
 * Joseph's method: one stepping axis per view (x when |cos t| >= |sin t| -
 * 1e-12, else y); on every voxel-centre plane of that axis the ray crosses at
 * source-to-pixel parameter 0 < tau < 1, the volume is interpolated
 * bilinearly in the other two axes (zero outside the grid); the sum is scaled
 * by the path length between planes.  vol, proj: device, storage dt. */
tfcb_status tfcb_project(const tfcb_geometry* g, tfcb_dtype dt, const void* vol, void* proj,
                         void* ws, size_t ws_bytes, void* stream);

/* vol = P^T proj: the exact transpose of tfcb_project (the adjoint of
 * Appendix 2, Eq. (A1); Eq. (3) is its continuous limit), evaluated voxel by
 * voxel as a gather, without atomics.  proj, vol: device, storage dt. */
tfcb_status tfcb_backproject(const tfcb_geometry* g, tfcb_dtype dt, const void* proj, void* vol,
                             void* ws, size_t ws_bytes, void* stream);

/* proj = P vol by Siddon's ray tracing (section 2.2.1), the paper's
 * projector: voxels are boxes of size dx dy dz around the voxel centres
 * (half-open along each axis, so a ray lying on a face between two voxels
 * counts in the upper one); each ray sums the voxel values times the length
 * of its source-to-pixel segment inside each box.  vol, proj: device,
 * storage dt.  ws: as for tfcb_project. */
tfcb_status tfcb_project_siddon(const tfcb_geometry* g, tfcb_dtype dt, const void* vol,
                                void* proj, void* ws, size_t ws_bytes, void* stream);

/* vol = the closed-form backprojection of Eq. (3) (section 2.2.2, Appendix
 * 2): per voxel centre x and view, dx dy dz / (du dv) L^3 / (SDD l^2) times
 * proj bilinearly interpolated where the ray from the source through x meets
 * the detector (pixel-centre samples; taps off the detector read zero);
 * L = source-to-hit distance, l = source-to-voxel distance.  Not the
 * transpose of either projector (the paper reports under 1 % adjoint
 * mismatch against ray tracing).  proj, vol: device, storage dt.  ws: as for
 * tfcb_backproject. */
tfcb_status tfcb_backproject_eq3(const tfcb_geometry* g, tfcb_dtype dt, const void* proj,
                                 void* vol, void* ws, size_t ws_bytes, void* stream);

/* vol = P^T proj exactly as tfcb_backproject computes it (same kernels, same
 * result bit for bit), for callers that cannot allocate device memory: code
 * under stream capture, tight serving loops, hosts that forbid hipMalloc.
 * Instead of a workspace it uses a static device array of
 * TFCB_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the call allocates nothing (no hipMalloc, hipFree
 * or allocating library routine).  The geometry's scratch need (32 B per
 * view, 32 B per detector column and view, one stored element per
 * projection pixel, each rounded up to 256 B) must fit: larger geometries
 * return TFCB_EUNSUPPORTED with nothing enqueued (the 512x512x70 workload's
 * 40 x 384 x 512 projections need 32.1 MB in FP32).  Every call on one GPU
 * shares that GPU's array: calls whose work overlaps on the device (on
 * different streams, or from different threads) race and give undefined
 * results; calls on one stream are ordered and safe.  proj, vol: device,
 * storage dt; asynchronous on `stream`. */
#define TFCB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tfcb_status tfcb_backproject_noalloc(const tfcb_geometry* g, tfcb_dtype dt, const void* proj,
                                     void* vol, void* stream);

/* out = H(W^T T_lambda W in) (section 2.1: the 27-band piecewise-linear
 * tight frame, the vector shrinkage of Eq. (2), positivity H when
 * positivity = 1).  W is convolution with half-sample symmetric extension and
 * W^T its exact adjoint (W^T W = I).  levels = 2 applies the same frame with
 * filters dilated by 2 to the level-1 low band, each level shrunk on its own
 * 26 high bands.  in, out: device [nz][ny][nx], storage dt, must not alias.
 * ws: device workspace (levels = 2 only; may be NULL for levels = 1). */
tfcb_status tfcb_framelet_shrink(int32_t nx, int32_t ny, int32_t nz, int32_t levels,
                                 double lambda, int32_t positivity, tfcb_dtype dt,
                                 const void* in, void* out, void* ws, size_t ws_bytes,
                                 void* stream);

/* FDK, the filtered-backprojection baseline the paper compares against
 * (section 3; the paper gives no details, this is the textbook
 * Feldkamp-Davis-Kress algorithm for an equally spaced full circular orbit
 * and a flat detector): every pixel weighted by SDD / sqrt(SDD^2 + u^2 + v^2),
 * every detector row convolved (zero outside the row) with the Ram-Lak ramp
 * kernel of pitch dp = du SAD / SDD (dp times the sum; taps 1 / (4 dp^2) at
 * lag 0, -1 / (pi n dp)^2 at odd lags n, 0 at even lags), then per voxel
 * pi / n_views times the sum over views of (SAD / U)^2 times the filtered
 * data interpolated bilinearly where the ray from the source through the
 * voxel centre meets the detector (taps off the detector read 0), U = SAD -
 * (x cos t + y sin t).  angles must be NULL; nu <= 8192.  proj, vol: device,
 * storage dt; ws: tfcb_fdk_workspace_size bytes (the filtered projections in
 * FP32); asynchronous on `stream`. */
tfcb_status tfcb_fdk_workspace_size(const tfcb_geometry* g, size_t* bytes);
tfcb_status tfcb_fdk(const tfcb_geometry* g, tfcb_dtype dt, const void* proj, void* vol,
                     void* ws, size_t ws_bytes, void* stream);

/* The ROF sub-problem of the TV comparison method (section 2.3):
 * out = H(argmin_f ||f - x||^2 + mu TV(f)) approximated by gradient descent
 * from f = x, where TV(f) sums sqrt(d^2 + eps^2) over the forward differences
 * d of every voxel to its next neighbour along x, y and z (index units, no
 * term past the last voxel; the l1 norm of the gradient, smoothed).  The
 * step s starts at 1/2; a trial f - s grad that lowers the energy is taken
 * and s doubles (up to 1/2), otherwise s halves and the trial is repeated
 * (at most 40 times in a row); the descent ends after the first accepted
 * step whose relative decrease is below tol, or after max_steps accepted
 * steps.  Energies in FP64 on the device, arithmetic FP32.  H (negative
 * voxels to 0) when positivity = 1.  x, out: device [nz][ny][nx], storage
 * dt, must not alias; ws: tfcb_rof_workspace_size bytes.  Reads a stop flag
 * back between chunks of descent steps, so the call synchronises `stream`.
 * steps: nullable HOST output, the accepted steps. */
tfcb_status tfcb_rof_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes);
tfcb_status tfcb_rof(int32_t nx, int32_t ny, int32_t nz, double mu, double eps, double tol,
                     int32_t max_steps, int32_t positivity, tfcb_dtype dt, const void* x,
                     void* out, void* ws, size_t ws_bytes, void* stream, int32_t* steps);

/* n CGLS steps (Appendix 1) warm-started from x, updated in place:
 * r = g - P x, s = P^T r, p = s, gamma = ||s||^2; then n times q = P p,
 * alpha = gamma / ||q||^2, x += alpha p, r -= alpha q and (except after the
 * last step) s = P^T r, beta = ||s||^2 / gamma, p = s + beta p.  The call
 * stops early (x left as is) when gamma or ||q||^2 <= 1e-300.  Reductions in
 * FP64.  x: device volume, proj: device projections, storage o->storage;
 * only o->storage, o->cgls_steps and o->op_pair of `o` are used (op_pair 1
 * takes the Eq. (3) backprojection in place of P^T).  stats (nullable,
 * HOST, written after a stream synchronisation): [0] = ||r||^2 at exit,
 * [1] = 1 if the guard stopped the call. */
tfcb_status tfcb_cgls(const tfcb_geometry* g, const tfcb_options* o, void* x, const void* proj,
                      void* ws, size_t ws_bytes, void* stream, double* stats);

/* Multigrid restriction of the projections for the next-coarser grid
 * (section 2.2.3; the paper leaves restriction open): coarse pixel (r, c) is
 * the mean of the fine pixels {2r, 2r+1} x {2c, 2c+1} that exist.
 * in: [n_views][nv][nu] of `fine`; out: [n_views][ceil(nv/2)][ceil(nu/2)]. */
tfcb_status tfcb_restrict_sino(const tfcb_geometry* fine, tfcb_dtype dt, const void* in,
                               void* out, void* stream);

/* Multigrid prolongation (section 2.2.3, linear interpolation): each fine
 * voxel centre maps to the coarse fractional index p / d_coarse +
 * (N_coarse - 1) / 2 per axis, clamped to [0, N_coarse - 1], and takes the
 * trilinear interpolant of the coarse volume there. */
tfcb_status tfcb_prolong_vol(const tfcb_geometry* coarse, const tfcb_geometry* fine,
                             tfcb_dtype dt, const void* in, void* out, void* stream);

/* --------------------------------------------------------- reconstruction */
/* The full method: for each grid from the coarsest (section 2.2.3), start
 * from 0 (coarsest) or the prolonged coarser result with t = 1, and run
 * iters[grid] outer iterations of Algorithm A2 (A1 when momentum = 0):
 * v = f_k + ((t_{k-1} - 1) / t_k)(f_k - f_{k-1}); x = CGLS(v);
 * f_{k+1} = H(W^T T_lambda W x); t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2.
 * proj: device FP32 [n_views][nv][nu] post-log data of the finest grid;
 * vol: device FP32 [nz][ny][nx] output (1/mm).  Synchronises `stream`.
 * report: nullable HOST pointer.  Returns TFCB_ENUMERIC (vol still written)
 * when the result holds a non-finite value.  With regulariser = 1 the same
 * schedule runs the TV comparison method of section 2.3 instead: per outer
 * iteration x = CGLS(f) warm-started from f, then f = H(ROF(x)) as in
 * tfcb_rof with mu = lambda. */
tfcb_status tfcb_reconstruct(const tfcb_geometry* g, const tfcb_options* o, const float* proj,
                             float* vol, void* ws, size_t ws_bytes, void* stream,
                             tfcb_report* report);

/* ---------------------------------------------------------------- serving */
/* Continuous batching of whole reconstructions (the method of
 * tfcb_reconstruct, per request; the TF regulariser only: a request with
 * regulariser = 1 is refused with TFCB_EUNSUPPORTED).  Requests of any
 * geometry and options are
 * submitted at any time and admitted in arrival order as soon as one of
 * max_slots slots is free and the request's workspace (tfcb_request_bytes)
 * fits in the caller-owned device arena; each admitted request keeps all of
 * its state on the device, runs on its own stream, and advances one outer
 * iteration per tfcb_server_step, so the iterations of concurrent requests
 * overlap on the GPU.  A request's result is bitwise identical to
 * tfcb_reconstruct of the same input, alone or in any mix.
 *
 * Ownership: the arena (device, 256-byte aligned) is the caller's and must
 * outlive the server; the server owns its streams, events and a few bytes
 * of pinned host memory, released by tfcb_server_destroy.  proj (device
 * FP32 projections) and vol (device FP32 output) of a submitted request are
 * read/written until the request is DONE, FAILED or CANCELLED.  A server
 * handle is not thread-safe. */
typedef struct tfcb_server tfcb_server;
#define TFCB_REQ_QUEUED 0
#define TFCB_REQ_RUNNING 1
#define TFCB_REQ_DONE 2
#define TFCB_REQ_FAILED 3    /* result holds the status, e.g. TFCB_ENUMERIC */
#define TFCB_REQ_CANCELLED 4

/* Device bytes one request occupies in the arena. */
tfcb_status tfcb_request_bytes(const tfcb_geometry* g, const tfcb_options* o, size_t* bytes);
/* max_slots: 1..64 requests in flight at once. */
tfcb_status tfcb_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                               tfcb_server** out);
/* Validates and queues a request; TFCB_ENOMEM if it can never fit the arena.
 * stream: the caller's stream that produces proj (a hipStream_t as void*,
 * NULL = the null stream).  An event is recorded on it here, and the
 * request's first kernel waits for that event, so work enqueued on `stream`
 * before this call (e.g. the upload or computation of proj) is complete
 * before proj is read.  Work enqueued on it afterwards is not waited for.
 * vol may be read by the caller once tfcb_server_poll reports DONE.
 * id: HOST output. */
tfcb_status tfcb_server_submit(tfcb_server* s, const tfcb_geometry* g, const tfcb_options* o,
                               const float* proj, float* vol, void* stream, uint64_t* id);
/* Non-blocking: retires finished requests, admits queued ones, and enqueues
 * the next outer iteration of each active request (at most two iterations
 * ahead of the device per request).  n_active, n_queued: nullable HOST. */
tfcb_status tfcb_server_step(tfcb_server* s, int32_t* n_active, int32_t* n_queued);
/* state: TFCB_REQ_*; t_done: completion time in seconds of the host's
 * monotonic clock (CLOCK_MONOTONIC), from the device's completion event;
 * result: the request's status.  All nullable HOST. */
tfcb_status tfcb_server_poll(tfcb_server* s, uint64_t id, int32_t* state, double* t_done,
                             tfcb_status* result);
/* Cancels a queued or running request (waits for its in-flight kernels). */
tfcb_status tfcb_server_cancel(tfcb_server* s, uint64_t id);
/* Waits for all in-flight work, then frees the handle. */
tfcb_status tfcb_server_destroy(tfcb_server* s);

#ifdef __cplusplus
}
#endif
#endif /* TFCB_H */
