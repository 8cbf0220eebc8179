// Host engine and C-ABI of libtfcb: validation, workspace carving and the
// reconstruction driver (Algorithm A2 with CGLS inside the multigrid
// schedule).  Host control stays on the CPU; every CGLS scalar stays on the
// device, so an outer iteration is a fixed sequence of kernel launches with
// no host round trip.
#include "driver.h"

using namespace tfcb;

extern "C" {

const char* tfcb_status_str(tfcb_status s) {
  switch (s) {
    case TFCB_OK: return "ok";
    case TFCB_EINVAL: return "invalid argument";
    case TFCB_ENOMEM: return "workspace too small";
    case TFCB_EDEVICE: return "device error";
    case TFCB_EUNSUPPORTED: return "unsupported";
    case TFCB_ENUMERIC: return "non-finite result";
    case TFCB_EBUSY: return "busy";
    default: return "unknown status";
  }
}

const char* tfcb_last_error(void) { return g_last_error.c_str(); }

const char* tfcb_version(void) { return "tfcb 0.1 gfx950"; }

tfcb_status tfcb_workspace_size(const tfcb_geometry* g, const tfcb_options* o, size_t* bytes) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_options(o));
  TFCB_TRY(validate_schedule(*g, *o));
  if (!bytes) return fail(TFCB_EINVAL, "bytes is NULL");
  Plan P;
  make_plan(*g, *o, nullptr, P);
  *bytes = P.bytes;
  return TFCB_OK;
}

tfcb_status tfcb_operator_workspace_size(const tfcb_geometry* g, tfcb_dtype dt, size_t* bytes) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  if (!bytes) return fail(TFCB_EINVAL, "bytes is NULL");
  *bytes = operator_ws_bytes(*g, dt);
  return TFCB_OK;
}

tfcb_status tfcb_framelet_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t levels,
                                         tfcb_dtype dt, size_t* bytes) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(TFCB_EINVAL, "sizes must be >= 1");
  if (levels != 1 && levels != 2) return fail(TFCB_EINVAL, "levels must be 1 or 2");
  TFCB_TRY(validate_dtype(dt));
  if (!bytes) return fail(TFCB_EINVAL, "bytes is NULL");
  const size_t V = (size_t)nx * ny * nz * dtype_size(dt);
  *bytes = levels == 2 ? 2 * align_up(V) : 0;
  return TFCB_OK;
}

tfcb_status tfcb_project(const tfcb_geometry* g, tfcb_dtype dt, const void* vol, void* proj,
                         void* ws, size_t ws_bytes, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  TFCB_TRY(check_ws(ws, ws_bytes, operator_ws_bytes(*g, dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    const size_t nN = pad_elems(g->ny, g->nx, g->nz), nT = pad_elems(g->nx, g->ny, g->nz);
    T* padN = static_cast<T*>(cv.take(nN * sizeof(T)));
    T* padT = static_cast<T*>(cv.take(nT * sizeof(T)));
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    const GeomDev gd = make_geom_dev(*g);
    TFCB_HIP(launch_fill(nN, 0.f, padN, s));
    TFCB_HIP(launch_fill(nT, 0.f, padT, s));
    TFCB_HIP(launch_pad_copies(g->nx, g->ny, g->nz, static_cast<const T*>(vol), padN, padT, s));
    TFCB_HIP(launch_project(gd, views, cols, (const T*)padN, (const T*)padT, 0,
                            static_cast<const T*>(nullptr), static_cast<T*>(proj),
                            static_cast<T*>(nullptr), nullptr, nullptr, s));
    return TFCB_OK;
  });
}

tfcb_status tfcb_backproject(const tfcb_geometry* g, tfcb_dtype dt, const void* proj, void* vol,
                             void* ws, size_t ws_bytes, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  TFCB_TRY(check_ws(ws, ws_bytes, operator_ws_bytes(*g, dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    T* rl = static_cast<T*>(cv.take(npix(*g) * sizeof(T)));
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    const GeomDev gd = make_geom_dev(*g);
    TFCB_HIP(launch_prescale(gd, cols, views, static_cast<const T*>(proj), rl, s));
    TFCB_HIP(launch_backproject(gd, views, cols, (const T*)rl, static_cast<T*>(vol), nullptr,
                                nullptr, s));
    return TFCB_OK;
  });
}

// Siddon P (section 2.2.1) of a native volume: its padded copies are built
// in the operator workspace, where tfcb_project keeps them too.
tfcb_status tfcb_project_siddon(const tfcb_geometry* g, tfcb_dtype dt, const void* vol,
                                void* proj, void* ws, size_t ws_bytes, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  TFCB_TRY(check_ws(ws, ws_bytes, operator_ws_bytes(*g, dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    const size_t nN = pad_elems(g->ny, g->nx, g->nz), nT = pad_elems(g->nx, g->ny, g->nz);
    T* padN = static_cast<T*>(cv.take(nN * sizeof(T)));
    T* padT = static_cast<T*>(cv.take(nT * sizeof(T)));
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    const GeomDev gd = make_geom_dev(*g);
    TFCB_HIP(launch_fill(nN, 0.f, padN, s));
    TFCB_HIP(launch_fill(nT, 0.f, padT, s));
    TFCB_HIP(launch_pad_copies(g->nx, g->ny, g->nz, static_cast<const T*>(vol), padN, padT, s));
    TFCB_HIP(launch_project_siddon(gd, views, (const T*)padN, (const T*)padT, 0,
                                   static_cast<const T*>(nullptr), static_cast<T*>(proj), nullptr,
                                   nullptr, s));
    return TFCB_OK;
  });
}

// The Eq. (3) backprojection (section 2.2.2) of plain projections.
tfcb_status tfcb_backproject_eq3(const tfcb_geometry* g, tfcb_dtype dt, const void* proj,
                                 void* vol, void* ws, size_t ws_bytes, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  TFCB_TRY(check_ws(ws, ws_bytes, operator_ws_bytes(*g, dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    const GeomDev gd = make_geom_dev(*g);
    TFCB_HIP(launch_backproject_eq3(gd, views, static_cast<const T*>(proj), static_cast<T*>(vol),
                                    nullptr, nullptr, s));
    return TFCB_OK;
  });
}

tfcb_status tfcb_framelet_shrink(int32_t nx, int32_t ny, int32_t nz, int32_t levels, double lambda,
                                 int32_t positivity, tfcb_dtype dt, const void* in, void* out,
                                 void* ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  TFCB_TRY(tfcb_framelet_workspace_size(nx, ny, nz, levels, dt, &need));
  if (!std::isfinite(lambda) || lambda < 0.0) return fail(TFCB_EINVAL, "lambda must be >= 0");
  TFCB_TRY(check_ptr(in, "in", dtype_size(dt)));
  TFCB_TRY(check_ptr(out, "out", dtype_size(dt)));
  if (in == out) return fail(TFCB_EINVAL, "in and out must not alias");
  TFCB_TRY(check_ws(ws, ws_bytes, need));
  if ((double)nx * ny * nz >= 2147483647.0) return fail(TFCB_EUNSUPPORTED, "volume too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  tfcb_geometry g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    T* t1 = levels == 2 ? static_cast<T*>(cv.take((size_t)nx * ny * nz * sizeof(T))) : nullptr;
    T* t2 = levels == 2 ? static_cast<T*>(cv.take((size_t)nx * ny * nz * sizeof(T))) : nullptr;
    return run_framelet<T>(g, levels, (float)lambda, positivity ? 1 : 0,
                           static_cast<const T*>(in), static_cast<T*>(out),
                           static_cast<const T*>(nullptr), static_cast<T*>(nullptr), 0.f, t1, t2,
                           s);
  });
}

static size_t fdk_ws_bytes(const tfcb_geometry& g) {
  Carver cv(nullptr);
  cv.take(sizeof(ViewInfo) * g.n_views);
  cv.take(sizeof(ColInfo) * (size_t)g.n_views * g.nu);
  cv.take(sizeof(float) * npix(g));
  return cv.off;
}

tfcb_status tfcb_fdk_workspace_size(const tfcb_geometry* g, size_t* bytes) {
  TFCB_TRY(validate_geometry(g));
  if (!bytes) return fail(TFCB_EINVAL, "bytes is NULL");
  *bytes = fdk_ws_bytes(*g);
  return TFCB_OK;
}

tfcb_status tfcb_fdk(const tfcb_geometry* g, tfcb_dtype dt, const void* proj, void* vol, void* ws,
                     size_t ws_bytes, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  if (g->angles)
    return fail(TFCB_EUNSUPPORTED, "FDK needs an equally spaced full orbit (angles = NULL)");
  if (!fdk_supported(g->nu)) return fail(TFCB_EUNSUPPORTED, "FDK needs nu <= 8192");
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ws(ws, ws_bytes, fdk_ws_bytes(*g)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    float* q = static_cast<float*>(cv.take(sizeof(float) * npix(*g)));
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    TFCB_HIP(launch_fdk(make_geom_dev(*g), views, static_cast<const T*>(proj), q,
                        static_cast<T*>(vol), s));
    return TFCB_OK;
  });
}

tfcb_status tfcb_rof_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(TFCB_EINVAL, "sizes must be >= 1");
  if ((double)nx * ny * nz >= 2147483647.0) return fail(TFCB_EUNSUPPORTED, "volume too large");
  if (!bytes) return fail(TFCB_EINVAL, "bytes is NULL");
  Carver cv(nullptr);
  cv.take((size_t)nx * ny * nz * sizeof(float));
  cv.take(rof_state_bytes());
  cv.take(sizeof(double) * rof_num_partials(nx, ny, nz));
  *bytes = cv.off;
  return TFCB_OK;
}

tfcb_status tfcb_rof(int32_t nx, int32_t ny, int32_t nz, double mu, double eps, double tol,
                     int32_t max_steps, int32_t positivity, tfcb_dtype dt, const void* x,
                     void* out, void* ws, size_t ws_bytes, void* stream, int32_t* steps) {
  size_t need = 0;
  TFCB_TRY(tfcb_rof_workspace_size(nx, ny, nz, &need));
  TFCB_TRY(validate_dtype(dt));
  if (!std::isfinite(mu) || mu < 0.0) return fail(TFCB_EINVAL, "mu must be finite and >= 0");
  if (!std::isfinite(eps) || !(eps > 0.0)) return fail(TFCB_EINVAL, "eps must be finite and > 0");
  if (!std::isfinite(tol) || tol < 0.0) return fail(TFCB_EINVAL, "tol must be finite and >= 0");
  if (max_steps < 0 || max_steps > 100000) return fail(TFCB_EINVAL, "max_steps must be 0..100000");
  TFCB_TRY(check_ptr(x, "x", dtype_size(dt)));
  TFCB_TRY(check_ptr(out, "out", dtype_size(dt)));
  if (x == out) return fail(TFCB_EINVAL, "x and out must not alias");
  TFCB_TRY(check_ws(ws, ws_bytes, need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(ws);
    float* g = static_cast<float*>(cv.take((size_t)nx * ny * nz * sizeof(float)));
    void* state = cv.take(rof_state_bytes());
    double* partials = static_cast<double*>(cv.take(sizeof(double) * rof_num_partials(nx, ny, nz)));
    int n = 0;
    TFCB_HIP(launch_rof<T>(nx, ny, nz, (float)mu, (float)eps, tol, max_steps, positivity ? 1 : 0,
                           static_cast<const T*>(x), static_cast<T*>(out), g, state, partials, &n,
                           s));
    if (steps) *steps = n;
    return TFCB_OK;
  });
}

tfcb_status tfcb_cgls(const tfcb_geometry* g, const tfcb_options* o, void* x, const void* proj,
                      void* ws, size_t ws_bytes, void* stream, double* stats) {
  TFCB_TRY(validate_geometry(g));
  if (!o) return fail(TFCB_EINVAL, "options is NULL");
  TFCB_TRY(validate_dtype(o->storage));
  if (o->cgls_steps < 1 || o->cgls_steps > 64) return fail(TFCB_EINVAL, "cgls_steps must be 1..64");
  if (o->op_pair != 0 && o->op_pair != 1) return fail(TFCB_EINVAL, "op_pair must be 0 or 1");
  TFCB_TRY(check_ptr(x, "x", dtype_size(o->storage)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(o->storage)));
  tfcb_options one = *o;
  one.n_grids = 1;
  one.iters[0] = 1;
  one.framelet_levels = 1;
  Plan P;
  make_plan(*g, one, nullptr, P);
  TFCB_TRY(check_ws(ws, ws_bytes, P.bytes));
  make_plan(*g, one, ws, P);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(o->storage, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    TFCB_HIP(launch_cgls_reset(P.sc, s));
    TFCB_TRY(setup_grid<T>(P.grid[0], s));
    TFCB_TRY(run_cgls<T>(P.grid[0], P.sc, static_cast<T*>(x), static_cast<const T*>(proj),
                         o->cgls_steps, s));
    if (stats) {
      CglsScalars h;
      TFCB_HIP(hipMemcpyAsync(&h, P.sc, sizeof h, hipMemcpyDeviceToHost, s));
      TFCB_HIP(hipStreamSynchronize(s));
      stats[0] = h.resid2;
      stats[1] = h.breakdowns > 0 ? 1.0 : 0.0;
    }
    return TFCB_OK;
  });
}

tfcb_status tfcb_restrict_sino(const tfcb_geometry* fine, tfcb_dtype dt, const void* in, void* out,
                               void* stream) {
  TFCB_TRY(validate_geometry(fine));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(in, "in", dtype_size(dt)));
  TFCB_TRY(check_ptr(out, "out", dtype_size(dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    TFCB_HIP(launch_restrict(fine->n_views, fine->nu, fine->nv, static_cast<const T*>(in),
                             static_cast<T*>(out), s));
    return TFCB_OK;
  });
}

tfcb_status tfcb_prolong_vol(const tfcb_geometry* coarse, const tfcb_geometry* fine, tfcb_dtype dt,
                             const void* in, void* out, void* stream) {
  if (!coarse || !fine) return fail(TFCB_EINVAL, "geometry is NULL");
  if (coarse->nx < 1 || coarse->ny < 1 || coarse->nz < 1 || fine->nx < 1 || fine->ny < 1 ||
      fine->nz < 1)
    return fail(TFCB_EINVAL, "sizes must be >= 1");
  if (!finite_pos(coarse->dx) || !finite_pos(coarse->dy) || !finite_pos(coarse->dz) ||
      !finite_pos(fine->dx) || !finite_pos(fine->dy) || !finite_pos(fine->dz))
    return fail(TFCB_EINVAL, "voxel sizes must be finite and > 0");
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(in, "in", dtype_size(dt)));
  TFCB_TRY(check_ptr(out, "out", dtype_size(dt)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    TFCB_HIP(launch_prolong(*coarse, *fine, static_cast<const T*>(in), static_cast<T*>(out), s));
    return TFCB_OK;
  });
}

tfcb_status tfcb_reconstruct(const tfcb_geometry* g, const tfcb_options* o, const float* proj,
                             float* vol, void* ws, size_t ws_bytes, void* stream,
                             tfcb_report* report) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_options(o));
  TFCB_TRY(validate_schedule(*g, *o));
  TFCB_TRY(check_ptr(proj, "proj", sizeof(float)));
  TFCB_TRY(check_ptr(vol, "vol", sizeof(float)));
  Plan P;
  make_plan(*g, *o, nullptr, P);
  TFCB_TRY(check_ws(ws, ws_bytes, P.bytes));
  make_plan(*g, *o, ws, P);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(o->storage, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    return reconstruct_t<T>(*g, *o, proj, vol, P, s, report);
  });
}

}  // extern "C"
