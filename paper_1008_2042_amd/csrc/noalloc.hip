// The backprojector for callers that cannot allocate device memory: the
// same kernels and launch shapes as tfcb_backproject, with the scratch that
// call carves from its workspace (the per-view and per-column ray tables and
// the length-prescaled projections) held in one static device array of
// TFCB_NOALLOC_SCRATCH_BYTES per GPU instead.
#include <mutex>

#include "driver.h"

// One copy per GPU, resident from the module's load until the process ends.
// Host code never uses this name as an address: it stands for the device
// symbol only, and its per-device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[TFCB_NOALLOC_SCRATCH_BYTES];

namespace tfcb {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per
// device with that device current.
tfcb_status scratch_address(void** out) {
  int dev = -1;
  TFCB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(TFCB_EUNSUPPORTED, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TFCB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TFCB_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TFCB_OK;
}

}  // namespace
}  // namespace tfcb

using namespace tfcb;

extern "C" {

tfcb_status tfcb_backproject_noalloc(const tfcb_geometry* g, tfcb_dtype dt, const void* proj,
                                     void* vol, void* stream) {
  TFCB_TRY(validate_geometry(g));
  TFCB_TRY(validate_dtype(dt));
  TFCB_TRY(check_ptr(vol, "vol", dtype_size(dt)));
  TFCB_TRY(check_ptr(proj, "proj", dtype_size(dt)));
  // the workspace of tfcb_backproject: views, columns, prescaled projections
  Carver sizer(nullptr);
  sizer.take(sizeof(ViewInfo) * g->n_views);
  sizer.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu);
  sizer.take(npix(*g) * dtype_size(dt));
  if (sizer.off > (size_t)TFCB_NOALLOC_SCRATCH_BYTES)
    return fail(TFCB_EUNSUPPORTED,
                "tfcb_backproject_noalloc needs %zu scratch bytes for this geometry, more than "
                "its static %zu (use tfcb_backproject with a workspace)",
                sizer.off, (size_t)TFCB_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  TFCB_TRY(scratch_address(&base));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dispatch(dt, [&](auto tag) -> tfcb_status {
    using T = decltype(tag);
    Carver cv(base);
    ViewInfo* views = static_cast<ViewInfo*>(cv.take(sizeof(ViewInfo) * g->n_views));
    ColInfo* cols = static_cast<ColInfo*>(cv.take(sizeof(ColInfo) * (size_t)g->n_views * g->nu));
    T* rl = static_cast<T*>(cv.take(npix(*g) * sizeof(T)));
    // every byte used below is written before it is read: tables, then rl
    TFCB_HIP(launch_geom_tables(*g, views, cols, s));
    const GeomDev gd = make_geom_dev(*g);
    TFCB_HIP(launch_prescale(gd, cols, views, static_cast<const T*>(proj), rl, s));
    TFCB_HIP(launch_backproject(gd, views, cols, (const T*)rl, static_cast<T*>(vol), nullptr,
                                nullptr, s));
    return TFCB_OK;
  });
}

}  // extern "C"
