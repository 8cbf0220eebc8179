// Per-view and per-(view, column) ray constants, computed on the device in
// FP64 from the scan geometry (section 3 geometry; Eq. (1) rays) and stored
// in FP32 for the projector kernels.
#include "tfcb_internal.h"

namespace tfcb {

// Views per launch whose angles travel inside the kernel arguments (1 KB),
// so the caller's host array is read when the launch is enqueued and no
// host-to-device copy or synchronisation is needed.
constexpr int kAnglesPerLaunch = 128;

struct GeomParams64 {
  double dx, dy, dz, du, dv, sad, sdd;
  int32_t nx, ny, nz, nu, nv, n_views;
  int32_t has_angles;
  int32_t k0;  // first view of this launch
  double ang[kAnglesPerLaunch];
};

__global__ void k_geom_tables(GeomParams64 g, ViewInfo* __restrict__ views,
                              ColInfo* __restrict__ cols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = g.k0 + blockIdx.y;
  if (c >= g.nu) return;
  const double th =
      g.has_angles ? g.ang[blockIdx.y] : 2.0 * M_PI * (double)k / (double)g.n_views;
  const double cs = cos(th), sn = sin(th);
  const double sx = g.sad * cs, sy = g.sad * sn;
  const int step_x = fabs(cs) >= fabs(sn) - 1e-12;
  if (c == 0) {
    ViewInfo v;
    v.step_x = step_x;
    v.pad = 0;
    v.cs = (float)cs;
    v.sn = (float)sn;
    v.sx = (float)sx;
    v.sy = (float)sy;
    v.pad2[0] = v.pad2[1] = 0.f;
    views[k] = v;
  }
  const double uc = ((double)c - 0.5 * (g.nu - 1)) * g.du;
  const double ax = -g.sdd * cs - uc * sn;
  const double ay = -g.sdd * sn + uc * cs;
  const double a_step = step_x ? ax : ay;
  const double a_trans = step_x ? ay : ax;
  const double s_step = step_x ? sx : sy;
  const double s_trans = step_x ? sy : sx;
  const int ns = step_x ? g.nx : g.ny;
  const int nt = step_x ? g.ny : g.nx;
  const double ds = step_x ? g.dx : g.dy;
  const double dtr = step_x ? g.dy : g.dx;

  const double b0 = -0.5 * (ns - 1) * ds;
  const double tau0 = (b0 - s_step) / a_step;
  const double dtau = ds / a_step;
  ColInfo ci;
  ci.tau0 = (float)tau0;
  ci.dtau = (float)dtau;
  ci.t0 = (float)((s_trans + tau0 * a_trans) / dtr + 0.5 * (nt - 1));
  ci.dt = (float)(dtau * a_trans / dtr);
  ci.a2 = (float)(a_step * a_step + a_trans * a_trans);
  ci.inv_astep = (float)(1.0 / fabs(a_step));
  // Planes whose crossing lies strictly between source and detector.
  int lo = ns, hi = -1;
  for (int p = 0; p < ns; ++p) {
    const double bp = ((double)p - 0.5 * (ns - 1)) * ds;
    const double tau = (bp - s_step) / a_step;
    if (tau > 0.0 && tau < 1.0) {
      lo = p < lo ? p : lo;
      hi = p;
    }
  }
  if (hi < 0) lo = 0;
  ci.p_lo = lo;
  ci.p_hi = hi;
  cols[(size_t)k * g.nu + c] = ci;
}

hipError_t launch_geom_tables(const tfcb_geometry& g, ViewInfo* views, ColInfo* cols,
                              hipStream_t s) {
  GeomParams64 p{};
  p.dx = g.dx; p.dy = g.dy; p.dz = g.dz; p.du = g.du; p.dv = g.dv;
  p.sad = g.sad; p.sdd = g.sdd;
  p.nx = g.nx; p.ny = g.ny; p.nz = g.nz; p.nu = g.nu; p.nv = g.nv; p.n_views = g.n_views;
  p.has_angles = g.angles != nullptr;
  for (int k0 = 0; k0 < g.n_views; k0 += kAnglesPerLaunch) {
    const int n = g.n_views - k0 < kAnglesPerLaunch ? g.n_views - k0 : kAnglesPerLaunch;
    p.k0 = k0;
    if (g.angles)
      for (int i = 0; i < n; ++i) p.ang[i] = g.angles[k0 + i];
    dim3 block(64);
    dim3 grid((g.nu + 63) / 64, n);
    hipLaunchKernelGGL(k_geom_tables, grid, block, 0, s, p, views, cols);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tfcb
