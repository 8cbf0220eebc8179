/* FP64 CPU oracle of the tight-frame (TF) cone-beam CT iteration of
 * Jia, Dong, Lou & Jiang, "GPU-based Iterative Cone Beam CT Reconstruction
 * Using Tight Frame Regularization" (arXiv 1008.2042).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never includes, links or calls anything here, and nothing here is shared
 * with it.
 *
 * Everything is IEEE double precision, plain loops, OpenMP only across
 * independent outputs (every result is deterministic).
 *
 * Conventions (the paper leaves them open; see the geometry comment in
 * tf_oracle.c):
 *   volume    f[k][j][i], i along x (fastest), voxel centres
 *             x_i = (i - (nx-1)/2) dx, same for y, z
 *   sinogram  g[view][r][c], c along the detector u axis (fastest)
 *   view k    theta_k = angles[k], or 2 pi k / n_views when angles is NULL
 */
#ifndef TF_ORACLE_H
#define TF_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz;
  int32_t nu, nv;
  double du, dv;
  double sad, sdd;
  int32_t n_views;
  const double* angles; /* NULL => equally spaced over 360 degrees */
} orc_geom;

typedef struct {
  double lambda;        /* shrink threshold (the paper's mu) */
  int32_t n_grids;      /* multigrid levels, 1..4 */
  int32_t iters[4];     /* outer iterations per grid, coarsest first */
  int32_t cgls_steps;   /* q = P p steps per CGLS call */
  int32_t framelet_levels; /* 1 or 2 */
  int32_t momentum;     /* 1 = Algorithm A2, 0 = Algorithm A1 */
  int32_t positivity;   /* 1 = apply H */
  int32_t bin_coarse_detector; /* 1 = 2x2 detector binning on coarser grids */
  int32_t op_pair;      /* 0 = Joseph P + exact transpose, 1 = Siddon P + Eq. (3) */
} orc_opts;

typedef struct {
  double resid2_last;      /* ||g - P x||^2 after the last CGLS update */
  int32_t cgls_breakdowns; /* CGLS calls stopped by the 1e-300 guard */
  int32_t iters_done[4];
} orc_report;

int orc_num_threads(void);

/* Cone-beam projection, Eq. (1) discretised by Joseph's method. */
void orc_project(const orc_geom* g, const double* f, double* proj);
/* The same, for a list of n rays (view, row, col) only. */
void orc_project_rays(const orc_geom* g, const double* f, int64_t n,
                      const int32_t* vrc, double* out);
/* Exact matrix transpose of orc_project (scatter form). */
void orc_backproject(const orc_geom* g, const double* proj, double* f);
/* The transpose evaluated at n voxels (k, j, i) only (gather over all rays). */
void orc_backproject_voxels(const orc_geom* g, const double* proj, int64_t n,
                            const int32_t* kji, double* out);

/* The paper's operator pair (section 2.2.1, Eq. (3)): Siddon's exact
 * radiological path through voxel boxes, and the closed-form voxel-driven
 * backprojection with bilinear detector interpolation (not the transpose of
 * either projector). */
void orc_project_siddon(const orc_geom* g, const double* f, double* proj);
void orc_project_siddon_rays(const orc_geom* g, const double* f, int64_t n,
                             const int32_t* vrc, double* out);
void orc_backproject_eq3(const orc_geom* g, const double* proj, double* f);
void orc_backproject_eq3_voxels(const orc_geom* g, const double* proj, int64_t n,
                                const int32_t* kji, double* out);

/* Framelet analysis W of one level: coeff[27][nz][ny][nx], band 9n+3m+l. */
void orc_framelet_analysis(int32_t nx, int32_t ny, int32_t nz, int32_t dil,
                           const double* f, double* coeff);
/* Exact adjoint W^T of orc_framelet_analysis. */
void orc_framelet_synthesis(int32_t nx, int32_t ny, int32_t nz, int32_t dil,
                            const double* coeff, double* f);
/* Vector shrink of Eq. (2), in place on coeff[27][V]. */
void orc_shrink(int64_t nvox, double lambda, double* coeff);
/* f_out = H(W^T T_lambda W f_in) with 1 or 2 framelet levels. */
void orc_framelet_shrink(int32_t nx, int32_t ny, int32_t nz, int32_t levels,
                         double lambda, int32_t positivity, const double* in,
                         double* out);

/* n CGLS steps (Appendix 1) warm-started from x (updated in place).
 * Returns 1 when the breakdown guard stopped the call.  resid2 (nullable)
 * receives ||g - P x||^2 at exit; resid_hist (nullable, n+1 entries) the
 * residual norm^2 after init and after each step. */
int orc_cgls(const orc_geom* g, double* x, const double* proj, int32_t n,
             double* resid2, double* resid_hist);
/* The same with the operator pair chosen (0 Joseph/transpose, 1 Siddon/Eq. (3)). */
int orc_cgls_pair(const orc_geom* g, int32_t pair, double* x, const double* proj, int32_t n,
                  double* resid2, double* resid_hist);

/* Multigrid transfer operators (section 2.2.3). */
void orc_coarse_geom(const orc_geom* fine, int32_t bin_detector, orc_geom* coarse);
void orc_restrict_sino(const orc_geom* fine, const double* in, double* out);
void orc_prolong_vol(const orc_geom* coarse, const orc_geom* fine,
                     const double* in, double* out);

/* Full reconstruction: Algorithm A2 (or A1) inside the coarse-to-fine schedule. */
int orc_reconstruct(const orc_geom* g, const orc_opts* o, const double* proj,
                    double* vol, orc_report* rep);
/* n_iters outer iterations on one grid, starting from f_cur = f_prev = vol. */
int orc_tf_iterations(const orc_geom* g, const orc_opts* o, const double* proj,
                      int32_t n_iters, double* vol, orc_report* rep);

/* The TV comparison method (section 2.3).  Energy of the ROF sub-problem
 * ||f - x||^2 + mu TV(f), TV(f) the l1 norm of the gradient summed over
 * voxels, smoothed: sum over voxels and axes of sqrt(d^2 + eps^2), d the
 * forward difference to the next voxel along the axis (index units; no
 * term past the last voxel). */
typedef struct {
  double mu;          /* TV weight mu_TV, >= 0 */
  double eps;         /* smoothing of |d|, > 0 */
  double tol;         /* stop when an accepted step lowers the energy by less
                         than this fraction of it (the paper's 0.1 %) */
  int32_t max_steps;  /* cap on accepted gradient steps per sub-problem */
} orc_tv;

double orc_tv_energy(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv,
                     const double* x, const double* f);
void orc_tv_gradient(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv,
                     const double* x, const double* f, double* grad);
/* The ROF sub-problem by gradient descent with an adaptive step, from f = x;
 * returns the number of accepted steps; energies (nullable, max_steps + 1
 * entries) receives the energy after each accepted step, [0] at f = x. */
int orc_rof(int32_t nx, int32_t ny, int32_t nz, const orc_tv* tv, const double* x,
            double* f, double* energies);
/* The TV method inside the same multigrid schedule: per outer iteration
 * x = CGLS(f), f = H(ROF(x)) (Algorithm A1 with step 2 replaced; momentum
 * and the framelet fields of o are not used).  rof_steps (nullable) is the
 * total number of accepted ROF steps. */
int orc_reconstruct_tv(const orc_geom* g, const orc_opts* o, const orc_tv* tv,
                       const double* proj, double* vol, orc_report* rep,
                       int32_t* rof_steps);

/* FDK (the paper's comparison baseline; textbook Feldkamp-Davis-Kress for an
 * equally spaced full orbit, angles must be NULL): cosine weighting, a
 * Ram-Lak ramp filter along detector rows, and the (SAD/U)^2-weighted
 * voxel-driven backprojection with bilinear detector interpolation. */
double orc_ramlak(int32_t n, double dp);
void orc_fdk_filter(const orc_geom* g, const double* proj, double* q);
void orc_fdk_backproject(const orc_geom* g, const double* q, double* vol);
int orc_fdk(const orc_geom* g, const double* proj, double* vol);

#endif
