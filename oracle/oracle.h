/*
 * Plain FP64 CPU oracle for the tensor-product multigrid and line-preconditioned
 * CG solvers of Mueller, Scheichl & Vainikko, "Petascale elliptic solvers for
 * anisotropic PDEs on GPU clusters" (arXiv:1402.3545).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library: it assembles A explicitly as CSR and runs the textbook
 * algorithms on it.
 *
 * Vectors are in the canonical z-contiguous order g = (j*nx + i)*nz + k.
 * Levels are numbered by depth: 0 is the finest grid (the paper's level L),
 * nlevels-1 the coarsest (the paper's level 1).
 */
#ifndef GMG_ORACLE_H
#define GMG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_problem or_problem;

/* Build the hierarchy.  bc_h: 0 = doubly periodic, 1 = homogeneous Dirichlet
 * on the four side walls (wall faces couple with 2 K_T to a zero value).
 * bc_v: 0 = Dirichlet top/bottom, 1 = Neumann.  zfaces: nz+1 increasing faces
 * in [0,1] (NULL = (k/nz)^2).  kh: nx*ny per-column coefficients in order
 * j*nx+i (NULL = 1).  Returns NULL on invalid input; or_last_error() says why. */
or_problem *or_create(int nx, int ny, int nz, int nlevels, int bc_h, int bc_v,
                      double kv, double sigma, const double *zfaces,
                      const double *kh, double rho, int ncoarse);
/* The same hierarchy without CSR matrices (only the row-wise functions and the
 * transfers work on it). */
or_problem *or_create_matfree(int nx, int ny, int nz, int nlevels, int bc_h, int bc_v,
                              double kv, double sigma, const double *zfaces,
                              const double *kh, double rho, int ncoarse);
void or_destroy(or_problem *p);
const char *or_last_error(void);

int or_shape(const or_problem *p, int depth, int *nx, int *ny, int *nz);
int64_t or_nnz(const or_problem *p, int depth);
int or_csr(const or_problem *p, int depth, int64_t *rowptr, int32_t *col, double *val);
int or_profiles(const or_problem *p, double *dz, double *tface);
int or_faces(const or_problem *p, int depth, double *kcol, double *cx, double *cy);
/* per column (j*nx+i): the summed couplings of its Dirichlet wall faces
 * (all zero for periodic boundaries) */
int or_walls(const or_problem *p, int depth, double *wall);

/* Single operations (the plain definitions). */
int or_spmv(const or_problem *p, int depth, const double *x, double *y);
int or_residual(const or_problem *p, int depth, const double *f, const double *u, double *r);
int or_line_solve(const or_problem *p, int depth, const double *r, double *z);
int or_smooth(or_problem *p, int depth, const double *f, double *u, double rho);
int or_restrict(const or_problem *p, int depth_fine, const double *rf, double *fc);
int or_prolongate_add(const or_problem *p, int depth_coarse, const double *uc, double *uf);
int or_restrict_smooth(or_problem *p, int depth_coarse, const double *rf, double *fc,
                       double *uc, double rho);

/* Algorithm 1 (one V(1,1) cycle on the finest level) and the two solvers. */
int or_vcycle(or_problem *p, const double *f, double *u);
int or_mg_solve(or_problem *p, const double *f, double *u, double rtol, int maxit,
                int *iters, double *history);
int or_pcg_solve(or_problem *p, const double *f, double *u, double rtol, int maxit,
                 int *iters, double *history, double *relres_true);

/* Row-wise forms (no stored matrix). */
int or_apply_rows(const or_problem *p, int depth, int64_t nrows, const int64_t *rows,
                  const double *x, double *y);
double or_residual_norm2_rows(const or_problem *p, int depth, const double *f, const double *u);
int or_line_solve_columns(const or_problem *p, int depth, int64_t ncols, const int64_t *cols,
                          const double *r, double *z);

double or_dot(int64_t n, const double *x, const double *y);
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
