/*
 * gmg.h -- C ABI of the MI355X (gfx950) tensor-product multigrid and
 * line-preconditioned CG library.
 *
 * Method: Mueller, Scheichl & Vainikko, "Petascale elliptic solvers for
 * anisotropic PDEs on GPU clusters" (arXiv:1402.3545).
 *
 * Operator (Sec. 2.1.1, column-block form; Sec. 3.1, matrix-free tensor-product
 * stencil).  Columns T = (i, j) of an nx x ny grid on the unit square, doubly
 * periodic or with homogeneous Dirichlet side walls (gmg_params.bc_h), nz
 * layers between the faces z_0 < ... < z_nz.  With |T| = hx*hy,
 * dz_k = z_{k+1} - z_k, cell centres zeta_k and vertical transmissibilities
 * t_k = kv / (zeta_k - zeta_{k-1}) (interior faces), t_0 = 2 kv / dz_0 and
 * t_nz = 2 kv / dz_{nz-1} (Dirichlet ends) or 0 (Neumann ends):
 *
 *   (A u)_{T,k} = |T| [ sigma dz_k u_{T,k} + t_k (u_{T,k} - u_{T,k-1})
 *                                        + t_{k+1} (u_{T,k} - u_{T,k+1}) ]
 *               + dz_k sum_{T' in N(T)} C_TT' (u_{T,k} - u_{T',k})
 *
 * where C_TT' is the harmonic mean of the column coefficients K_T, K_T' times
 * the face-length / centre-distance ratio (hy/hx in x, hx/hy in y), and
 * u_{T,-1} = u_{T,nz} = 0.  With Dirichlet side walls a wall is a neighbour
 * of value 0 at half a cell, coupled with 2 K_T times the face ratio.  M = blockdiag(A_T) is the vertical line operator of
 * Sec. 2.2.  Coarse levels halve nx and ny (horizontal-only semicoarsening),
 * average K over the four children and rediscretise.
 *
 * Field layout on the device (Sec. 3.1, x-contiguous ordering): element
 * (i, j, k) of a level is at index (j*nz + k)*ldx + i, ldx >= nx padded to a
 * multiple of 32 elements; gmg_field_layout() returns ldx and the element count
 * of each level.  Padding elements are never read.
 *
 * Levels are numbered by depth: 0 is the finest grid (the paper's level L),
 * nlevels-1 the coarsest (the paper's level 1).
 *
 * Conventions for every entry point:
 *  - Pointers named f, u, x, y, r, z are DEVICE pointers owned by the caller,
 *    in the layout above, 8-byte (GMG_F64) or 4-byte (GMG_F32) elements,
 *    aligned to at least 16 bytes.  The library keeps no reference to them.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Kernels are enqueued
 *    on it; spmv, line_solve, line_smooth, gmg_residual, gmg_restrict_smooth,
 *    gmg_prolongate and gmg_vcycle return without synchronising.  The solvers
 *    synchronise the stream before they return their scalars.
 *  - A context must not be used from two host threads or two streams at once.
 *  - Every function returns GMG_OK or a negative gmg_status; nothing aborts or
 *    prints.  gmg_last_error() gives a message for the calling thread's last
 *    failure.
 */
#ifndef GMG_H
#define GMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmg_ctx gmg_ctx;

typedef enum {
  GMG_OK = 0,
  GMG_EINVAL = -1,       /* bad argument: shape, pointer, tolerance, level */
  GMG_ENOMEM = -2,       /* device or host allocation failed */
  GMG_EHIP = -3,         /* a HIP runtime call failed */
  GMG_ENOCONV = -4,      /* solver hit maxit, or a reduction became NaN/Inf */
  GMG_EUNSUPPORTED = -5  /* valid request this build does not implement */
} gmg_status;

typedef enum { GMG_F64 = 0, GMG_F32 = 1 } gmg_prec;

typedef struct {
  int32_t nx, ny, nz;     /* finest grid; nx, ny >= 2 and divisible by
                             2^(nlevels-1) (the coarsest level may be a single
                             column per direction); 2 <= nz <= 128 */
  int32_t nlevels;        /* >= 1 */
  int32_t bc_h;           /* 0 = doubly periodic; 1 = homogeneous Dirichlet on the
                             four side walls (Sec. 2.1.1): a wall face couples the
                             outermost column to zero with 2 K times the face
                             ratio, and prolongation reflects oddly at walls */
  int32_t bc_v;           /* 0 = Dirichlet top and bottom, 1 = Neumann */
  double kv;              /* vertical coefficient K_v >= 0 */
  double sigma;           /* zero-order coefficient > 0 */
  const double *zfaces;   /* HOST, nz+1 strictly increasing faces; NULL = (k/nz)^2 */
  const double *kh;       /* HOST, nx*ny positive column coefficients, index j*nx+i;
                             NULL = 1 */
  double rho;             /* smoother damping (Sec. 5: 2/3) */
  int32_t ncoarse;        /* smoothing steps on the coarsest level (Sec. 2.2: 2) */
  int32_t prec_precond;   /* GMG_F64 or GMG_F32: precision of the V-cycle used by
                             gmg_vcycle / gmg_solve / pcg_solve(precond=1) */
} gmg_params;

/* Fill *p with the defaults: bc periodic/Dirichlet, kv 1, sigma 1, rho 2/3,
 * ncoarse 2, prec_precond GMG_F64, zfaces and kh NULL. */
void gmg_default_params(gmg_params *p);

/* Build a context: vertical profiles, per-level face couplings (FP64 and FP32
 * copies), the level hierarchy and all scratch, on the current HIP device.
 * The host arrays zfaces/kh are copied; the caller may free them afterwards.
 * Synchronises `stream`.  *out receives the context (NULL on failure). */
int gmg_setup(const gmg_params *p, void *stream, gmg_ctx **out);

/* Free every device and host resource of the context.  NULL is accepted. */
int gmg_destroy(gmg_ctx *c);

/* Layout of level `level`: leading dimension ldx (elements) and the number
 * of elements a field of that level occupies (ny * nz * ldx). */
int gmg_field_layout(const gmg_ctx *c, int level, int64_t *ldx, int64_t *elems);

/* y = A x on level `level` (the SpMV of Sec. 2.2, eq. for y <- A x).  x and y
 * must not overlap. */
int spmv(gmg_ctx *c, int level, int prec, const void *x, void *y, void *stream);

/* z = M^{-1} r: the vertical line solve (Sec. 2.2, preconditioner y <- M^{-1} x;
 * one tridiagonal system per column).  r and z may be the same buffer. */
int line_solve(gmg_ctx *c, int level, int prec, const void *r, void *z, void *stream);

/* nsweeps steps of the block-Jacobi smoother u <- u + rho M^{-1} (f - A u)
 * (Sec. 2.2, smoother equation; kernel "Smooth" of Sec. 3.1).  u is updated in
 * place as seen by the caller (the library ping-pongs through its own buffer). */
int line_smooth(gmg_ctx *c, int level, int prec, const void *f, void *u, int nsweeps,
                double rho, void *stream);

/* r = f - A u (kernel "Residual", Sec. 3.1).  If norm2 is not NULL it receives
 * ||r||_2^2 accumulated in FP64 (this synchronises the stream). */
int gmg_residual(gmg_ctx *c, int level, int prec, const void *f, const void *u, void *r,
                 double *norm2, void *stream);

/* Allocation-free variant of gmg_residual, for callers that cannot allocate
 * device memory or synchronise: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  r = f - A u as gmg_residual (same
 * kernels and launch shape, so r and the norm are bitwise those of
 * gmg_residual); if norm2 is not NULL it is a DEVICE pointer (8-byte aligned,
 * caller-owned) that receives ||r||_2^2 accumulated in FP64, written on
 * `stream` -- the call never synchronises and never allocates.  The
 * per-workgroup partial sums go to a static 1 MiB device array, one per GPU,
 * held until the process ends (its address is taken once per device at
 * gmg_setup or at the first call on a device).  Every call on a GPU shares
 * that array: calls that overlap on one GPU (two streams, two host threads)
 * race and must be serialised by the caller; nothing in it needs clearing,
 * since each launch writes all the partials it reads.  With norm2 set,
 * GMG_EINVAL for a level whose residual launch has more than 131072
 * workgroups (64 x 4 columns x 32 layers each, i.e. above about 1.07e9 cells
 * of a level whose sizes are multiples of those).  Launches are not recorded
 * by gmg_timing_*. */
int gmg_residual_noalloc(gmg_ctx *c, int level, int prec, const void *f, const void *u, void *r,
                         double *norm2, void *stream);

/* Kernel "ResSmooth" (Sec. 3.1, Algorithm 1): fc = R rf, the sum over the four
 * horizontal children, then uc = rho M^{-1} fc (one smoothing step from a zero
 * initial guess).  level is the COARSE level (>= 1); rf lives on level-1. */
int gmg_restrict_smooth(gmg_ctx *c, int level, int prec, const void *rf, void *fc, void *uc,
                        double rho, void *stream);

/* Kernel "Prolongate" (Sec. 3.1, Algorithm 1): uf += P uc, cell-centred bilinear
 * interpolation in the horizontal (weights 9/16, 3/16, 3/16, 1/16; periodic,
 * or behind a Dirichlet wall the parent's mirror image with opposite sign).
 * level is the COARSE level (>= 1); uf lives on level-1. */
int gmg_prolongate(gmg_ctx *c, int level, int prec, const void *uc, void *uf, void *stream);

/* One V(1,1) cycle of Algorithm 1 on the finest level in the precision
 * prec_precond: f and u are fields of that precision; u is updated in place.
 * On the coarsest level the exact solve is replaced by ResSmooth followed by
 * ncoarse-1 Smooth steps. */
int gmg_vcycle(gmg_ctx *c, const void *f, void *u, void *stream);

/* Multigrid solve of A u = f (FP64 f, u on the device; u holds the initial
 * guess).  prec_precond == GMG_F64: V-cycles until ||f - A u|| / ||f - A u_0||
 * < rtol (Sec. 2.2, stopping test).  prec_precond == GMG_F32: FP64 iterative
 * refinement, each step one FP32 V-cycle on the FP64 residual.  *iters gets
 * the number of cycles, *relres the final FP64 relative residual, history
 * (host, maxit+1 doubles, may be NULL) the relative residual after each cycle.
 * Returns GMG_ENOCONV if maxit is reached or the residual is not finite. */
int gmg_solve(gmg_ctx *c, const double *f, double *u, double rtol, int maxit, int *iters,
              double *relres, double *history, void *stream);

/* Preconditioned CG (Sec. 2.2; fused kernels of Sec. 3.1).  precond = 0: the
 * vertical line preconditioner M in FP64, with the two fused kernels
 * (SpMV + vector updates + <p,q>; line solve + residual update + <r,r>, <r,z>);
 * the iterate takes its steps alpha p two at a time, in the first kernel of
 * every other iteration, and those still pending at exit in a final update
 * (the same iterates as one step per iteration).
 * precond = 1: flexible CG with one V-cycle (in prec_precond) as the
 * preconditioner.  precond = 2: flexible CG with the line preconditioner M
 * applied in prec_precond (with GMG_F32: FP32 Thomas on the FP32-rounded
 * residual, an inexact preconditioner the flexible recurrence tolerates).
 * Stops when the recursively updated ||r|| / ||r_0|| < rtol;
 * *relres gets the TRUE relative residual ||f - A u|| / ||f - A u_0|| at exit,
 * history (host, maxit+1, may be NULL) the recursive one per iteration. */
int pcg_solve(gmg_ctx *c, const double *f, double *u, double rtol, int maxit, int precond,
              int *iters, double *relres, double *history, void *stream);

/* Batched solves: `ninst` independent instances (each with its own grid size,
 * level count and coefficients, inst[i]; rho and ncoarse must agree), each
 * with `nrhs` right-hand sides, solved together by FP64 iterative refinement
 * with FP32 V-cycles of Algorithm 1.  Every V-cycle phase of all pairs runs in
 * one grouped launch per phase; each refinement step is one hipGraph replay;
 * converged (instance, rhs) pairs are masked on the device.  The context owns
 * the fields of every pair (about 40 bytes per unknown and right-hand side).
 * Single-instance entry points reject a batched context. */
int gmg_batch_setup(const gmg_params *inst, int ninst, int nrhs, void *stream, gmg_ctx **out);

/* Layout of instance `instance` (its finest level), as gmg_field_layout. */
int gmg_batch_layout(const gmg_ctx *c, int instance, int64_t *ldx, int64_t *elems);

/* f[i*nrhs + r], u[i*nrhs + r]: DEVICE FP64 fields of instance i, rhs r in that
 * instance's layout; u holds the initial guess and receives the solution.
 * iters, relres: HOST arrays of ninst*nrhs (may be NULL): cycles and final
 * relative residual ||f - A u|| / ||f - A u_0|| of each pair.  Synchronises
 * `stream`.  GMG_ENOCONV if any pair missed rtol within maxit cycles. */
int gmg_batch_solve(gmg_ctx *c, const double *const *f, double *const *u, double rtol,
                    int maxit, int *iters, double *relres, void *stream);

/* Per-kernel timing (measurement support; the paper's per-kernel, per-level
 * breakdown tables, Sec. 5.3).  While enabled, every kernel the context
 * launches is bracketed by two HIP events on its launch stream.
 * gmg_timing_enable(c, 1) clears earlier records and starts recording;
 * gmg_timing_enable(c, 0) stops.  gmg_timing_read() waits for the recorded
 * events and returns, for one kernel kind / level / precision, the number of
 * launches and their summed duration in milliseconds since the last enable.
 * level = -1 sums over all levels.  GMG_K_CG_SPMV and GMG_K_CG_TRIDIAG are
 * the two fused kernels of the line-preconditioned CG; GMG_K_CORRECT is the
 * fused update + residual of the mixed-precision refinement; GMG_K_FCG the
 * vector kernels of the flexible CG; GMG_K_RESIDUAL_RESTRICT the V-cycle's
 * fused fine-level residual + restriction (timed under the fine level; the
 * residual is not stored); GMG_K_AUX fills and final updates.  Inside the
 * V-cycle each coarse level starts with a scaled line solve, timed as
 * GMG_K_LINE_SOLVE of that level.  GMG_K_PROLONG_SMOOTH is the V-cycle's
 * prolongation onto a level folded into that level's post-smoother (one
 * kernel instead of GMG_K_PROLONGATE + GMG_K_SMOOTH; timed under the fine
 * level), used where its launch shape says so (below). */
typedef enum {
  GMG_K_SPMV = 0, GMG_K_RESIDUAL = 1, GMG_K_LINE_SOLVE = 2, GMG_K_SMOOTH = 3,
  GMG_K_RESTRICT_SMOOTH = 4, GMG_K_PROLONGATE = 5, GMG_K_CG_SPMV = 6, GMG_K_CG_TRIDIAG = 7,
  GMG_K_REDUCE = 8, GMG_K_AUX = 9, GMG_K_CORRECT = 10, GMG_K_FCG = 11,
  GMG_K_RESIDUAL_RESTRICT = 12, GMG_K_PROLONG_SMOOTH = 13, GMG_K_COUNT = 14
} gmg_kernel;
int gmg_timing_enable(gmg_ctx *c, int enable);
int gmg_timing_read(gmg_ctx *c, int kernel, int level, int prec, int64_t *count,
                    double *total_ms);
/* Restrict the timing to the kernel kinds whose bit (1u << gmg_kernel) is set
 * in kernel_mask; ~0u (the default) times every kernel.  Untimed kernels are
 * launched without events, so a measurement of one kernel kind adds no
 * overhead to the others.  Takes effect for launches after the call. */
int gmg_timing_filter(gmg_ctx *c, uint32_t kernel_mask);

/* A plain streaming copy of `bytes` bytes (a multiple of 8) from src to dst,
 * device arrays owned by the caller, 16-byte aligned and not overlapping:
 * the achievable-copy ceiling that the kernels' HBM bandwidth is judged
 * against (Sec. 5 reports bandwidth as a fraction of the hardware's; a copy
 * shows what a read + write stream reaches on this GPU).  8-byte
 * non-temporal loads and stores, grid-stride.  Asynchronous on `stream`.
 * GMG_EINVAL for NULL or unaligned pointers, a bad size, or overlap. */
int gmg_copy_probe(const void *src, void *dst, int64_t bytes, void *stream);

/* Layout conversion of one field on the device between the canonical
 * z-contiguous order (j*nx + i)*nz + k -- the order of the caller's host data
 * and of the synthetic inputs -- and the x-contiguous order of
 * gmg_field_layout (Sec. 3.1 stores fields x-contiguous; Sec. 5.1 reports
 * the host transfer and this transpose as part of the total solution time).
 * level selects the grid, prec the element type (GMG_F64 / GMG_F32); src and
 * dst are distinct device arrays of nx*ny*nz (z-contiguous) and `elems` of
 * gmg_field_layout (x-contiguous) elements, owned by the caller; padding
 * columns of the x-contiguous field are not written.  Asynchronous on
 * `stream`.  GMG_EINVAL for a bad level or precision, NULL or unaligned
 * pointers, src == dst. */
int gmg_transpose_in(gmg_ctx *c, int level, int prec, const void *src_z, void *dst_x,
                     void *stream);
int gmg_transpose_out(gmg_ctx *c, int level, int prec, const void *src_x, void *dst_z,
                      void *stream);

/* A whole solve from host memory (Sec. 5.1 "total solution time"): copies
 * f_host and the initial guess u_host (both FP64, z-contiguous order,
 * nx*ny*nz values, caller-owned pageable or pinned host memory) to the
 * device, converts their layout, runs gmg_solve (method 0: multigrid, or
 * refinement with FP32 cycles when the context's preconditioner is FP32) or
 * pcg_solve (method 1: line preconditioner, 2: V-cycle preconditioner,
 * flexible CG), converts u back and copies it into u_host.  The copies go
 * through two pinned host buffers of up to 128 MiB, in chunks: host threads
 * fill (or empty) one buffer while the DMA engine drains (or fills) the other.
 * On first use the context allocates three level-0 FP64 device fields and
 * the two pinned buffers, and keeps them until gmg_destroy (GMG_ENOMEM when
 * either allocation fails).  timings_ms (may be NULL) receives 5 host-clock
 * values, each step ending in a synchronisation: host to device copies,
 * layout conversion in, solve, layout conversion out, device to host copy.
 * Synchronises `stream`; not safe for concurrent calls on one context.
 * Returns the solve's status (GMG_ENOCONV still copies the last iterate out). */
int gmg_solve_host(gmg_ctx *c, int method, const double *f_host, double *u_host, double rtol,
                   int maxit, int *iters, double *relres, double *timings_ms, void *stream);

/* Launch shapes and the autotuner.  Sec. 5.1 fixes one thread-block layout
 * for every kernel; here each kernel kind (gmg_kernel), level and precision
 * has its own shape, which only changes how the work is cut into workgroups:
 *   rows  - grid rows per workgroup of the stencil kernels (SpMV, residual,
 *           fused residual+restriction, prolongation, CG direction kernel,
 *           refinement update, flexible-CG kernels): 4, 8 or 16 wavefronts
 *           of 64 columns.  Line kernels use 4 wavefronts of 32 columns (the
 *           twisted elimination, rows = 4); the line solve and the smoother
 *           (GMG_K_LINE_SOLVE, GMG_K_SMOOTH) also take rows = 1: one
 *           wavefront per column, solved by parallel cyclic reduction
 *           (n_z <= 128), for levels with too few columns to fill the GPU;
 *           the smoother also takes rows = 2: the twisted elimination with
 *           the horizontal neighbours staged in LDS by the workgroup (each u
 *           value of the tile and its halo read once) instead of read per lane,
 *           and rows = 3: the same staging with the two halves of each column
 *           in two wavefronts (tiles of 64 columns by 2 grid rows), for
 *           levels with n_z of 32, 64 or 128, n_x a multiple of 64 and n_y
 *           even; on other levels rows = 3 runs as rows = 2.
 *           GMG_K_PROLONG_SMOOTH of level l (l < nlevels - 1) takes rows = 4
 *           (the default: the V-cycle prolongates from level l+1 and then
 *           post-smooths level l, two kernels) or rows = 2 or 3 (one kernel:
 *           the staged smoother of that shape adds the prolongated correction
 *           to every value it stages, so u + P u_c is never stored; the same
 *           arithmetic).
 *   group - tile columns per dispatch group: tiles are walked group by group
 *           and tile rows follow each other inside a group, so that a tile's
 *           neighbours run close in time and share an XCD's L2; 0 walks the
 *           tiles row by row (the default).
 * Results are identical for every shape except for the summation order of
 * the FP64 reductions (norms and dot products).
 * gmg_set_launch / gmg_get_launch: one entry of the context's table;
 * GMG_EINVAL for a bad kernel id, level or precision, rows not in {4, 8, 16}
 * (or 1 for the line solve and smoother, 2 or 3 for the smoother;
 * GMG_K_PROLONG_SMOOTH takes 4, 2 or 3 only), group outside [0, 4096], and for
 * batched contexts.
 * gmg_autotune: for every level and for the precisions the context's solvers
 * use, runs each candidate shape (rows 4/8/16, 4/1 or 4/1/2/3, group 0/1/2/4/8) of
 * each kernel kind `reps` times on the context's own work buffers (their contents are
 * overwritten; caller memory is not touched), times it with HIP events on
 * `stream` and keeps the fastest; the folded prolongation (rows = 2 or 3 of
 * GMG_K_PROLONG_SMOOTH, groups 0/1/2/4/8) is kept for a level where it beats
 * the best prolongation plus the best smoother.  Synchronises `stream`.
 * reps in [1, 1000]. */
int gmg_set_launch(gmg_ctx *c, int kernel, int level, int prec, int rows, int group);
int gmg_get_launch(const gmg_ctx *c, int kernel, int level, int prec, int *rows, int *group);
int gmg_autotune(gmg_ctx *c, int reps, void *stream);

/* Launch mode of the iterative solvers (gmg_solve, pcg_solve, and the solve
 * inside gmg_solve_host).  Their scalars and stopping test live on the device
 * and every kernel of an iteration returns at once after the solve has
 * stopped, so the host enqueues predicted batches of iterations and reads the
 * solver state only between batches (Algorithm 1's loop of Sec. 2.2 without a
 * host round trip per cycle).  enable = 1 (the default): each batch of the
 * multigrid, refinement and flexible-CG solves is replayed from a hipGraph of
 * one iteration (two for the refinement, whose iterate alternates between two
 * buffers, and for flexible CG, whose directions do; line-PCG's four-kernel
 * iteration is always launched directly),
 * captured on the context's own
 * stream at the first solve with a given pair of caller fields and kept until
 * gmg_destroy, a launch-shape change (gmg_set_launch, gmg_autotune) or
 * gmg_set_graphs(c, 0); at most 8 graphs per context.  enable = 0: the same
 * kernels launched one by one (iterations with a kernel kind being timed by
 * gmg_timing_* always are).  Results are bitwise identical either way. */
int gmg_set_graphs(gmg_ctx *c, int enable);

/* The number of times the last gmg_solve or pcg_solve on the context waited
 * for device scalars (a synchronisation of the stream), its final wait
 * included; GMG_EINVAL for a NULL or batched context. */
int gmg_solver_polls(const gmg_ctx *c);

/* Message describing the calling thread's last non-OK status. */
const char *gmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMG_H */
