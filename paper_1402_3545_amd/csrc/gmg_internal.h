// Internal declarations of the gfx950 library: device-side level views, the
// host context, and the kernel launchers shared by kernels.hip and gmg_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gmg.h"

namespace gmg {

// Device view of one level of the hierarchy in precision T.  Element (i,j,k)
// of a field lives at ((j*nz + k)*ldx + i).  Row (T,k) of the operator is
//   diag_k(T) u_k + sub_k u_{k-1} + sup_k u_{k+1}
//     - dz_k (ce u_E + cw u_W + cn u_N + cs u_S),
//   diag_k(T) = dg_k + dz_k (ce + cw + cn + cs),
// where ce/cn are the couplings through the east/north face of the column (cx,
// cy arrays, index j*nx+i) and cw/cs those through its west/south face (the
// east/north couplings of the neighbour).  sub_0 = sup_{nz-1} = 0.
template <typename T>
struct Lvl {
  int nx, ny, nz;
  int64_t ldx;
  const T* __restrict__ cx;
  const T* __restrict__ cy;
  const T* __restrict__ sub;
  const T* __restrict__ sup;
  const T* __restrict__ dg;
  const T* __restrict__ dz;
  // per column (j*nx + i): summed couplings of the column's Dirichlet wall
  // faces, added to the diagonal (all zero with periodic boundaries)
  const T* __restrict__ wall;
  int bch;  // 0 doubly periodic, 1 Dirichlet side walls (prolongation reflects)
  // device flag (a solver's "done"): kernels given a view with a gate return
  // at once while it is set, so iterations enqueued past convergence cost
  // only their launches and the host reads the solver state rarely
  const int* gate = nullptr;
};

// Scalars shared between the kernels of one CG solve; lives in device memory
// so that no iteration needs a host round trip.
struct CgState {
  double alpha, beta, kappa, sigma;  // step, direction update, <r,z>, <p,Ap>
  double rr, rr0, thresh2;           // ||r||^2, ||r_0||^2, rtol^2 ||r_0||^2
  int iter, done, maxit, status;     // status: 0 running/converged, 1 maxit,
                                     // 2 non-finite, 3 breakdown
  double rtol;                       // multigrid / refinement stopping test
  double alpha_prev;                 // line-PCG: the step before alpha
};

// One work item of a grouped launch: one kernel applied to one level of one
// (instance, right-hand side) pair.  Items of a launch are sorted by blk0, the
// item's first workgroup.
template <typename T>
struct GItem {
  Lvl<T> L;      // level the kernel works on (resrestrict, prolongate: the FINE level)
  Lvl<T> X;      // resrestrict, prolongate, prolong-smooth: the COARSE level
  const T* a;    // line: rhs (solve) or u (smooth); resrestrict: u; prolongate: u_c
  const T* b;    // smooth, resrestrict: f
  T* o;          // line: output; resrestrict: f_c; prolongate: u_f (updated)
  const T* c;    // prolong-smooth: u_c (a: u_f, b: f, o: the smoothed u_f + P u_c)
  int nti, ntj;  // tiles of the item
  int blk0;      // first workgroup of the item in its launch
  int pair;      // (instance, rhs) index: activity mask, partial-sum segment
};

// Grouped FP64 refinement step u' = u + e, r = f - A u' (FP32 copy), ||r||^2.
struct GItemCR {
  Lvl<double> L;
  const double* u;
  const float* e;
  const double* f;
  double* uout;
  float* r32;
  int nti, ntj, blk0, pair;
};

// Per-pair state of a batched solve (device).
struct PairState {
  double rr0, rr, thresh2;
  int iters, maxit, status;   // status: 0 converged / running, 1 maxit, 2 non-finite
  int blk0, nblk;             // partial-sum segment of the pair in the residual launch
};

// One multigrid level as owned by the context.
struct LevelBuf {
  int nx, ny, nz;
  int64_t ldx, elems;
  double area;
  double *cx64 = nullptr, *cy64 = nullptr, *sub64 = nullptr, *sup64 = nullptr,
         *dg64 = nullptr, *wall64 = nullptr;
  float *cx32 = nullptr, *cy32 = nullptr, *sub32 = nullptr, *sup32 = nullptr,
        *dg32 = nullptr, *wall32 = nullptr;
  // V-cycle work fields in the context's precond precision (bytes per
  // element = esize): u, ualt (ping-pong partner), f.  Level 0 uses the
  // caller's f and u, so only ualt is allocated there.  (The residual is
  // never stored: it is fused with the restriction.)
  void *u = nullptr, *ualt = nullptr, *f = nullptr;
};

// Launch shape of a kernel: rows = grid rows per workgroup of the stencil
// kernels (4, 8 or 16 wavefronts of 64 columns; the line kernels always use 4
// wavefronts of 32 columns), group = tile columns per dispatch group (tiles
// are walked group by group, tile rows inside a group; 0 = row-major order).
struct Shape {
  int rows = 4;
  int group = 0;
};

constexpr int kMaxLevels = 20;

// Slot of (kernel kind, level, precision) in the per-context tables.
inline size_t tslot(int kind, int level, int prec) {
  return ((size_t)kind * kMaxLevels + level) * 2 + prec;
}

}  // namespace gmg

struct gmg_timed_launch {
  int kind, level, prec;
  hipEvent_t a, b;
};

namespace gmg {
struct Batch;
}

// An instantiated hipGraph of a batch of one solver's iterations, for one
// pair of caller fields (their addresses are in the kernels' arguments).
struct gmg_graph {
  int kind;
  const void *f, *u;
  hipGraphExec_t exec;
};

struct gmg_ctx {
  gmg_params p;
  // the iterative solvers' iterations are enqueued as hipGraph replays
  // (gmg_set_graphs); graphs are cached per solver and caller fields and
  // dropped when a launch shape changes
  bool graphs_on = true;
  std::vector<gmg_graph> graphs;
  hipStream_t cap = nullptr;         // capture stream (non-blocking, default priority)
  // set while a solver enqueues its iterations: views then carry it as their
  // gate (the device "done" flag of the solver state)
  const int* gate = nullptr;
  int polls = 0;                     // host waits for device scalars in the last solve
  // launch shape per [kind][level][prec] (gmg::tslot), set by gmg_set_launch
  // or gmg_autotune; every context starts with the default shapes
  std::vector<gmg::Shape> shape =
      std::vector<gmg::Shape>((size_t)GMG_K_COUNT * gmg::kMaxLevels * 2);
  gmg::Batch* batch = nullptr;       // non-null: a batched context (gmg_batch_setup)
  // per-kernel timing (of the kernel kinds whose bit is set in timing_mask)
  bool timing = false;
  uint32_t timing_mask = ~0u;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<gmg_timed_launch> pending;
  // accumulated [kind][level][prec] -> (count, ms)
  std::vector<int64_t> tcount;
  std::vector<double> tms;
  std::vector<double> zf, kh;
  int nlevels = 0, nz = 0, esize = 8;
  double *dz64 = nullptr;
  float *dz32 = nullptr;
  std::vector<gmg::LevelBuf> lev;
  // finest-level FP64 solver vectors and FP32 IR vectors
  double *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr, *vt = nullptr;
  float *er32 = nullptr, *eu32 = nullptr;
  double *partials = nullptr;
  int64_t max_partials = 0;
  gmg::CgState* state = nullptr;     // device
  gmg::CgState* hstate = nullptr;    // pinned host mirror
  double* dhist = nullptr;           // device history buffer
  double* hhist = nullptr;           // its pinned host mirror (dhist_len values)
  int dhist_len = 0;
  double* hscal = nullptr;           // pinned host scalars
  // gmg_solve_host: z-contiguous staging and x-contiguous f, u (FP64, level
  // 0), allocated on first use
  double *hz = nullptr, *hf = nullptr, *hu = nullptr;
  // gmg_solve_host: two pinned host staging buffers of stage_bytes each and
  // the events of their last copies, allocated on first use
  void* stage[2] = {};
  hipEvent_t stage_ev[2] = {};
  size_t stage_bytes = 0;
};

namespace gmg {

template <typename T>
Lvl<T> view(const gmg_ctx* c, int d);

int setup_impl(const gmg_params* p, void* stream, gmg_ctx** out, bool fields);
// device address of the current device's static scratch array of the
// allocation-free entry point (looked up once per device; noalloc.hip)
int scratch_address(double** out);
int set_error(int code, const char* msg);
int validate_params(const gmg_params* p);
void batch_free(Batch* b);

// ---- launchers (kernels.hip); every launcher returns the hipError_t of the launch
enum class Stencil { SPMV = 0, RESIDUAL = 1, RESIDUAL_NORM = 2, RESIDUAL_NORM_DOWN = 3 };


template <typename T>
hipError_t launch_stencil(const Lvl<T>& L, Stencil mode, const T* x, const T* f, T* y,
                          float* ydown, double* partials, int64_t* nblocks, hipStream_t s, Shape sh = {});

template <typename T>
hipError_t launch_line_solve(const Lvl<T>& L, const T* r, T* z, hipStream_t s, Shape sh = {});

template <typename T>
hipError_t launch_smooth(const Lvl<T>& L, const T* f, const T* uin, T* uout, T rho,
                         hipStream_t s, Shape sh = {});
// uout = one Smooth of (uin + P uc) on F with right-hand side f: the V-cycle's
// prolongation from C folded into the post-smoother (staged form; sh.group
// is the tile order).  uin is read only; uout must not alias uin or uc.
template <typename T>
hipError_t launch_prolong_smooth(const Lvl<T>& F, const Lvl<T>& C, const T* f, const T* uin,
                                 const T* uc, T* uout, T rho, hipStream_t s, Shape sh = {});

template <typename T>
hipError_t launch_restrict_smooth(const Lvl<T>& C, const Lvl<T>& F, const T* rf, T* fc, T* uc,
                                  T rho, hipStream_t s, Shape sh = {});

// z = scale * M^-1 r (first smoothing step from a zero guess when scale = rho)
template <typename T>
hipError_t launch_line_solve_scaled(const Lvl<T>& L, const T* r, T* z, T scale, hipStream_t s, Shape sh = {});

// Smooth that also returns ||f - A u_in||^2 per workgroup (line_blocks partials)
template <typename T>
hipError_t launch_smooth_norm(const Lvl<T>& L, const T* f, const T* uin, T* uout, T rho,
                              double* partials, int64_t* nblocks, hipStream_t s, Shape sh = {});

// fc = R (f - A u): residual of level F restricted to level C, r never stored
template <typename T>
hipError_t launch_resrestrict(const Lvl<T>& F, const Lvl<T>& C, const T* u, const T* f, T* fc,
                              hipStream_t s, Shape sh = {});

// uout = u + e, r32 = f - A uout, partial ||r||^2
hipError_t launch_correct_residual(const Lvl<double>& L, const double* u, const float* e,
                                   const double* f, double* uout, float* r32, double* partials,
                                   int64_t* nblocks, hipStream_t s, Shape sh = {});

template <typename T>
hipError_t launch_prolongate(const Lvl<T>& C, const Lvl<T>& F, const T* uc, T* uf,
                             hipStream_t s, Shape sh = {});

// CG direction step: p_new = z + beta p_old, q = A z + beta q, <p_new, q>.
// p_old is read from pr and p_new written to pw (distinct buffers).
// paired: also u += alpha_prev pw_old + alpha pr (pw's old contents are the
// direction before p_old), the two pending steps of the iterate.
hipError_t launch_cg_p1(const Lvl<double>& L, double* u, const double* pr, double* pw,
                        const double* z, double* q, const CgState* st, bool paired,
                        double* partials, int64_t* nblocks, hipStream_t s, Shape sh = {});
hipError_t launch_cg_p2(const Lvl<double>& L, double* r, const double* q, double* z,
                        const CgState* st, int init, double* partials, int64_t* nblocks,
                        hipStream_t s, Shape sh = {});
// finalize kernels: reduce partials in a fixed order and update the CG state
hipError_t launch_cg_fin1(CgState* st, const double* partials, int64_t nblocks, hipStream_t s);
hipError_t launch_cg_fin2(CgState* st, const double* partials, int64_t nblocks, int init,
                          double* hist, hipStream_t s);
// line-PCG and flexible CG with paired updates: the steps of the
// directions not yet applied to u (direction j lives in p[j & 1])
hipError_t launch_pcg_final_update(const Lvl<double>& L, double* u, const double* p0,
                                   const double* p1, const CgState* st, hipStream_t s);
hipError_t launch_reduce(const double* partials, int64_t nblocks, int ncomp, double* out,
                         hipStream_t s);
// multigrid / refinement: ||f - A u||^2 from the partials -> relative
// residual, history, stopping test (init: the initial residual)
hipError_t launch_mg_fin(CgState* st, const double* partials, int64_t nblocks, int init,
                         double* hist, hipStream_t s);
// flexible CG (variable preconditioner)
template <typename TZ>
hipError_t launch_fcg_zq(const Lvl<double>& L, const TZ* z, const double* q, double* partials,
                         int64_t* nblocks, hipStream_t s);
// p_new = z + beta p_old (p_old from pr, p_new to pw, distinct buffers);
// q = A z + beta q; <p_new,q>, <p_new,r>; paired: also
// u += alpha_prev pw_old + alpha pr (the two pending steps of the iterate)
template <typename TZ>
hipError_t launch_fcg_dir(const Lvl<double>& L, const TZ* z, double* u, const double* pr,
                          double* pw, double* q, const double* r, const CgState* st, bool paired,
                          double* partials, int64_t* nblocks, hipStream_t s, Shape sh = {});
// r -= alpha q (+ FP32 copy), ||r||^2
hipError_t launch_fcg_update(const Lvl<double>& L, double* r, const double* q, float* rdown,
                             const CgState* st, double* partials, int64_t* nblocks,
                             hipStream_t s, Shape sh = {});
// which: 0 beta, 1 alpha, 2 residual / convergence
hipError_t launch_fcg_fin(int which, CgState* st, const double* partials, int64_t nblocks,
                          double* hist, hipStream_t s);

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
// dst = src over the field of level L (gated by L.gate)
template <typename T>
hipError_t launch_copy_level(const Lvl<T>& L, const T* src, T* dst, hipStream_t s);
// streaming copy of n doubles (bandwidth measurement)
hipError_t launch_copy_probe(const double* src, double* dst, int64_t n, hipStream_t s);
// canonical z-contiguous (j*nx+i)*nz+k <-> x-contiguous (j*nz+k)*ldx+i
template <typename T>
hipError_t launch_transpose(const T* src, T* dst, int nx, int ny, int nz, int64_t ldx,
                            bool to_x, hipStream_t s);
hipError_t launch_add_f32_to_f64(double* u, const float* e, int64_t n, hipStream_t s);

// grouped launches (batched solves)
enum class GKind { LINE_SOLVE = 0, SMOOTH = 1, RESRESTRICT = 2, PROLONGATE = 3, PROLONG_SMOOTH = 4 };
// exact: every item has columns of exactly 2 * half layers (32, 64 or 128)
hipError_t launch_grouped_f32(GKind kind, int half, bool exact, const GItem<float>* items,
                              int nitems, int nblocks, const int* active, float rho,
                              hipStream_t s);
hipError_t launch_grouped_cr(const GItemCR* items, int nitems, int nblocks, const int* active,
                             double* partials, hipStream_t s);
// one workgroup per pair: sum its partials, update its state and activity
hipError_t launch_pair_reduce(PairState* ps, int* active, const double* partials, int npairs,
                              int init, hipStream_t s);
// tiles of each kernel shape for a level of nx x ny x nz
int64_t line_tiles_x(int nx);
int64_t line_tiles_y(int ny);
int64_t stencil_tiles_x(int nx);
int64_t stencil_tiles_y(int ny);
int64_t stencil_tiles_k(int nz);

int64_t stencil_blocks(int nx, int ny, int nz);
int64_t line_blocks(int nx, int ny);

}  // namespace gmg
