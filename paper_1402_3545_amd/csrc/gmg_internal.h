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
};

// Scalars shared between the kernels of one CG solve; lives in device memory
// so that no iteration needs a host round trip.
struct CgState {
  double alpha, beta, kappa, sigma;  // step, direction update, <r,z>, <p,Ap>
  double rr, rr0, thresh2;           // ||r||^2, ||r_0||^2, rtol^2 ||r_0||^2
  int iter, done, maxit, status;     // status: 0 running/converged, 2 breakdown
};

// One multigrid level as owned by the context.
struct LevelBuf {
  int nx, ny, nz;
  int64_t ldx, elems;
  double area;
  double *cx64 = nullptr, *cy64 = nullptr, *sub64 = nullptr, *sup64 = nullptr,
         *dg64 = nullptr;
  float *cx32 = nullptr, *cy32 = nullptr, *sub32 = nullptr, *sup32 = nullptr,
        *dg32 = nullptr;
  // V-cycle work fields in the context's precond precision (bytes per
  // element = esize): u, ualt (ping-pong partner), f, r.  Level 0 uses the
  // caller's f and u, so only ualt and r are allocated there.
  void *u = nullptr, *ualt = nullptr, *f = nullptr, *r = nullptr;
};

}  // namespace gmg

struct gmg_timed_launch {
  int kind, level, prec;
  hipEvent_t a, b;
};

struct gmg_ctx {
  gmg_params p;
  // per-kernel timing
  bool timing = false;
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
  int dhist_len = 0;
  double* hscal = nullptr;           // pinned host scalars
};

namespace gmg {

template <typename T>
Lvl<T> view(const gmg_ctx* c, int d);

// ---- launchers (kernels.hip); every launcher returns the hipError_t of the launch
enum class Stencil { SPMV = 0, RESIDUAL = 1, RESIDUAL_NORM = 2, RESIDUAL_NORM_DOWN = 3 };

template <typename T>
hipError_t launch_stencil(const Lvl<T>& L, Stencil mode, const T* x, const T* f, T* y,
                          float* ydown, double* partials, int64_t* nblocks, hipStream_t s);

template <typename T>
hipError_t launch_line_solve(const Lvl<T>& L, const T* r, T* z, hipStream_t s);

template <typename T>
hipError_t launch_smooth(const Lvl<T>& L, const T* f, const T* uin, T* uout, T rho,
                         hipStream_t s);

template <typename T>
hipError_t launch_restrict_smooth(const Lvl<T>& C, const Lvl<T>& F, const T* rf, T* fc, T* uc,
                                  T rho, hipStream_t s);

template <typename T>
hipError_t launch_prolongate(const Lvl<T>& C, const Lvl<T>& F, const T* uc, T* uf,
                             hipStream_t s);

hipError_t launch_cg_p1(const Lvl<double>& L, double* u, double* p, const double* z, double* q,
                        const CgState* st, double* partials, int64_t* nblocks, hipStream_t s);
hipError_t launch_cg_p2(const Lvl<double>& L, double* r, const double* q, double* z,
                        const CgState* st, int init, double* partials, int64_t* nblocks,
                        hipStream_t s);
// finalize kernels: reduce partials in a fixed order and update the CG state
hipError_t launch_cg_fin1(CgState* st, const double* partials, int64_t nblocks, hipStream_t s);
hipError_t launch_cg_fin2(CgState* st, const double* partials, int64_t nblocks, int init,
                          double* hist, hipStream_t s);
hipError_t launch_cg_final_update(const Lvl<double>& L, double* u, const double* p,
                                  const CgState* st, hipStream_t s);
hipError_t launch_reduce(const double* partials, int64_t nblocks, int ncomp, double* out,
                         hipStream_t s);
// flexible CG (variable preconditioner)
template <typename TZ>
hipError_t launch_fcg_zq(const Lvl<double>& L, const TZ* z, const double* q, double* partials,
                         int64_t* nblocks, hipStream_t s);
template <typename TZ>
hipError_t launch_fcg_dir(const Lvl<double>& L, const TZ* z, double* p, double* q,
                          const double* r, const CgState* st, double* partials, int64_t* nblocks,
                          hipStream_t s);
hipError_t launch_fcg_update(const Lvl<double>& L, double* u, double* r, const double* p,
                             const double* q, float* rdown, const CgState* st, double* partials,
                             int64_t* nblocks, hipStream_t s);
// which: 0 beta, 1 alpha, 2 residual / convergence
hipError_t launch_fcg_fin(int which, CgState* st, const double* partials, int64_t nblocks,
                          double* hist, hipStream_t s);

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
hipError_t launch_add_f32_to_f64(double* u, const float* e, int64_t n, hipStream_t s);

int64_t stencil_blocks(int nx, int ny, int nz);
int64_t line_blocks(int nx, int ny);

}  // namespace gmg
