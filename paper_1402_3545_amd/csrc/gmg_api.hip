// C ABI of the gfx950 multigrid / line-CG library: context setup (vertical
// profiles, per-level face couplings, level hierarchy), the single-operation
// entry points and the solver drivers.  Every step of the path runs in the
// kernels of kernels.hip; this file only validates, allocates and enqueues.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <thread>
#include <vector>

#include <type_traits>

#include "gmg_internal.h"

using gmg::CgState;
using gmg::LevelBuf;
using gmg::Lvl;
using gmg::Stencil;

namespace {

thread_local char g_err[512];

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(GMG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

template <typename T>
hipError_t dmalloc(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool level_ok(const gmg_ctx* c, int level) {
  return c && !c->batch && level >= 0 && level < c->nlevels;
}

int validate(const gmg_params* p) {
  if (!p) return fail(GMG_EINVAL, "params is NULL");
  if (p->nlevels < 1 || p->nlevels > 20) return fail(GMG_EINVAL, "nlevels must be in [1, 20]");
  if (p->nx < 2 || p->ny < 2) return fail(GMG_EINVAL, "nx, ny must be >= 2");
  if (p->nz < 2) return fail(GMG_EINVAL, "nz must be >= 2");
  if (p->nz > 128) return fail(GMG_EUNSUPPORTED, "nz > 128 is not supported (nz = %d)", p->nz);
  const int64_t div = int64_t(1) << (p->nlevels - 1);
  if (p->nx % div || p->ny % div)
    return fail(GMG_EINVAL, "nx=%d, ny=%d must be divisible by 2^(nlevels-1)=%lld", p->nx,
                p->ny, (long long)div);
  if (p->bc_h != 0 && p->bc_h != 1) return fail(GMG_EINVAL, "bc_h must be 0 or 1");
  if (p->bc_v != 0 && p->bc_v != 1) return fail(GMG_EINVAL, "bc_v must be 0 or 1");
  if (!(p->kv >= 0.0) || !isfinite(p->kv)) return fail(GMG_EINVAL, "kv must be finite, >= 0");
  if (!(p->sigma > 0.0) || !isfinite(p->sigma)) return fail(GMG_EINVAL, "sigma must be > 0");
  if (!(p->rho > 0.0) || !(p->rho <= 2.0)) return fail(GMG_EINVAL, "rho must be in (0, 2]");
  if (p->ncoarse < 1) return fail(GMG_EINVAL, "ncoarse must be >= 1");
  if (p->prec_precond != GMG_F64 && p->prec_precond != GMG_F32)
    return fail(GMG_EINVAL, "prec_precond must be GMG_F64 or GMG_F32");
  if (p->zfaces) {
    if (!isfinite(p->zfaces[0])) return fail(GMG_EINVAL, "zfaces must be finite");
    for (int k = 0; k < p->nz; ++k)
      if (!(p->zfaces[k + 1] > p->zfaces[k]) || !isfinite(p->zfaces[k + 1]))
        return fail(GMG_EINVAL, "zfaces must be finite and strictly increasing");
  }
  if (p->kh) {
    const int64_t nc = (int64_t)p->nx * p->ny;
    for (int64_t q = 0; q < nc; ++q)
      if (!(p->kh[q] > 0.0) || !isfinite(p->kh[q]))
        return fail(GMG_EINVAL, "kh must be finite and > 0 (column %lld)", (long long)q);
  }
  return GMG_OK;
}

template <typename T>
int upload(T** dst, const std::vector<double>& src) {
  std::vector<T> tmp(src.begin(), src.end());
  HIP_TRY(dmalloc(dst, tmp.size()));
  HIP_TRY(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return GMG_OK;
}

}  // namespace

namespace gmg {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
int validate_params(const gmg_params* p) { return validate(p); }

template <>
Lvl<double> view<double>(const gmg_ctx* c, int d) {
  const LevelBuf& L = c->lev[d];
  return Lvl<double>{L.nx,    L.ny,    L.nz,  L.ldx,    L.cx64,    L.cy64,
                     L.sub64, L.sup64, L.dg64, c->dz64, L.wall64, c->p.bc_h, c->gate};
}

template <>
Lvl<float> view<float>(const gmg_ctx* c, int d) {
  const LevelBuf& L = c->lev[d];
  return Lvl<float>{L.nx,    L.ny,    L.nz,  L.ldx,    L.cx32,    L.cy32,
                    L.sub32, L.sup32, L.dg32, c->dz32, L.wall32, c->p.bc_h, c->gate};
}

}  // namespace gmg

extern "C" {

const char* gmg_last_error(void) { return g_err; }

void gmg_default_params(gmg_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->nlevels = 1;
  p->kv = 1.0;
  p->sigma = 1.0;
  p->rho = 2.0 / 3.0;
  p->ncoarse = 2;
  p->prec_precond = GMG_F64;
}

int gmg_destroy(gmg_ctx* c) {
  if (!c) return GMG_OK;
  if (c->batch) gmg::batch_free(c->batch);
  for (LevelBuf& L : c->lev) {
    dfree(L.cx64); dfree(L.cy64); dfree(L.sub64); dfree(L.sup64); dfree(L.dg64);
    dfree(L.cx32); dfree(L.cy32); dfree(L.sub32); dfree(L.sup32); dfree(L.dg32);
    dfree(L.wall64); dfree(L.wall32);
    if (L.u) (void)hipFree(L.u);
    if (L.ualt) (void)hipFree(L.ualt);
    if (L.f) (void)hipFree(L.f);
  }
  dfree(c->dz64); dfree(c->dz32);
  dfree(c->vr); dfree(c->vz); dfree(c->vp); dfree(c->vq); dfree(c->vt);
  dfree(c->er32); dfree(c->eu32);
  dfree(c->hz); dfree(c->hf); dfree(c->hu);
  for (int b = 0; b < 2; ++b) {
    if (c->stage[b]) (void)hipHostFree(c->stage[b]);
    if (c->stage_ev[b]) (void)hipEventDestroy(c->stage_ev[b]);
  }
  dfree(c->partials);
  dfree(c->state);
  dfree(c->dhist);
  if (c->hhist) (void)hipHostFree(c->hhist);
  if (c->hstate) (void)hipHostFree(c->hstate);
  if (c->hscal) (void)hipHostFree(c->hscal);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  for (gmg_graph& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return GMG_OK;
}

int gmg_setup(const gmg_params* p, void* stream, gmg_ctx** out) {
  return gmg::setup_impl(p, stream, out, true);
}

}  // extern "C"

// Context construction; with fields = false only the coefficients (profiles,
// face couplings) and small scratch are built -- the batched solver owns the
// fields of its instances itself.
int gmg::setup_impl(const gmg_params* p, void* stream, gmg_ctx** out, bool fields) {
  if (!out) return fail(GMG_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate(p);
  if (st) return st;
  gmg_ctx* c = new (std::nothrow) gmg_ctx();
  if (!c) return fail(GMG_ENOMEM, "host allocation failed");
  c->p = *p;
  c->nlevels = p->nlevels;
  const int nz = c->nz = p->nz;
  c->esize = p->prec_precond == GMG_F32 ? 4 : 8;
  c->zf.resize(nz + 1);
  for (int k = 0; k <= nz; ++k)
    c->zf[k] = p->zfaces ? p->zfaces[k] : ((double)k / nz) * ((double)k / nz);
  c->p.zfaces = nullptr;
  c->p.kh = nullptr;

  // vertical profiles: layer thickness, face transmissibilities (Sec. 3.1: the
  // vectors a, b, c, d are shared by every column and level)
  std::vector<double> dz(nz), tf(nz + 1);
  for (int k = 0; k < nz; ++k) dz[k] = c->zf[k + 1] - c->zf[k];
  for (int k = 1; k < nz; ++k) {
    const double lo = 0.5 * (c->zf[k - 1] + c->zf[k]);
    const double hi = 0.5 * (c->zf[k] + c->zf[k + 1]);
    tf[k] = p->kv / (hi - lo);
  }
  tf[0] = p->bc_v == 0 ? 2.0 * p->kv / dz[0] : 0.0;
  tf[nz] = p->bc_v == 0 ? 2.0 * p->kv / dz[nz - 1] : 0.0;

  auto cleanup = [&](int code) { gmg_destroy(c); return code; };
  if ((st = upload(&c->dz64, dz)) || (st = upload(&c->dz32, dz))) return cleanup(st);

  // per-level column coefficients: K of the finest level from the caller, the
  // mean of the four children on coarser levels; harmonic face means
  std::vector<double> K((size_t)p->nx * p->ny, 1.0);
  if (p->kh) std::copy(p->kh, p->kh + K.size(), K.begin());
  c->lev.resize(c->nlevels);
  for (int d = 0; d < c->nlevels; ++d) {
    LevelBuf& L = c->lev[d];
    L.nx = p->nx >> d;
    L.ny = p->ny >> d;
    L.nz = nz;
    L.ldx = round_up(L.nx, 32);
    L.elems = (int64_t)L.ny * nz * L.ldx;
    const double hx = 1.0 / L.nx, hy = 1.0 / L.ny;
    L.area = hx * hy;
    if (d > 0) {
      const int fnx = c->lev[d - 1].nx;
      std::vector<double> Kc((size_t)L.nx * L.ny);
      for (int J = 0; J < L.ny; ++J)
        for (int I = 0; I < L.nx; ++I) {
          const double s = K[(size_t)(2 * J) * fnx + 2 * I] + K[(size_t)(2 * J) * fnx + 2 * I + 1] +
                           K[(size_t)(2 * J + 1) * fnx + 2 * I] +
                           K[(size_t)(2 * J + 1) * fnx + 2 * I + 1];
          Kc[(size_t)J * L.nx + I] = 0.25 * s;
        }
      K.swap(Kc);
    }
    // Dirichlet side walls (Sec. 2.1.1): no face crosses the domain edge (the
    // wrap-around couplings are zero, so the kernels' periodic neighbour reads
    // contribute nothing), and each wall face, half a cell from the column
    // centre, couples the column to the zero wall value with 2 K times the
    // face ratio -- a diagonal-only term kept per column.
    const bool walls = p->bc_h == 1;
    std::vector<double> cx(K.size()), cy(K.size()), wall(K.size(), 0.0);
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i) {
        const size_t q = (size_t)j * L.nx + i;
        const double kc = K[q];
        const double ke = K[(size_t)j * L.nx + (i + 1) % L.nx];
        const double kn = K[(size_t)((j + 1) % L.ny) * L.nx + i];
        cx[q] = (walls && i == L.nx - 1) ? 0.0 : (hy / hx) * 2.0 * kc * ke / (kc + ke);
        cy[q] = (walls && j == L.ny - 1) ? 0.0 : (hx / hy) * 2.0 * kc * kn / (kc + kn);
        // a periodic level one column wide is its own neighbour: the flux
        // through those faces vanishes identically, and leaving the coupling
        // in would move a self term out of the column block M into A - M,
        // which changes the line smoother
        if (L.nx == 1) cx[q] = 0.0;
        if (L.ny == 1) cy[q] = 0.0;
        if (walls) {
          const int nwx = (i == 0) + (i == L.nx - 1), nwy = (j == 0) + (j == L.ny - 1);
          wall[q] = nwx * (hy / hx) * 2.0 * kc + nwy * (hx / hy) * 2.0 * kc;
        }
      }
    std::vector<double> sub(nz), sup(nz), dg(nz);
    for (int k = 0; k < nz; ++k) {
      sub[k] = k > 0 ? -L.area * tf[k] : 0.0;
      sup[k] = k < nz - 1 ? -L.area * tf[k + 1] : 0.0;
      dg[k] = L.area * (p->sigma * dz[k] + tf[k] + tf[k + 1]);
    }
    if ((st = upload(&L.cx64, cx)) || (st = upload(&L.cy64, cy)) || (st = upload(&L.sub64, sub)) ||
        (st = upload(&L.sup64, sup)) || (st = upload(&L.dg64, dg)) || (st = upload(&L.cx32, cx)) ||
        (st = upload(&L.cy32, cy)) || (st = upload(&L.sub32, sub)) ||
        (st = upload(&L.sup32, sup)) || (st = upload(&L.dg32, dg)) ||
        (st = upload(&L.wall64, wall)) || (st = upload(&L.wall32, wall)))
      return cleanup(st);
    const size_t bytes = (size_t)L.elems * c->esize;
    hipError_t e = hipSuccess;
    if (!fields) continue;
    if (d > 0) {
      if ((e = hipMalloc(&L.u, bytes)) != hipSuccess || (e = hipMalloc(&L.f, bytes)) != hipSuccess)
        return cleanup(fail(GMG_ENOMEM, "level %d fields: %s", d, hipGetErrorString(e)));
    }
    if ((e = hipMalloc(&L.ualt, bytes)) != hipSuccess)
      return cleanup(fail(GMG_ENOMEM, "level %d fields: %s", d, hipGetErrorString(e)));
  }
  const int64_t n0 = c->lev[0].elems;
  hipError_t e;
  if (fields && ((e = dmalloc(&c->vr, n0)) || (e = dmalloc(&c->vz, n0)) ||
                 (e = dmalloc(&c->vp, n0)) || (e = dmalloc(&c->vq, n0)) ||
                 (e = dmalloc(&c->vt, n0))))
    return cleanup(fail(GMG_ENOMEM, "solver vectors: %s", hipGetErrorString(e)));
  if (fields && p->prec_precond == GMG_F32) {
    if ((e = dmalloc(&c->er32, n0)) || (e = dmalloc(&c->eu32, n0)))
      return cleanup(fail(GMG_ENOMEM, "FP32 vectors: %s", hipGetErrorString(e)));
  }
  const LevelBuf& L0 = c->lev[0];
  c->max_partials = 2 * std::max(gmg::stencil_blocks(L0.nx, L0.ny, nz),
                                 gmg::line_blocks(L0.nx, L0.ny));
  if ((e = dmalloc(&c->partials, c->max_partials + 8)) ||  // + scalar slots
      (e = dmalloc(&c->state, 1)) ||
      (e = hipHostMalloc((void**)&c->hstate, sizeof(CgState), hipHostMallocDefault)) ||
      (e = hipHostMalloc((void**)&c->hscal, 8 * sizeof(double), hipHostMallocDefault)))
    return cleanup(fail(GMG_ENOMEM, "scratch: %s", hipGetErrorString(e)));
  // zero-fill the level fields once so that padding never holds NaN patterns
  hipStream_t s = as_stream(stream);
  for (int d = 0; d < c->nlevels; ++d) {
    LevelBuf& L = c->lev[d];
    for (void* q : {L.u, L.ualt, L.f})
      if (q && (e = hipMemsetAsync(q, 0, (size_t)L.elems * c->esize, s)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMemsetAsync"));
  }
  for (double* q : {c->vr, c->vz, c->vp, c->vq, c->vt})
    if (q && (e = hipMemsetAsync(q, 0, (size_t)n0 * 8, s)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemsetAsync"));
  for (float* q : {c->er32, c->eu32})
    if (q && (e = hipMemsetAsync(q, 0, (size_t)n0 * 4, s)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemsetAsync"));
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup(hip_fail(e, "setup sync"));
  // this device's static scratch of the allocation-free residual (once per device)
  if ((st = gmg::scratch_address(nullptr))) return cleanup(st);
  *out = c;
  return GMG_OK;
}

extern "C" {

int gmg_field_layout(const gmg_ctx* c, int level, int64_t* ldx, int64_t* elems) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  if (ldx) *ldx = c->lev[level].ldx;
  if (elems) *elems = c->lev[level].elems;
  return GMG_OK;
}

}  // extern "C"

namespace {

int check_prec(int prec) {
  if (prec != GMG_F64 && prec != GMG_F32) return fail(GMG_EINVAL, "prec must be 0 or 1");
  return GMG_OK;
}

int check_ptrs(std::initializer_list<const void*> ps) {
  for (const void* q : ps) {
    if (!q) return fail(GMG_EINVAL, "NULL field pointer");
    if (reinterpret_cast<uintptr_t>(q) % 16)
      return fail(GMG_EINVAL, "field pointer not 16-byte aligned");
  }
  return GMG_OK;
}

template <typename T>
constexpr int prec_of() {
  return sizeof(T) == 8 ? GMG_F64 : GMG_F32;
}

hipEvent_t pool_event(gmg_ctx* c) {
  if (c->evused == c->evpool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->evpool.push_back(e);
  }
  return c->evpool[c->evused++];
}

// Enqueue one kernel launch; while timing is on, bracket it by two events on
// the launch stream.
// A launcher that takes a gmg::Shape gets the context's launch shape of
// (kind, level, prec).
template <typename F>
hipError_t timed(gmg_ctx* c, int kind, int level, int prec, hipStream_t s, F&& launch) {
  auto go = [&]() -> hipError_t {
    if constexpr (std::is_invocable_v<F, gmg::Shape>)
      return launch(c->shape[gmg::tslot(kind, level, prec)]);
    else
      return launch();
  };
  if (!c->timing || !((c->timing_mask >> kind) & 1u)) return go();
  hipEvent_t a = pool_event(c), b = pool_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  if ((e = go()) != hipSuccess) return e;
  if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
  c->pending.push_back({kind, level, prec, a, b});
  return hipSuccess;
}

int drain_timing(gmg_ctx* c) {
  for (const gmg_timed_launch& t : c->pending) {
    HIP_TRY(hipEventSynchronize(t.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    const size_t q = gmg::tslot(t.kind, t.level, t.prec);
    c->tcount[q] += 1;
    c->tms[q] += ms;
  }
  c->pending.clear();
  c->evused = 0;
  return GMG_OK;
}

// nsweeps smoothing steps on level d with the field pair (cur, other); the
// buffer holding the result goes to *result.
template <typename T>
hipError_t smooth_steps(gmg_ctx* c, int d, const T* f, T* cur, T* other, int n, T rho,
                        hipStream_t s, T** result) {
  const Lvl<T> L = gmg::view<T>(c, d);
  for (int q = 0; q < n; ++q) {
    hipError_t e = timed(c, GMG_K_SMOOTH, d, prec_of<T>(), s,
                         [&](gmg::Shape sh) { return gmg::launch_smooth<T>(L, f, cur, other, rho, s, sh); });
    if (e != hipSuccess) return e;
    std::swap(cur, other);
  }
  *result = cur;
  return hipSuccess;
}

// One V(1,1) cycle of Algorithm 1 in precision T on the caller's (f0, u0).
//  zero_guess:  u0 is taken as 0 (its content is not read); the first
//               smoothing step is then rho M^-1 f0, a scaled line solve.
//  presmoothed: the caller has already put the finest level's pre-smoothed
//               iterate into lev[0].ualt (see the multigrid solve, which
//               takes its convergence norm from that smoothing step).
// The fine-level residual is fused with the restriction (f_c = R(f - A u),
// the residual itself is never stored), so each coarse level starts with the
// scaled line solve u_c = rho M_c^-1 f_c: the values of ResSmooth.
template <typename T>
int vcycle_impl(gmg_ctx* c, const T* f0, T* u0, hipStream_t s, bool zero_guess = false,
                bool presmoothed = false) {
  const int L = c->nlevels;
  const int P = prec_of<T>();
  const T rho = (T)c->p.rho;
  std::vector<T*> cur(L, nullptr);
  std::vector<const T*> fl(L, nullptr);
  fl[0] = f0;
  for (int d = 1; d < L; ++d) fl[d] = static_cast<const T*>(c->lev[d].f);
  T* ualt0 = static_cast<T*>(c->lev[0].ualt);
  const Lvl<T> V0 = gmg::view<T>(c, 0);
  // finest-level pre-smoothing into ualt0
  int pre_done = 0;
  if (presmoothed) {
    pre_done = 1;
  } else if (zero_guess) {
    HIP_TRY(timed(c, GMG_K_LINE_SOLVE, 0, P, s,
                  [&](gmg::Shape sh) { return gmg::launch_line_solve_scaled<T>(V0, f0, ualt0, rho, s, sh); }));
    pre_done = 1;
  }
  if (L == 1) {
    T* res = nullptr;
    T* from = pre_done ? ualt0 : u0;
    T* other = pre_done ? u0 : ualt0;
    HIP_TRY(smooth_steps<T>(c, 0, f0, from, other, c->p.ncoarse - pre_done, rho, s, &res));
    if (res != u0)
      HIP_TRY(timed(c, GMG_K_AUX, 0, P, s,
                    [&] { return gmg::launch_copy_level<T>(V0, res, u0, s); }));
    return GMG_OK;
  }
  if (!pre_done)
    HIP_TRY(timed(c, GMG_K_SMOOTH, 0, P, s,
                  [&](gmg::Shape sh) { return gmg::launch_smooth<T>(V0, f0, u0, ualt0, rho, s, sh); }));
  cur[0] = ualt0;
  // descend
  for (int d = 0; d < L; ++d) {
    const Lvl<T> V = gmg::view<T>(c, d);
    LevelBuf& B = c->lev[d];
    if (d > 0) {
      HIP_TRY(timed(c, GMG_K_LINE_SOLVE, d, P, s, [&](gmg::Shape sh) {
        return gmg::launch_line_solve_scaled<T>(V, fl[d], static_cast<T*>(B.u), rho, s, sh);
      }));
      cur[d] = static_cast<T*>(B.u);
    }
    if (d == L - 1) {
      T* other = cur[d] == B.u ? static_cast<T*>(B.ualt) : static_cast<T*>(B.u);
      HIP_TRY(smooth_steps<T>(c, d, fl[d], cur[d], other, c->p.ncoarse - 1, rho, s, &cur[d]));
    } else {
      const Lvl<T> C = gmg::view<T>(c, d + 1);
      T* fc = static_cast<T*>(c->lev[d + 1].f);
      HIP_TRY(timed(c, GMG_K_RESIDUAL_RESTRICT, d, P, s, [&](gmg::Shape sh) {
        return gmg::launch_resrestrict<T>(V, C, cur[d], fl[d], fc, s, sh);
      }));
    }
  }
  // ascend: add the prolongated correction, post-smooth
  for (int d = L - 2; d >= 0; --d) {
    const Lvl<T> V = gmg::view<T>(c, d);
    const Lvl<T> C = gmg::view<T>(c, d + 1);
    T* other = (d == 0) ? u0
                        : (cur[d] == c->lev[d].u ? static_cast<T*>(c->lev[d].ualt)
                                                 : static_cast<T*>(c->lev[d].u));
    const int fold = c->shape[gmg::tslot(GMG_K_PROLONG_SMOOTH, d, P)].rows;
    if (fold == 2 || fold == 3) {
      // one kernel: smooth u + P u_c without storing it
      HIP_TRY(timed(c, GMG_K_PROLONG_SMOOTH, d, P, s, [&](gmg::Shape sh) {
        return gmg::launch_prolong_smooth<T>(V, C, fl[d], cur[d], cur[d + 1], other, rho, s, sh);
      }));
    } else {
      HIP_TRY(timed(c, GMG_K_PROLONGATE, d + 1, P, s, [&](gmg::Shape sh) {
        return gmg::launch_prolongate<T>(C, V, cur[d + 1], cur[d], s, sh);
      }));
      HIP_TRY(timed(c, GMG_K_SMOOTH, d, P, s, [&](gmg::Shape sh) {
        return gmg::launch_smooth<T>(V, fl[d], cur[d], other, rho, s, sh);
      }));
    }
    cur[d] = other;
  }
  return GMG_OK;
}

template <typename T>
int line_smooth_t(gmg_ctx* c, int level, const T* f, T* u, int nsweeps, T rho, hipStream_t s) {
  // ping-pong through a context buffer of the same precision and level
  T* tmp = nullptr;
  const LevelBuf& B = c->lev[level];
  const bool own = (c->esize == (int)sizeof(T));
  if (own)
    tmp = static_cast<T*>(B.ualt);
  else
    HIP_TRY(hipMallocAsync((void**)&tmp, (size_t)B.elems * sizeof(T), s));
  T* res = nullptr;
  HIP_TRY(smooth_steps<T>(c, level, f, u, tmp, nsweeps, rho, s, &res));
  if (res != u)
    HIP_TRY(hipMemcpyAsync(u, res, (size_t)B.elems * sizeof(T), hipMemcpyDeviceToDevice, s));
  if (!own) HIP_TRY(hipFreeAsync(tmp, s));
  return GMG_OK;
}

// r = f - A u on level 0 with ||r||^2 into *out (host), synchronising.  With
// rdown the residual is also written as FP32.
template <typename T>
int residual_norm2(gmg_ctx* c, const T* f, const T* u, T* r, float* rdown, double* out,
                   hipStream_t s) {
  const Lvl<T> V = gmg::view<T>(c, 0);
  int64_t nb = 0;
  double* dst = c->partials + c->max_partials;
  HIP_TRY(timed(c, GMG_K_RESIDUAL, 0, prec_of<T>(), s, [&](gmg::Shape sh) {
    return gmg::launch_stencil<T>(
        V, rdown ? Stencil::RESIDUAL_NORM_DOWN : Stencil::RESIDUAL_NORM, u, f, r, rdown,
        c->partials, &nb, s, sh);
  }));
  HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, s,
                [&] { return gmg::launch_reduce(c->partials, nb, 1, dst, s); }));
  HIP_TRY(hipMemcpyAsync(c->hscal, dst, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  ++c->polls;
  *out = c->hscal[0];
  return GMG_OK;
}

// How many iterations to enqueue before the host reads the device state
// again: the count still needed at the slower of the mean decay rate of
// ||r||^2 so far and its rate since the previous read (multigrid converges
// faster in its first cycles), plus one, clamped to [1, 32]; doubling from
// the previous batch until two iterations have run.  Iterations enqueued past
// convergence return at once, so a low guess costs one more read and a high
// one a few empty launches.
int predicted_chunk(const CgState& h, int it_prev, double rr_prev, int prev) {
  if (h.iter < 2 || !(h.rr > 0.0) || !(h.rr < h.rr0)) return std::min(2 * prev, 32);
  const double need = log(h.thresh2 / h.rr);       // < 0 until converged
  if (!(need < 0.0)) return 1;
  double rate = log(h.rr / h.rr0) / h.iter;        // < 0
  if (it_prev >= 1 && h.iter > it_prev && rr_prev > 0.0 && h.rr < rr_prev)
    rate = std::max(rate, log(h.rr / rr_prev) / (h.iter - it_prev));
  return (int)std::min(32.0, std::max(1.0, ceil(need / rate) + 1.0));
}

int ensure_hist(gmg_ctx* c, int maxit) {
  if (c->dhist_len < maxit + 1) {
    dfree(c->dhist);
    if (c->hhist) (void)hipHostFree(c->hhist);
    c->hhist = nullptr;
    c->dhist_len = 0;
    HIP_TRY(dmalloc(&c->dhist, (size_t)maxit + 1));
    HIP_TRY(hipHostMalloc((void**)&c->hhist, ((size_t)maxit + 1) * sizeof(double),
                          hipHostMallocDefault));
    c->dhist_len = maxit + 1;
  }
  return GMG_OK;
}

// ---- device-side iteration loops --------------------------------------------
// The iterative solvers keep their scalars and stopping test on the device
// (CgState) and every kernel of an iteration is gated on its "done" flag, so
// iterations enqueued past convergence return at once.  The host enqueues
// predicted batches of iterations -- one hipGraph replay per `per`
// iterations, unless graphs are off or one of the iteration's kernel kinds is
// being timed -- and reads the state only after each batch.

enum GraphKind { GK_MG = 0, GK_IR = 1, GK_FCG = 2, GK_FCG_LINE = 3, GK_PCG = 4 };

constexpr uint32_t kbit(int k) { return 1u << k; }
// kernel kinds one iteration of each loop launches
constexpr uint32_t kVcycleKinds = kbit(GMG_K_LINE_SOLVE) | kbit(GMG_K_SMOOTH) |
                                  kbit(GMG_K_RESIDUAL_RESTRICT) | kbit(GMG_K_PROLONGATE) |
                                  kbit(GMG_K_PROLONG_SMOOTH) | kbit(GMG_K_REDUCE) |
                                  kbit(GMG_K_AUX);
constexpr uint32_t kIrKinds = kVcycleKinds | kbit(GMG_K_CORRECT);
constexpr uint32_t kFcgKinds = kVcycleKinds | kbit(GMG_K_FCG);
constexpr uint32_t kPcgKinds = kbit(GMG_K_CG_SPMV) | kbit(GMG_K_CG_TRIDIAG) | kbit(GMG_K_REDUCE);

// Views built while this lives carry the solver state's "done" flag as gate.
struct GateScope {
  gmg_ctx* c;
  explicit GateScope(gmg_ctx* cc) : c(cc) { c->gate = &c->state->done; }
  ~GateScope() { c->gate = nullptr; }
};

void drop_graphs(gmg_ctx* c) {
  for (gmg_graph& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// The cached graph of `per` iterations of solver `kind` on the caller's
// fields (fk, uk), captured on the context's own stream at first use.
template <typename U>
int graph_for(gmg_ctx* c, int kind, const void* fk, const void* uk, int per, U&& unit,
              hipGraphExec_t* out) {
  for (const gmg_graph& g : c->graphs)
    if (g.kind == kind && g.f == fk && g.u == uk) {
      *out = g.exec;
      return GMG_OK;
    }
  if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  const bool timing = c->timing;
  c->timing = false;  // no event records inside a graph
  int st = GMG_OK;
  for (int r = 0; r < per && !st; ++r) st = unit(c->cap, r);
  c->timing = timing;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (st || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st ? st : hip_fail(e, "hipStreamEndCapture");
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
  if (c->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({kind, fk, uk, x});
  *out = x;
  return GMG_OK;
}

// Enqueue iterations (unit(stream, r) enqueues one; r = index within a group
// of `per`, for solvers whose iterate alternates between two buffers) in
// predicted batches until the device state is done or `maxit` iterations
// have been enqueued; `first` iterations go before the first read.  The
// caller has enqueued the initialisation (which may already set done).  On
// return c->hstate holds the final state.
template <typename U>
int run_iterations(gmg_ctx* c, hipStream_t s, int kind, const void* fk, const void* uk,
                   uint32_t kinds, int maxit, int per, int first, U&& unit) {
  hipGraphExec_t exec = nullptr;
  // line-PCG's iteration is four kernels: replaying it from a graph measured
  // slower than launching them (0.50 against 0.46 ms for the ten iterations
  // of the 64^3 workload, the same at 1024^2 x 128)
  const bool eager = !c->graphs_on || kind == GK_PCG || (c->timing && (c->timing_mask & kinds));
  if (!eager && maxit > 0) {
    const int st = graph_for(c, kind, fk, uk, per, unit, &exec);
    if (st) return st;
  }
  int launched = 0, chunk = first, it_prev = 0;
  double rr_prev = 0.0;
  for (;;) {
    const int nq = (std::min(chunk, maxit - launched) + per - 1) / per * per;
    for (int q = 0; q < nq; q += per) {
      if (exec) {
        HIP_TRY(hipGraphLaunch(exec, s));
      } else {
        for (int r = 0; r < per; ++r) {
          const int st = unit(s, r);
          if (st) return st;
        }
      }
    }
    launched += std::max(nq, 0);
    HIP_TRY(hipMemcpyAsync(c->hstate, c->state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    // the history so far rides along (pinned mirror), so reading it at the
    // end needs no further wait
    HIP_TRY(hipMemcpyAsync(c->hhist, c->dhist, (size_t)(std::max(maxit, 0) + 1) * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    ++c->polls;
    if (c->hstate->done || launched >= maxit) break;
    chunk = predicted_chunk(*c->hstate, it_prev, rr_prev, chunk);
    it_prev = c->hstate->iter;
    rr_prev = c->hstate->rr;
  }
  return GMG_OK;
}

// Flexible CG preconditioned by one V-cycle of precision TZ per iteration
// (TZ = float: the FP32 cycle runs on an FP32 copy of the FP64 residual and
// its FP32 correction enters the FP64 recurrences directly).
template <typename TZ>
int fcg_impl(gmg_ctx* c, const double* f, double* u, double rtol, int maxit, int* iters,
             double* relres, double* history, hipStream_t s, bool line_only = false) {
  const bool mixed = sizeof(TZ) == 4;
  const Lvl<double> V = gmg::view<double>(c, 0);
  const int64_t n0 = c->lev[0].elems;
  int st;
  if ((st = ensure_hist(c, maxit))) return st;
  double rr0 = 0.0;
  if ((st = residual_norm2<double>(c, f, u, c->vr, mixed ? c->er32 : nullptr, &rr0, s))) return st;
  if (iters) *iters = 0;
  if (relres) *relres = rr0 > 0.0 ? 1.0 : 0.0;
  if (history) history[0] = 1.0;
  if (!isfinite(rr0)) return fail(GMG_ENOCONV, "initial residual is not finite");
  if (rr0 == 0.0) return GMG_OK;
  CgState init{};
  init.maxit = maxit;
  init.rr0 = rr0;
  init.rr = rr0;
  init.thresh2 = rtol * rtol * rr0;
  init.sigma = 1.0;
  const double one = 1.0;
  HIP_TRY(hipMemcpyAsync(c->state, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->dhist, &one, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s,
                [&] { return gmg::launch_fill<double>(c->vp, n0, 0.0, s); }));
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s,
                [&] { return gmg::launch_fill<double>(c->vq, n0, 0.0, s); }));
  TZ* z = mixed ? reinterpret_cast<TZ*>(c->eu32) : reinterpret_cast<TZ*>(c->vz);
  const TZ* rin = mixed ? reinterpret_cast<const TZ*>(c->er32) : reinterpret_cast<const TZ*>(c->vr);
  {
    GateScope gate(c);
    // one iteration; every kernel returns at once once the state is done.
    // Direction i goes to buffer i & 1 (vp, vt); odd iterations leave u
    // alone, even ones apply the two pending steps.
    auto unit = [&](hipStream_t q, int ri) -> int {
      const Lvl<TZ> VZg = gmg::view<TZ>(c, 0);
      const Lvl<double> Vg = gmg::view<double>(c, 0);
      if (line_only) {
        // the vertical line preconditioner alone, in the preconditioner's
        // precision: z = M^-1 r (on the FP32 copy of r in mixed precision)
        HIP_TRY(timed(c, GMG_K_LINE_SOLVE, 0, prec_of<TZ>(), q, [&](gmg::Shape sh) {
          return gmg::launch_line_solve_scaled<TZ>(VZg, rin, z, TZ(1), q, sh);
        }));
      } else {
        const int sv = vcycle_impl<TZ>(c, rin, z, q, true, false);
        if (sv) return sv;
      }
      int64_t nb = 0;
      HIP_TRY(timed(c, GMG_K_FCG, 0, GMG_F64, q,
                    [&] { return gmg::launch_fcg_zq<TZ>(Vg, z, c->vq, c->partials, &nb, q); }));
      HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
        return gmg::launch_fcg_fin(0, c->state, c->partials, nb, nullptr, q);
      }));
      HIP_TRY(timed(c, GMG_K_FCG, 0, GMG_F64, q, [&](gmg::Shape sh) {
        return gmg::launch_fcg_dir<TZ>(Vg, z, u, ri == 0 ? c->vp : c->vt, ri == 0 ? c->vt : c->vp,
                                       c->vq, c->vr, c->state, ri == 1, c->partials, &nb, q, sh);
      }));
      HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
        return gmg::launch_fcg_fin(1, c->state, c->partials, nb, nullptr, q);
      }));
      HIP_TRY(timed(c, GMG_K_FCG, 0, GMG_F64, q, [&](gmg::Shape sh) {
        return gmg::launch_fcg_update(Vg, c->vr, c->vq, mixed ? c->er32 : nullptr, c->state,
                                      c->partials, &nb, q, sh);
      }));
      HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
        return gmg::launch_fcg_fin(2, c->state, c->partials, nb, c->dhist, q);
      }));
      return GMG_OK;
    };
    if ((st = run_iterations(c, s, line_only ? GK_FCG_LINE : GK_FCG, f, u, kFcgKinds, maxit, 2,
                             4, unit)))
      return st;
  }
  // the steps still owed to the iterate (the direction kernels of even
  // iterations apply the earlier ones in pairs)
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s, [&] {
    return gmg::launch_pcg_final_update(V, u, c->vp, c->vt, c->state, s);
  }));
  const CgState hs = *c->hstate;
  if (history) memcpy(history, c->hhist, (size_t)(hs.iter + 1) * sizeof(double));
  double rr = 0.0;
  if ((st = residual_norm2<double>(c, f, u, c->vt, nullptr, &rr, s))) return st;
  if (iters) *iters = hs.iter;
  if (relres) *relres = sqrt(rr / rr0);
  if (hs.status == 1 || !hs.done)
    return fail(GMG_ENOCONV, "no convergence to %g in %d iterations", rtol, maxit);
  if (hs.status >= 2)
    return fail(GMG_ENOCONV, "flexible CG breakdown or non-finite value at iteration %d",
                hs.iter);
  return GMG_OK;
}

// ---- autotuner --------------------------------------------------------------
// Candidate launch shapes: rows per workgroup and tile columns per dispatch
// group (0 = row-major).  Stencil kernels: 4, 8 or 16 rows; line kernels: the
// twisted elimination (4) and, for the line solve and the smoother, one
// wavefront per column by cyclic reduction (1, tile order irrelevant); the
// smoother also with its neighbours staged in LDS (2), and staged with two
// wavefronts per column by direct loads (3).
constexpr int kStencilRows[] = {4, 8, 16};
constexpr int kLineRows[] = {4};
constexpr int kLinePcrRows[] = {4, 1};
constexpr int kSmoothRows[] = {4, 1, 2, 3};
constexpr int kTuneGroups[] = {0, 1, 2, 4, 8};

enum class Cand { STENCIL, LINE, LINE_PCR, SMOOTH };

// Time `reps` launches of every candidate shape of one kernel kind and store
// the fastest in the context's table.  `nti` is the kernel's tile count across
// (groups at or above it are row-major again and are skipped).
template <typename F>
int tune_kind(gmg_ctx* c, int kind, int level, int prec, Cand cand, int nti, int reps,
              hipStream_t s, hipEvent_t ea, hipEvent_t eb, F&& launch,
              float* best_out = nullptr) {
  gmg::Shape best{};
  float best_ms = 0.0f;
  bool have = false;
  const int* rows_c = cand == Cand::STENCIL    ? kStencilRows
                      : cand == Cand::LINE     ? kLineRows
                      : cand == Cand::LINE_PCR ? kLinePcrRows
                                               : kSmoothRows;
  const int nrows = cand == Cand::STENCIL    ? 3
                    : cand == Cand::LINE     ? 1
                    : cand == Cand::LINE_PCR ? 2
                                             : 4;
  for (int q0 = 0; q0 < nrows; ++q0) {
    const int rows = rows_c[q0];
    for (int group : kTuneGroups) {
      if (group >= nti || (rows == 1 && group != 0)) continue;
      const gmg::Shape sh{rows, group};
      HIP_TRY(launch(sh));  // warm-up
      HIP_TRY(hipEventRecord(ea, s));
      for (int q = 0; q < reps; ++q) HIP_TRY(launch(sh));
      HIP_TRY(hipEventRecord(eb, s));
      HIP_TRY(hipEventSynchronize(eb));
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, ea, eb));
      if (!have || ms < best_ms) {
        best = sh;
        best_ms = ms;
        have = true;
      }
    }
  }
  c->shape[gmg::tslot(kind, level, prec)] = best;
  if (best_out) *best_out = best_ms;
  return GMG_OK;
}

// The kernels the solvers launch on level d in precision T, run on the
// context's own work buffers (level 0: the solver vectors).
template <typename T>
int tune_levels(gmg_ctx* c, int reps, hipStream_t s, hipEvent_t ea, hipEvent_t eb) {
  using gmg::Shape;
  const int P = prec_of<T>();
  const int L = c->nlevels;
  const T rho = (T)c->p.rho;
  for (int d = 0; d < L; ++d) {
    const Lvl<T> V = gmg::view<T>(c, d);
    T *x0, *x1, *x2;
    if (d > 0) {
      x0 = static_cast<T*>(c->lev[d].u);
      x1 = static_cast<T*>(c->lev[d].ualt);
      x2 = static_cast<T*>(c->lev[d].f);
    } else if constexpr (sizeof(T) == 8) {
      x0 = reinterpret_cast<T*>(c->vt);
      x1 = reinterpret_cast<T*>(c->vz);
      x2 = reinterpret_cast<T*>(c->vr);
    } else {
      x0 = reinterpret_cast<T*>(c->eu32);
      x1 = static_cast<T*>(c->lev[0].ualt);
      x2 = reinterpret_cast<T*>(c->er32);
    }
    if (!x0 || !x1 || !x2 || (d + 1 < L && (!c->lev[d + 1].u || !c->lev[d + 1].f)))
      return fail(GMG_EINVAL, "autotune: level %d work buffers are missing", d);
    const int nts = (int)gmg::stencil_tiles_x(V.nx), ntl = (int)gmg::line_tiles_x(V.nx);
    int64_t nb = 0;
    int st;
    if ((st = tune_kind(c, GMG_K_SPMV, d, P, Cand::STENCIL, nts, reps, s, ea, eb, [&](Shape sh) {
           return gmg::launch_stencil<T>(V, Stencil::SPMV, x0, nullptr, x1, nullptr, nullptr,
                                         nullptr, s, sh);
         })))
      return st;
    if ((st = tune_kind(c, GMG_K_RESIDUAL, d, P, Cand::STENCIL, nts, reps, s, ea, eb, [&](Shape sh) {
           return gmg::launch_stencil<T>(V, Stencil::RESIDUAL_NORM, x0, x2, x1, nullptr,
                                         c->partials, &nb, s, sh);
         })))
      return st;
    if ((st = tune_kind(c, GMG_K_LINE_SOLVE, d, P, Cand::LINE_PCR, ntl, reps, s, ea, eb, [&](Shape sh) {
           return gmg::launch_line_solve_scaled<T>(V, x2, x1, rho, s, sh);
         })))
      return st;
    float ms_smooth = 0.0f;
    if ((st = tune_kind(c, GMG_K_SMOOTH, d, P, Cand::SMOOTH, ntl, reps, s, ea, eb, [&](Shape sh) {
           return gmg::launch_smooth<T>(V, x2, x0, x1, rho, s, sh);
         }, &ms_smooth)))
      return st;
    if (d + 1 < L) {
      const Lvl<T> C = gmg::view<T>(c, d + 1);
      T* fc = static_cast<T*>(c->lev[d + 1].f);
      T* uc = static_cast<T*>(c->lev[d + 1].u);
      if ((st = tune_kind(c, GMG_K_RESIDUAL_RESTRICT, d, P, Cand::STENCIL,
                          (int)gmg::stencil_tiles_x(C.nx), reps, s, ea, eb, [&](Shape sh) {
                            return gmg::launch_resrestrict<T>(V, C, x0, x2, fc, s, sh);
                          })))
        return st;
      // prolongation from level d+1 onto level d, kept under the coarse level
      float ms_prol = 0.0f;
      if ((st = tune_kind(c, GMG_K_PROLONGATE, d + 1, P, Cand::STENCIL, nts, reps, s, ea, eb,
                          [&](Shape sh) {
                            return gmg::launch_prolongate<T>(C, V, uc, x1, s, sh);
                          }, &ms_prol)))
        return st;
      // the prolongation folded into the post-smoother: kept where it beats
      // the two kernels
      Shape fused{4, 0};
      float best_ms = ms_smooth + ms_prol;
      for (int q0 = 0; q0 < 2 * (int)(sizeof(kTuneGroups) / sizeof(int)); ++q0) {
        // rows 2: one wavefront per column; rows 3: two (where the level fits)
        const int group = kTuneGroups[q0 >> 1];
        if (group >= ntl) continue;
        const Shape sh{(q0 & 1) ? 3 : 2, group};
        auto go = [&] { return gmg::launch_prolong_smooth<T>(V, C, x2, x0, uc, x1, rho, s, sh); };
        HIP_TRY(go());  // warm-up
        HIP_TRY(hipEventRecord(ea, s));
        for (int q = 0; q < reps; ++q) HIP_TRY(go());
        HIP_TRY(hipEventRecord(eb, s));
        HIP_TRY(hipEventSynchronize(eb));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ea, eb));
        if (ms < best_ms) {
          best_ms = ms;
          fused = sh;
        }
      }
      c->shape[gmg::tslot(GMG_K_PROLONG_SMOOTH, d, P)] = fused;
    }
  }
  return GMG_OK;
}

// The FP64 finest-level solver kernels: CG, refinement update, flexible CG.
int tune_solver(gmg_ctx* c, int reps, hipStream_t s, hipEvent_t ea, hipEvent_t eb) {
  using gmg::Shape;
  const Lvl<double> V = gmg::view<double>(c, 0);
  const int nts = (int)gmg::stencil_tiles_x(V.nx), ntl = (int)gmg::line_tiles_x(V.nx);
  const bool mixed = c->p.prec_precond == GMG_F32;
  if (!c->vt || !c->vp || !c->vz || !c->vq || !c->vr || !c->partials || !c->state ||
      (mixed && (!c->er32 || !c->eu32)))
    return fail(GMG_EINVAL, "autotune: solver work buffers are missing");
  // a running CG state with alpha = beta = 0: the kernels then leave r and u
  // unchanged
  gmg::CgState idle{};
  idle.maxit = 1 << 30;
  HIP_TRY(hipMemcpyAsync(c->state, &idle, sizeof(idle), hipMemcpyHostToDevice, s));
  int64_t nb = 0;
  int st;
  if ((st = tune_kind(c, GMG_K_CG_SPMV, 0, GMG_F64, Cand::STENCIL, nts, reps, s, ea, eb, [&](Shape sh) {
         // the heavier (even, paired) form of line-PCG's direction step
         return gmg::launch_cg_p1(V, c->vt, c->vp, c->vr, c->vz, c->vq, c->state, true,
                                  c->partials, &nb, s, sh);
       })))
    return st;
  if ((st = tune_kind(c, GMG_K_CG_TRIDIAG, 0, GMG_F64, Cand::LINE, ntl, reps, s, ea, eb,
                      [&](Shape sh) {
                        return gmg::launch_cg_p2(V, c->vr, c->vq, c->vz, c->state, 0,
                                                 c->partials, &nb, s, sh);
                      })))
    return st;
  if (mixed) {
    if ((st = tune_kind(c, GMG_K_RESIDUAL, 0, GMG_F64, Cand::STENCIL, nts, reps, s, ea, eb,
                        [&](Shape sh) {
                          return gmg::launch_stencil<double>(V, Stencil::RESIDUAL_NORM_DOWN,
                                                             c->vt, c->vr, c->vz, c->er32,
                                                             c->partials, &nb, s, sh);
                        })))
      return st;
    if ((st = tune_kind(c, GMG_K_CORRECT, 0, GMG_F64, Cand::STENCIL, nts, reps, s, ea, eb,
                        [&](Shape sh) {
                          return gmg::launch_correct_residual(V, c->vt, c->eu32, c->vr, c->vz,
                                                              c->er32, c->partials, &nb, s, sh);
                        })))
      return st;
  }
  if ((st = tune_kind(c, GMG_K_FCG, 0, GMG_F64, Cand::STENCIL, nts, reps, s, ea, eb, [&](Shape sh) {
         // the odd-iteration form (it leaves u alone), vp -> vt
         hipError_t e =
             mixed ? gmg::launch_fcg_dir<float>(V, c->eu32, nullptr, c->vp, c->vt, c->vq, c->vr,
                                                c->state, false, c->partials, &nb, s, sh)
                   : gmg::launch_fcg_dir<double>(V, c->vz, nullptr, c->vp, c->vt, c->vq, c->vr,
                                                 c->state, false, c->partials, &nb, s, sh);
         if (e != hipSuccess) return e;
         return gmg::launch_fcg_update(V, c->vr, c->vq, mixed ? c->er32 : nullptr, c->state,
                                       c->partials, &nb, s, sh);
       })))
    return st;
  return GMG_OK;
}

}  // namespace

extern "C" {

int gmg_timing_enable(gmg_ctx* c, int enable) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (enable) {
    c->pending.clear();
    c->evused = 0;
    c->tcount.assign((size_t)GMG_K_COUNT * gmg::kMaxLevels * 2, 0);
    c->tms.assign((size_t)GMG_K_COUNT * gmg::kMaxLevels * 2, 0.0);
  }
  c->timing = enable != 0;
  return GMG_OK;
}

int gmg_timing_filter(gmg_ctx* c, uint32_t kernel_mask) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  c->timing_mask = kernel_mask;
  return GMG_OK;
}

int gmg_timing_read(gmg_ctx* c, int kernel, int level, int prec, int64_t* count,
                    double* total_ms) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (kernel < 0 || kernel >= GMG_K_COUNT) return fail(GMG_EINVAL, "bad kernel id %d", kernel);
  if (level < -1 || level >= c->nlevels) return fail(GMG_EINVAL, "bad level %d", level);
  int st;
  if ((st = check_prec(prec))) return st;
  if (c->tcount.empty()) {
    if (count) *count = 0;
    if (total_ms) *total_ms = 0.0;
    return GMG_OK;
  }
  if ((st = drain_timing(c))) return st;
  int64_t n = 0;
  double ms = 0.0;
  for (int d = (level < 0 ? 0 : level); d <= (level < 0 ? c->nlevels - 1 : level); ++d) {
    n += c->tcount[gmg::tslot(kernel, d, prec)];
    ms += c->tms[gmg::tslot(kernel, d, prec)];
  }
  if (count) *count = n;
  if (total_ms) *total_ms = ms;
  return GMG_OK;
}

int gmg_copy_probe(const void* src, void* dst, int64_t bytes, void* stream) {
  int st;
  if ((st = check_ptrs({src, dst}))) return st;
  if (bytes < 0 || bytes % 8) return fail(GMG_EINVAL, "copy: bytes must be a multiple of 8");
  const char *a = static_cast<const char*>(src), *b = static_cast<const char*>(dst);
  if (a < b + bytes && b < a + bytes) return fail(GMG_EINVAL, "copy: src and dst overlap");
  HIP_TRY(gmg::launch_copy_probe(static_cast<const double*>(src), static_cast<double*>(dst),
                                 bytes / 8, as_stream(stream)));
  return GMG_OK;
}

int gmg_transpose_in(gmg_ctx* c, int level, int prec, const void* src_z, void* dst_x,
                     void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({src_z, dst_x}))) return st;
  if (src_z == dst_x) return fail(GMG_EINVAL, "transpose: src and dst must differ");
  const LevelBuf& B = c->lev[level];
  hipStream_t s = as_stream(stream);
  HIP_TRY(prec == GMG_F64
              ? gmg::launch_transpose<double>((const double*)src_z, (double*)dst_x, B.nx, B.ny,
                                              B.nz, B.ldx, true, s)
              : gmg::launch_transpose<float>((const float*)src_z, (float*)dst_x, B.nx, B.ny,
                                             B.nz, B.ldx, true, s));
  return GMG_OK;
}

int gmg_transpose_out(gmg_ctx* c, int level, int prec, const void* src_x, void* dst_z,
                      void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({src_x, dst_z}))) return st;
  if (src_x == dst_z) return fail(GMG_EINVAL, "transpose: src and dst must differ");
  const LevelBuf& B = c->lev[level];
  hipStream_t s = as_stream(stream);
  HIP_TRY(prec == GMG_F64
              ? gmg::launch_transpose<double>((const double*)src_x, (double*)dst_z, B.nx, B.ny,
                                              B.nz, B.ldx, false, s)
              : gmg::launch_transpose<float>((const float*)src_x, (float*)dst_z, B.nx, B.ny,
                                             B.nz, B.ldx, false, s));
  return GMG_OK;
}

}  // extern "C"

namespace {

// Host-side copy of one staged chunk, split over a few threads: a single
// thread's memcpy from pageable memory runs well below the link's rate.
void par_memcpy(void* dst, const void* src, size_t n) {
  const unsigned hw = std::thread::hardware_concurrency();
  const size_t nt = std::max<size_t>(1, std::min<size_t>(8, hw ? hw / 2 : 1));
  const size_t per = (n / nt + 4095) / 4096 * 4096;
  if (nt == 1 || n < (4u << 20)) {
    memcpy(dst, src, n);
    return;
  }
  std::vector<std::thread> th;
  size_t done = 0;  // bytes handed to threads
  try {
    for (size_t t = 0; t < nt; ++t) {
      const size_t a = t * per;
      if (a >= n) break;
      const size_t len = std::min(per, n - a);
      th.emplace_back(
          [=] { memcpy(static_cast<char*>(dst) + a, static_cast<const char*>(src) + a, len); });
      done = a + len;
    }
  } catch (...) {
    // no thread to be had: the caller's thread copies the rest
  }
  if (done < n) memcpy(static_cast<char*>(dst) + done, static_cast<const char*>(src) + done, n - done);
  for (std::thread& t : th) t.join();
}

// Pinned staging for the host transfers of gmg_solve_host: two buffers of up
// to kStageBytes, allocated at first use.
constexpr size_t kStageBytes = size_t(128) << 20;

int ensure_stage(gmg_ctx* c, size_t bytes) {
  if (c->stage_bytes) return GMG_OK;
  const size_t sz = std::min(kStageBytes, std::max<size_t>(bytes, 1));
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipHostMalloc(&c->stage[b], sz, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->stage_ev[b], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (int b = 0; b < 2; ++b) {
      if (c->stage[b]) (void)hipHostFree(c->stage[b]);
      if (c->stage_ev[b]) (void)hipEventDestroy(c->stage_ev[b]);
      c->stage[b] = nullptr;
      c->stage_ev[b] = nullptr;
    }
    return fail(GMG_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
  }
  c->stage_bytes = sz;
  return GMG_OK;
}

// host (pageable) -> device through the two pinned buffers: the host fills
// one while the DMA engine drains the other
int upload(gmg_ctx* c, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t ch = c->stage_bytes;
  for (size_t q = 0, off = 0; off < bytes; ++q, off += ch) {
    const int b = (int)(q & 1);
    const size_t len = std::min(ch, bytes - off);
    if (q >= 2) HIP_TRY(hipEventSynchronize(c->stage_ev[b]));  // its last DMA has read it
    par_memcpy(c->stage[b], static_cast<const char*>(src) + off, len);
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(dst) + off, c->stage[b], len,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(c->stage_ev[b], s));
  }
  return GMG_OK;
}

// device -> host (pageable): the DMA fills one buffer while the host empties
// the other
int download(gmg_ctx* c, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t ch = c->stage_bytes;
  size_t prev_off = 0, prev_len = 0;
  int prev_b = -1;
  for (size_t q = 0, off = 0; off < bytes; ++q, off += ch) {
    const int b = (int)(q & 1);
    const size_t len = std::min(ch, bytes - off);
    HIP_TRY(hipMemcpyAsync(c->stage[b], static_cast<const char*>(src) + off, len,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(c->stage_ev[b], s));
    if (prev_b >= 0) {
      HIP_TRY(hipEventSynchronize(c->stage_ev[prev_b]));
      par_memcpy(static_cast<char*>(dst) + prev_off, c->stage[prev_b], prev_len);
    }
    prev_b = b;
    prev_off = off;
    prev_len = len;
  }
  if (prev_b >= 0) {
    HIP_TRY(hipEventSynchronize(c->stage_ev[prev_b]));
    par_memcpy(static_cast<char*>(dst) + prev_off, c->stage[prev_b], prev_len);
  }
  return GMG_OK;
}

}  // namespace

extern "C" {

int gmg_solve_host(gmg_ctx* c, int method, const double* f_host, double* u_host, double rtol,
                   int maxit, int* iters, double* relres, double* timings_ms, void* stream) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (!f_host || !u_host) return fail(GMG_EINVAL, "NULL host array");
  if (method < 0 || method > 2) return fail(GMG_EINVAL, "method must be 0, 1 or 2");
  const LevelBuf& B = c->lev[0];
  const size_t ncan = (size_t)B.nx * B.ny * B.nz;
  const size_t bytes = ncan * sizeof(double);
  if (!c->hz) {
    hipError_t e;
    if ((e = dmalloc(&c->hz, (int64_t)ncan)) || (e = dmalloc(&c->hf, B.elems)) ||
        (e = dmalloc(&c->hu, B.elems))) {
      dfree(c->hz); dfree(c->hf); dfree(c->hu);
      c->hz = c->hf = c->hu = nullptr;
      return fail(GMG_ENOMEM, "host-solve buffers: %s", hipGetErrorString(e));
    }
  }
  int st;
  if ((st = ensure_stage(c, bytes))) return st;
  hipStream_t s = as_stream(stream);
  using clock = std::chrono::steady_clock;
  auto ms_since = [](clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(clock::now() - t0).count();
  };
  auto sync = [&]() -> int { HIP_TRY(hipStreamSynchronize(s)); return GMG_OK; };
  // copies in: f, then the initial guess u, each converted to the solver's
  // layout once it is on the device (each step timed on the host clock)
  HIP_TRY(hipStreamSynchronize(s));
  double t_copy_in = 0.0, t_layout_in = 0.0;
  for (int fld = 0; fld < 2; ++fld) {
    const void* src = fld == 0 ? (const void*)f_host : (const void*)u_host;
    double* dst = fld == 0 ? c->hf : c->hu;
    auto tc = clock::now();
    if ((st = upload(c, src, c->hz, bytes, s)) || (st = sync())) return st;
    t_copy_in += ms_since(tc);
    auto tl = clock::now();
    HIP_TRY(gmg::launch_transpose<double>(c->hz, dst, B.nx, B.ny, B.nz, B.ldx, true, s));
    if ((st = sync())) return st;
    t_layout_in += ms_since(tl);
  }
  auto ts = clock::now();
  const int solve_st =
      method == 0 ? gmg_solve(c, c->hf, c->hu, rtol, maxit, iters, relres, nullptr, stream)
                  : pcg_solve(c, c->hf, c->hu, rtol, maxit, method == 2 ? 1 : 0, iters, relres,
                              nullptr, stream);
  if (solve_st != GMG_OK && solve_st != GMG_ENOCONV) return solve_st;
  if ((st = sync())) return st;
  const double t_solve = ms_since(ts);
  auto tl = clock::now();
  HIP_TRY(gmg::launch_transpose<double>(c->hu, c->hz, B.nx, B.ny, B.nz, B.ldx, false, s));
  if ((st = sync())) return st;
  const double t_layout_out = ms_since(tl);
  auto tc = clock::now();
  if ((st = download(c, c->hz, u_host, bytes, s))) return st;
  const double t_copy_out = ms_since(tc);
  if (timings_ms) {
    timings_ms[0] = t_copy_in;     // host -> device copies (host staging included)
    timings_ms[1] = t_layout_in;   // layout conversions in
    timings_ms[2] = t_solve;       // solve
    timings_ms[3] = t_layout_out;  // layout conversion out
    timings_ms[4] = t_copy_out;    // device -> host copy (host staging included)
  }
  return solve_st;  // GMG_ENOCONV keeps the solve's message
}

int gmg_set_launch(gmg_ctx* c, int kernel, int level, int prec, int rows, int group) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (kernel < 0 || kernel >= GMG_K_COUNT) return fail(GMG_EINVAL, "bad kernel id %d", kernel);
  if (level < 0 || level >= c->nlevels) return fail(GMG_EINVAL, "bad level %d", level);
  int st;
  if ((st = check_prec(prec))) return st;
  const bool pcr_ok = kernel == GMG_K_LINE_SOLVE || kernel == GMG_K_SMOOTH;
  if (kernel == GMG_K_PROLONG_SMOOTH) {
    if (rows != 4 && rows != 2 && rows != 3)
      return fail(GMG_EINVAL,
                  "rows of the folded prolongation must be 4 (off), 2 or 3, got %d", rows);
  } else if (!(rows == 4 || rows == 8 || rows == 16 || (rows == 1 && pcr_ok) ||
               ((rows == 2 || rows == 3) && kernel == GMG_K_SMOOTH))) {
    return fail(GMG_EINVAL,
                "rows must be 4, 8 or 16 (1 for the line solve and smoother, 2 or 3 for the "
                "smoother), got %d",
                rows);
  }
  if (group < 0 || group > 4096) return fail(GMG_EINVAL, "group must be in [0, 4096]");
  c->shape[gmg::tslot(kernel, level, prec)] = gmg::Shape{rows, group};
  drop_graphs(c);  // captured launches carry the old shape
  return GMG_OK;
}

int gmg_solver_polls(const gmg_ctx* c) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  return c->polls;
}

int gmg_set_graphs(gmg_ctx* c, int enable) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  c->graphs_on = enable != 0;
  if (!c->graphs_on) drop_graphs(c);
  return GMG_OK;
}

int gmg_get_launch(const gmg_ctx* c, int kernel, int level, int prec, int* rows, int* group) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (kernel < 0 || kernel >= GMG_K_COUNT) return fail(GMG_EINVAL, "bad kernel id %d", kernel);
  if (level < 0 || level >= c->nlevels) return fail(GMG_EINVAL, "bad level %d", level);
  int st;
  if ((st = check_prec(prec))) return st;
  const gmg::Shape sh = c->shape[gmg::tslot(kernel, level, prec)];
  if (rows) *rows = sh.rows;
  if (group) *group = sh.group;
  return GMG_OK;
}

int gmg_autotune(gmg_ctx* c, int reps, void* stream) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  if (reps < 1 || reps > 1000) return fail(GMG_EINVAL, "reps must be in [1, 1000]");
  hipStream_t s = as_stream(stream);
  hipEvent_t ea = nullptr, eb = nullptr;
  HIP_TRY(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    (void)hipEventDestroy(ea);
    return fail(GMG_EHIP, "hipEventCreate failed");
  }
  drop_graphs(c);
  int st = c->p.prec_precond == GMG_F32 ? tune_levels<float>(c, reps, s, ea, eb)
                                         : tune_levels<double>(c, reps, s, ea, eb);
  if (!st) st = tune_solver(c, reps, s, ea, eb);
  const hipError_t e = hipStreamSynchronize(s);
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (st) return st;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return GMG_OK;
}

int spmv(gmg_ctx* c, int level, int prec, const void* x, void* y, void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({x, y}))) return st;
  if (x == y) return fail(GMG_EINVAL, "spmv: x and y must not overlap");
  hipStream_t s = as_stream(stream);
  if (prec == GMG_F64)
    HIP_TRY(timed(c, GMG_K_SPMV, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_stencil<double>(gmg::view<double>(c, level), Stencil::SPMV,
                                         (const double*)x, nullptr, (double*)y, nullptr, nullptr,
                                         nullptr, s, sh);
    }));
  else
    HIP_TRY(timed(c, GMG_K_SPMV, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_stencil<float>(gmg::view<float>(c, level), Stencil::SPMV,
                                        (const float*)x, nullptr, (float*)y, nullptr, nullptr,
                                        nullptr, s, sh);
    }));
  return GMG_OK;
}

int line_solve(gmg_ctx* c, int level, int prec, const void* r, void* z, void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({r, z}))) return st;
  hipStream_t s = as_stream(stream);
  if (prec == GMG_F64)
    HIP_TRY(timed(c, GMG_K_LINE_SOLVE, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_line_solve<double>(gmg::view<double>(c, level), (const double*)r,
                                            (double*)z, s, sh);
    }));
  else
    HIP_TRY(timed(c, GMG_K_LINE_SOLVE, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_line_solve<float>(gmg::view<float>(c, level), (const float*)r,
                                           (float*)z, s, sh);
    }));
  return GMG_OK;
}

int line_smooth(gmg_ctx* c, int level, int prec, const void* f, void* u, int nsweeps, double rho,
                void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({f, u}))) return st;
  if (nsweeps < 0) return fail(GMG_EINVAL, "nsweeps must be >= 0");
  if (!(rho > 0.0) || !(rho <= 2.0)) return fail(GMG_EINVAL, "rho must be in (0, 2]");
  if (f == u) return fail(GMG_EINVAL, "f and u must not overlap");
  hipStream_t s = as_stream(stream);
  if (prec == GMG_F64)
    return line_smooth_t<double>(c, level, (const double*)f, (double*)u, nsweeps, rho, s);
  return line_smooth_t<float>(c, level, (const float*)f, (float*)u, nsweeps, (float)rho, s);
}

int gmg_residual(gmg_ctx* c, int level, int prec, const void* f, const void* u, void* r,
                 double* norm2, void* stream) {
  if (!level_ok(c, level)) return fail(GMG_EINVAL, "bad context or level %d", level);
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({f, u, r}))) return st;
  if (r == u || r == f) return fail(GMG_EINVAL, "r must not overlap f or u");
  hipStream_t s = as_stream(stream);
  int64_t nb = 0;
  const Stencil mode = norm2 ? Stencil::RESIDUAL_NORM : Stencil::RESIDUAL;
  if (prec == GMG_F64)
    HIP_TRY(timed(c, GMG_K_RESIDUAL, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_stencil<double>(gmg::view<double>(c, level), mode, (const double*)u,
                                         (const double*)f, (double*)r, nullptr, c->partials, &nb, s, sh);
    }));
  else
    HIP_TRY(timed(c, GMG_K_RESIDUAL, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_stencil<float>(gmg::view<float>(c, level), mode, (const float*)u,
                                        (const float*)f, (float*)r, nullptr, c->partials, &nb, s, sh);
    }));
  if (norm2) {
    double* dst = c->partials + c->max_partials;
    HIP_TRY(timed(c, GMG_K_REDUCE, level, GMG_F64, s,
                  [&] { return gmg::launch_reduce(c->partials, nb, 1, dst, s); }));
    HIP_TRY(hipMemcpyAsync(c->hscal, dst, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *norm2 = c->hscal[0];
  }
  return GMG_OK;
}

int gmg_restrict_smooth(gmg_ctx* c, int level, int prec, const void* rf, void* fc, void* uc,
                        double rho, void* stream) {
  if (!c || c->batch || level < 1 || level >= c->nlevels)
    return fail(GMG_EINVAL, "restrict_smooth needs a coarse level in [1, nlevels)");
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({rf, fc, uc}))) return st;
  if (fc == uc) return fail(GMG_EINVAL, "fc and uc must differ");
  hipStream_t s = as_stream(stream);
  if (prec == GMG_F64)
    HIP_TRY(timed(c, GMG_K_RESTRICT_SMOOTH, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_restrict_smooth<double>(gmg::view<double>(c, level),
                                                 gmg::view<double>(c, level - 1),
                                                 (const double*)rf, (double*)fc, (double*)uc, rho, s, sh);
    }));
  else
    HIP_TRY(timed(c, GMG_K_RESTRICT_SMOOTH, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_restrict_smooth<float>(gmg::view<float>(c, level),
                                                gmg::view<float>(c, level - 1), (const float*)rf,
                                                (float*)fc, (float*)uc, (float)rho, s, sh);
    }));
  return GMG_OK;
}

int gmg_prolongate(gmg_ctx* c, int level, int prec, const void* uc, void* uf, void* stream) {
  if (!c || c->batch || level < 1 || level >= c->nlevels)
    return fail(GMG_EINVAL, "prolongate needs a coarse level in [1, nlevels)");
  int st;
  if ((st = check_prec(prec)) || (st = check_ptrs({uc, uf}))) return st;
  hipStream_t s = as_stream(stream);
  if (prec == GMG_F64)
    HIP_TRY(timed(c, GMG_K_PROLONGATE, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_prolongate<double>(gmg::view<double>(c, level),
                                            gmg::view<double>(c, level - 1), (const double*)uc,
                                            (double*)uf, s, sh);
    }));
  else
    HIP_TRY(timed(c, GMG_K_PROLONGATE, level, prec, s, [&](gmg::Shape sh) {
      return gmg::launch_prolongate<float>(gmg::view<float>(c, level),
                                           gmg::view<float>(c, level - 1), (const float*)uc,
                                           (float*)uf, s, sh);
    }));
  return GMG_OK;
}

int gmg_vcycle(gmg_ctx* c, const void* f, void* u, void* stream) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  int st;
  if ((st = check_ptrs({f, u}))) return st;
  if (f == u) return fail(GMG_EINVAL, "f and u must not overlap");
  hipStream_t s = as_stream(stream);
  if (c->p.prec_precond == GMG_F64) return vcycle_impl<double>(c, (const double*)f, (double*)u, s);
  return vcycle_impl<float>(c, (const float*)f, (float*)u, s);
}

int gmg_solve(gmg_ctx* c, const double* f, double* u, double rtol, int maxit, int* iters,
              double* relres, double* history, void* stream) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  c->polls = 0;
  int st;
  if ((st = check_ptrs({f, u}))) return st;
  if (!(rtol > 0.0)) return fail(GMG_EINVAL, "rtol must be > 0");
  if (maxit < 0) return fail(GMG_EINVAL, "maxit must be >= 0");
  if (f == u) return fail(GMG_EINVAL, "f and u must not overlap");
  hipStream_t s = as_stream(stream);
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  if (history) history[0] = 1.0;
  if ((st = ensure_hist(c, maxit))) return st;
  const bool f64 = c->p.prec_precond == GMG_F64;
  CgState init{};
  init.maxit = maxit;
  init.rtol = rtol;
  HIP_TRY(hipMemcpyAsync(c->state, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
  const double rho = c->p.rho;
  double* ualt0 = static_cast<double*>(c->lev[0].ualt);
  {
    GateScope gate(c);
    if (f64) {
      // The first smoothing step of every cycle computes f - A u of the
      // current iterate in its forward sweep; its norm is the stopping test
      // of the previous cycle, so no separate residual pass is needed.  The
      // step writes lev[0].ualt, so u still holds the tested iterate when
      // the solve stops (the next cycle's kernels are gated off).
      auto smooth_test = [&](hipStream_t q, int init_) -> int {
        const Lvl<double> V0 = gmg::view<double>(c, 0);
        int64_t nb = 0;
        HIP_TRY(timed(c, GMG_K_SMOOTH, 0, GMG_F64, q, [&](gmg::Shape sh) {
          return gmg::launch_smooth_norm<double>(V0, f, u, ualt0, rho, c->partials, &nb, q, sh);
        }));
        HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
          return gmg::launch_mg_fin(c->state, c->partials, nb, init_, c->dhist, q);
        }));
        return GMG_OK;
      };
      if ((st = smooth_test(s, 1))) return st;
      auto unit = [&](hipStream_t q, int) -> int {
        const int sv = vcycle_impl<double>(c, f, u, q, false, true);
        return sv ? sv : smooth_test(q, 0);
      };
      if ((st = run_iterations(c, s, GK_MG, f, u, kVcycleKinds, maxit, 1, 4, unit))) return st;
    } else {
      // FP64 iterative refinement with FP32 cycles: e = V32(r32) from a zero
      // guess, then u' = u + e, r = f - A u', r32 and ||r||^2 in one fused
      // pass.  The iterate alternates between the caller's u (before odd
      // steps) and an internal buffer (before even steps).
      {
        const Lvl<double> V0 = gmg::view<double>(c, 0);
        int64_t nb = 0;
        HIP_TRY(timed(c, GMG_K_RESIDUAL, 0, GMG_F64, s, [&](gmg::Shape sh) {
          return gmg::launch_stencil<double>(V0, Stencil::RESIDUAL_NORM_DOWN, u, f, c->vr,
                                             c->er32, c->partials, &nb, s, sh);
        }));
        HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, s, [&] {
          return gmg::launch_mg_fin(c->state, c->partials, nb, 1, c->dhist, s);
        }));
      }
      auto unit = [&](hipStream_t q, int r) -> int {
        double* ucur = r == 0 ? u : c->vt;
        double* unext = r == 0 ? c->vt : u;
        const int sv = vcycle_impl<float>(c, c->er32, c->eu32, q, true, false);
        if (sv) return sv;
        const Lvl<double> V0 = gmg::view<double>(c, 0);
        int64_t nb = 0;
        HIP_TRY(timed(c, GMG_K_CORRECT, 0, GMG_F64, q, [&](gmg::Shape sh) {
          return gmg::launch_correct_residual(V0, ucur, c->eu32, f, unext, c->er32, c->partials,
                                              &nb, q, sh);
        }));
        HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
          return gmg::launch_mg_fin(c->state, c->partials, nb, 0, c->dhist, q);
        }));
        return GMG_OK;
      };
      if ((st = run_iterations(c, s, GK_IR, f, u, kIrKinds, maxit, 2, 4, unit))) return st;
    }
  }
  const CgState hs = *c->hstate;
  // refinement: after an odd number of steps the iterate is in the internal buffer
  bool pending = false;
  if (!f64 && (hs.iter & 1)) {
    HIP_TRY(hipMemcpyAsync(u, c->vt, (size_t)c->lev[0].elems * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    pending = true;
  }
  if (history && hs.iter >= 0) memcpy(history, c->hhist, (size_t)(hs.iter + 1) * sizeof(double));
  if (pending) {
    HIP_TRY(hipStreamSynchronize(s));
    ++c->polls;
  }
  if (iters) *iters = hs.iter;
  if (relres) *relres = hs.rr0 > 0.0 ? sqrt(hs.rr / hs.rr0) : (hs.rr0 == 0.0 ? 0.0 : NAN);
  if (hs.status == 2) {
    if (hs.iter == 0) return fail(GMG_ENOCONV, "initial residual is not finite");
    return fail(GMG_ENOCONV, "residual became non-finite at cycle %d", hs.iter);
  }
  if (!hs.done || hs.status == 1)
    return fail(GMG_ENOCONV, "no convergence to %g in %d cycles", rtol, maxit);
  return GMG_OK;
}

int pcg_solve(gmg_ctx* c, const double* f, double* u, double rtol, int maxit, int precond,
              int* iters, double* relres, double* history, void* stream) {
  if (!c || c->batch) return fail(GMG_EINVAL, "context is NULL or batched");
  c->polls = 0;
  int st;
  if ((st = check_ptrs({f, u}))) return st;
  if (!(rtol > 0.0)) return fail(GMG_EINVAL, "rtol must be > 0");
  if (maxit < 0) return fail(GMG_EINVAL, "maxit must be >= 0");
  if (f == u) return fail(GMG_EINVAL, "f and u must not overlap");
  if (precond < 0 || precond > 2) return fail(GMG_EINVAL, "precond must be 0, 1 or 2");
  hipStream_t s = as_stream(stream);
  if (precond >= 1) {
    const bool line_only = precond == 2;
    if (c->p.prec_precond == GMG_F32)
      return fcg_impl<float>(c, f, u, rtol, maxit, iters, relres, history, s, line_only);
    return fcg_impl<double>(c, f, u, rtol, maxit, iters, relres, history, s, line_only);
  }
  const Lvl<double> V = gmg::view<double>(c, 0);
  const int64_t n0 = c->lev[0].elems;
  if ((st = ensure_hist(c, maxit))) return st;
  // initial state: r = f - A u, z = M^-1 r, kappa = <r,z>, p = q = 0
  CgState init{};
  init.maxit = maxit;
  init.thresh2 = rtol * rtol;  // scaled by ||r_0||^2 on the device
  HIP_TRY(hipMemcpyAsync(c->state, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
  int64_t nb = 0;
  HIP_TRY(timed(c, GMG_K_RESIDUAL, 0, GMG_F64, s, [&](gmg::Shape sh) {
    return gmg::launch_stencil<double>(V, Stencil::RESIDUAL, u, f, c->vr, nullptr, nullptr,
                                       nullptr, s, sh);
  }));
  HIP_TRY(timed(c, GMG_K_CG_TRIDIAG, 0, GMG_F64, s, [&](gmg::Shape sh) {
    return gmg::launch_cg_p2(V, c->vr, c->vr, c->vz, c->state, 1, c->partials, &nb, s, sh);
  }));
  HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, s,
                [&] { return gmg::launch_cg_fin2(c->state, c->partials, nb, 1, c->dhist, s); }));
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s,
                [&] { return gmg::launch_fill<double>(c->vp, n0, 0.0, s); }));
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s,
                [&] { return gmg::launch_fill<double>(c->vq, n0, 0.0, s); }));
  // iterations in predicted batches of pairs; kernels of iterations after
  // convergence return at once.  Direction i goes to buffer i & 1 (vp, vt):
  // odd iterations leave u alone, even ones apply the two pending steps.
  {
    GateScope gate(c);
    auto unit = [&](hipStream_t q, int r) -> int {
      const Lvl<double> Vg = gmg::view<double>(c, 0);
      int64_t nb1 = 0, nb2 = 0;
      double* pr = r == 0 ? c->vp : c->vt;
      double* pw = r == 0 ? c->vt : c->vp;
      HIP_TRY(timed(c, GMG_K_CG_SPMV, 0, GMG_F64, q, [&](gmg::Shape sh) {
        return gmg::launch_cg_p1(Vg, u, pr, pw, c->vz, c->vq, c->state, r == 1, c->partials,
                                 &nb1, q, sh);
      }));
      HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q,
                    [&] { return gmg::launch_cg_fin1(c->state, c->partials, nb1, q); }));
      HIP_TRY(timed(c, GMG_K_CG_TRIDIAG, 0, GMG_F64, q, [&](gmg::Shape sh) {
        return gmg::launch_cg_p2(Vg, c->vr, c->vq, c->vz, c->state, 0, c->partials, &nb2, q, sh);
      }));
      HIP_TRY(timed(c, GMG_K_REDUCE, 0, GMG_F64, q, [&] {
        return gmg::launch_cg_fin2(c->state, c->partials, nb2, 0, c->dhist, q);
      }));
      return GMG_OK;
    };
    if ((st = run_iterations(c, s, GK_PCG, f, u, kPcgKinds, maxit, 2, 4, unit))) return st;
  }
  HIP_TRY(timed(c, GMG_K_AUX, 0, GMG_F64, s, [&] {
    return gmg::launch_pcg_final_update(V, u, c->vp, c->vt, c->state, s);
  }));
  const CgState hs = *c->hstate;
  if (history && hs.iter >= 0) memcpy(history, c->hhist, (size_t)(hs.iter + 1) * sizeof(double));
  double rr = 0.0;
  if ((st = residual_norm2<double>(c, f, u, c->vt, nullptr, &rr, s))) return st;
  if (iters) *iters = hs.iter;
  if (relres) *relres = hs.rr0 > 0.0 ? sqrt(rr / hs.rr0) : 0.0;
  if (hs.rr0 == 0.0) return GMG_OK;
  if (hs.status == 1 || (!hs.done && hs.iter >= maxit))
    return fail(GMG_ENOCONV, "no convergence to %g in %d iterations", rtol, maxit);
  if (hs.status >= 2)
    return fail(GMG_ENOCONV, "CG breakdown or non-finite reduction at iteration %d", hs.iter);
  return GMG_OK;
}

}  // extern "C"
