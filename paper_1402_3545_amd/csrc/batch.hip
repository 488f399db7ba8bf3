// Batched solves: many independent instances (own grid size, level count and
// coefficients), each with several right-hand sides, solved together by FP64
// iterative refinement with FP32 V-cycles (Algorithm 1).
//
// Every V-cycle phase of every (instance, rhs) pair that needs it runs in one
// grouped launch (kernels.hip: one workgroup finds its work item in a device
// table); line-kernel phases are split by the compile-time column height.  The
// whole refinement step -- FP32 V-cycle, FP64 correction + residual, per-pair
// norms and convergence masks -- is captured once into a hipGraph per
// ping-pong parity and replayed each cycle; converged pairs' workgroups exit
// at once.  Fields live in two arenas (FP64, FP32) owned by the context.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "gmg_internal.h"

namespace gmg {

namespace {

int half_class(int nz) {
  int h = 4;
  while (2 * h < nz) h *= 2;
  return h;
}

struct PairBufs {
  double *f = nullptr, *uA = nullptr, *uB = nullptr;
  float *r32 = nullptr, *e32 = nullptr, *ualt0 = nullptr;
  std::vector<float*> u, ualt, fc;  // per level (index 0 unused)
};

struct Launch {
  int kind;  // GKind value
  int half;
  int exact;  // line kinds: every item's columns have exactly 2 * half layers
  size_t item_off;
  int nitems;
  int nblocks;
};

}  // namespace

struct Batch {
  int ninst = 0, nrhs = 0, npairs = 0;
  float rho = 2.0f / 3.0f;
  int ncoarse = 2;
  std::vector<gmg_ctx*> inst;
  std::vector<int> pair_inst;
  std::vector<PairBufs> pb;
  double* a64 = nullptr;
  float* a32 = nullptr;
  size_t n64 = 0, n32 = 0;
  float* e32_all = nullptr;  // contiguous e32 of all pairs
  size_t e32_len = 0;
  std::vector<Launch> vc;
  GItem<float>* ditems = nullptr;
  GItemCR* dcr[2] = {nullptr, nullptr};
  int cr_nitems = 0, cr_nblocks = 0;
  std::vector<int> pair_blk0, pair_nblk;
  PairState* dstate = nullptr;
  PairState* hstate = nullptr;
  int* dactive = nullptr;
  int* hactive = nullptr;
  double* partials = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
};

void batch_free(Batch* b) {
  if (!b) return;
  for (gmg_ctx* c : b->inst) gmg_destroy(c);
  for (hipGraphExec_t g : b->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void* q : {(void*)b->a64, (void*)b->a32, (void*)b->ditems, (void*)b->dcr[0],
                  (void*)b->dcr[1], (void*)b->dstate, (void*)b->dactive, (void*)b->partials})
    if (q) (void)hipFree(q);
  if (b->hstate) (void)hipHostFree(b->hstate);
  if (b->hactive) (void)hipHostFree(b->hactive);
  delete b;
}

int hip_err(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_error(GMG_EHIP, m.c_str());
}

namespace {

#define BTRY(expr)                                  \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return gmg::hip_err(e_, #expr); \
  } while (0)

// Enqueue one refinement step (parity 0: uA -> uB, 1: uB -> uA) on stream s.
int enqueue_step(Batch* b, int parity, hipStream_t s) {
  for (const Launch& l : b->vc)
    BTRY(launch_grouped_f32((GKind)l.kind, l.half, l.exact != 0, b->ditems + l.item_off,
                            l.nitems, l.nblocks, b->dactive, b->rho, s));
  BTRY(launch_grouped_cr(b->dcr[parity], b->cr_nitems, b->cr_nblocks, b->dactive, b->partials, s));
  BTRY(launch_pair_reduce(b->dstate, b->dactive, b->partials, b->npairs, 0, s));
  return GMG_OK;
}

int build(Batch* b, hipStream_t s) {
  // ---- arenas ----
  std::vector<size_t> e0(b->npairs);
  size_t n64 = 0, n32 = 0;
  for (int q = 0; q < b->npairs; ++q) {
    const gmg_ctx* c = b->inst[b->pair_inst[q]];
    e0[q] = (size_t)c->lev[0].elems;
    n64 += 3 * e0[q];
    n32 += 3 * e0[q];
    for (int d = 1; d < c->nlevels; ++d) n32 += 3 * (size_t)c->lev[d].elems;
  }
  b->n64 = n64;
  b->n32 = n32;
  BTRY(hipMalloc((void**)&b->a64, std::max<size_t>(n64, 1) * sizeof(double)));
  BTRY(hipMalloc((void**)&b->a32, std::max<size_t>(n32, 1) * sizeof(float)));
  BTRY(hipMemsetAsync(b->a64, 0, n64 * sizeof(double), s));
  BTRY(hipMemsetAsync(b->a32, 0, n32 * sizeof(float), s));
  size_t o64 = 0, o32 = 0;
  b->pb.assign(b->npairs, PairBufs());
  for (int q = 0; q < b->npairs; ++q) {
    b->pb[q].f = b->a64 + o64; o64 += e0[q];
    b->pb[q].uA = b->a64 + o64; o64 += e0[q];
    b->pb[q].uB = b->a64 + o64; o64 += e0[q];
  }
  // FP32: e32 of all pairs first (one contiguous range to clear), then the rest
  b->e32_all = b->a32;
  for (int q = 0; q < b->npairs; ++q) {
    b->pb[q].e32 = b->a32 + o32;
    o32 += e0[q];
  }
  b->e32_len = o32;
  for (int q = 0; q < b->npairs; ++q) {
    const gmg_ctx* c = b->inst[b->pair_inst[q]];
    PairBufs& P = b->pb[q];
    P.r32 = b->a32 + o32; o32 += e0[q];
    P.ualt0 = b->a32 + o32; o32 += e0[q];
    P.u.assign(c->nlevels, nullptr);
    P.ualt.assign(c->nlevels, nullptr);
    P.fc.assign(c->nlevels, nullptr);
    for (int d = 1; d < c->nlevels; ++d) {
      const size_t ed = (size_t)c->lev[d].elems;
      P.u[d] = b->a32 + o32; o32 += ed;
      P.ualt[d] = b->a32 + o32; o32 += ed;
      P.fc[d] = b->a32 + o32; o32 += ed;
    }
  }

  // ---- V-cycle launch lists (static: every pointer is in the arenas) ----
  std::vector<GItem<float>> items;
  auto emit = [&](GKind kind, int half, std::vector<GItem<float>>& its) {
    if (its.empty()) return;
    // the exact-height line kernels exist for columns of 32, 64 and 128 layers
    bool exact = half >= 16;
    for (const GItem<float>& it : its) exact = exact && it.L.nz == 2 * half;
    Launch l{(int)kind, half, exact ? 1 : 0, items.size(), (int)its.size(), 0};
    int blk = 0;
    for (GItem<float>& it : its) {
      it.blk0 = blk;
      int nb;
      if (kind == GKind::LINE_SOLVE || kind == GKind::SMOOTH || kind == GKind::PROLONG_SMOOTH) {
        nb = it.nti * it.ntj;
      } else if (kind == GKind::RESRESTRICT) {
        nb = it.nti * it.ntj * (int)stencil_tiles_k(it.X.nz);
      } else {
        nb = it.nti * it.ntj * (int)stencil_tiles_k(it.L.nz);
      }
      blk += nb;
      items.push_back(it);
    }
    l.nblocks = blk;
    b->vc.push_back(l);
  };
  auto line_item = [&](int q, int d, const float* in, const float* f, float* out) {
    GItem<float> it{};
    const gmg_ctx* c = b->inst[b->pair_inst[q]];
    it.L = view<float>(c, d);
    it.a = in;
    it.b = f;
    it.o = out;
    it.nti = (int)line_tiles_x(it.L.nx);
    it.ntj = (int)line_tiles_y(it.L.ny);
    it.pair = q;
    return it;
  };
  const int halves[] = {4, 8, 16, 32, 64};
  auto emit_by_half = [&](GKind kind, std::vector<GItem<float>>& its) {
    for (int h : halves) {
      std::vector<GItem<float>> sel;
      for (const GItem<float>& it : its)
        if (half_class(it.L.nz) == h) sel.push_back(it);
      emit(kind, h, sel);
    }
  };
  int Lmax = 0;
  for (gmg_ctx* c : b->inst) Lmax = std::max(Lmax, c->nlevels);
  // cur[q][d]: buffer holding the pair's level-d iterate while the cycle is built
  std::vector<std::vector<float*>> cur(b->npairs);
  for (int q = 0; q < b->npairs; ++q) cur[q].assign(b->inst[b->pair_inst[q]]->nlevels, nullptr);
  auto rhs_of = [&](int q, int d) -> const float* {
    return d == 0 ? b->pb[q].r32 : b->pb[q].fc[d];
  };
  auto other_of = [&](int q, int d) -> float* {
    PairBufs& P = b->pb[q];
    if (d == 0) return cur[q][0] == P.e32 ? P.ualt0 : P.e32;
    return cur[q][d] == P.u[d] ? P.ualt[d] : P.u[d];
  };
  const int nc = b->ncoarse;
  for (int D = 0; D < Lmax; ++D) {
    // scaled line solve u_D = rho M^-1 f_D (zero initial guess on every level)
    std::vector<GItem<float>> ls;
    for (int q = 0; q < b->npairs; ++q) {
      const int Lq = b->inst[b->pair_inst[q]]->nlevels;
      if (D >= Lq) continue;
      PairBufs& P = b->pb[q];
      float* out;
      if (D > 0) {
        out = P.u[D];
      } else if (Lq > 1) {
        out = P.ualt0;
      } else {
        // single level: the ncoarse outputs alternate so that the last is e32
        out = ((nc - 1) % 2 == 0) ? P.e32 : P.ualt0;
      }
      ls.push_back(line_item(q, D, rhs_of(q, D), nullptr, out));
      cur[q][D] = out;
    }
    emit_by_half(GKind::LINE_SOLVE, ls);
    // remaining smoothing steps on each pair's coarsest level
    for (int sweep = 1; sweep < nc; ++sweep) {
      std::vector<GItem<float>> sm;
      for (int q = 0; q < b->npairs; ++q) {
        const int Lq = b->inst[b->pair_inst[q]]->nlevels;
        if (D != Lq - 1) continue;
        float* out = other_of(q, D);
        sm.push_back(line_item(q, D, cur[q][D], rhs_of(q, D), out));
        cur[q][D] = out;
      }
      emit_by_half(GKind::SMOOTH, sm);
    }
    // residual restricted to the next level
    std::vector<GItem<float>> rr;
    for (int q = 0; q < b->npairs; ++q) {
      const gmg_ctx* c = b->inst[b->pair_inst[q]];
      if (D >= c->nlevels - 1) continue;
      GItem<float> it{};
      it.L = view<float>(c, D);
      it.X = view<float>(c, D + 1);
      it.a = cur[q][D];
      it.b = rhs_of(q, D);
      it.o = b->pb[q].fc[D + 1];
      it.nti = (int)stencil_tiles_x(it.X.nx);
      it.ntj = (int)stencil_tiles_y(it.X.ny);
      it.pair = q;
      rr.push_back(it);
    }
    emit(GKind::RESRESTRICT, 0, rr);
  }
  // ascend: the prolongation folded into the staged post-smoother (one
  // grouped launch per column-height class and level: u_f + P u_c is
  // smoothed without being stored)
  for (int D = Lmax - 2; D >= 0; --D) {
    std::vector<GItem<float>> ps;
    for (int q = 0; q < b->npairs; ++q) {
      const gmg_ctx* c = b->inst[b->pair_inst[q]];
      if (D >= c->nlevels - 1) continue;
      float* out = D == 0 ? b->pb[q].e32 : other_of(q, D);
      GItem<float> it = line_item(q, D, cur[q][D], rhs_of(q, D), out);
      it.X = view<float>(c, D + 1);
      it.c = cur[q][D + 1];
      ps.push_back(it);
      cur[q][D] = out;
    }
    emit_by_half(GKind::PROLONG_SMOOTH, ps);
  }
  for (int q = 0; q < b->npairs; ++q)
    if (cur[q][0] != b->pb[q].e32) return set_error(GMG_EINVAL, "internal: cycle output misplaced");
  BTRY(hipMalloc((void**)&b->ditems, std::max<size_t>(items.size(), 1) * sizeof(GItem<float>)));
  BTRY(hipMemcpy(b->ditems, items.data(), items.size() * sizeof(GItem<float>),
                 hipMemcpyHostToDevice));

  // ---- FP64 refinement step items, both parities ----
  std::vector<GItemCR> cr[2];
  int blk = 0;
  b->pair_blk0.assign(b->npairs, 0);
  b->pair_nblk.assign(b->npairs, 0);
  for (int q = 0; q < b->npairs; ++q) {
    const gmg_ctx* c = b->inst[b->pair_inst[q]];
    const Lvl<double> L0 = view<double>(c, 0);
    const int nti = (int)stencil_tiles_x(L0.nx), ntj = (int)stencil_tiles_y(L0.ny);
    const int nb = nti * ntj * (int)stencil_tiles_k(L0.nz);
    for (int par = 0; par < 2; ++par) {
      GItemCR it{};
      it.L = L0;
      it.u = par == 0 ? b->pb[q].uA : b->pb[q].uB;
      it.uout = par == 0 ? b->pb[q].uB : b->pb[q].uA;
      it.e = b->pb[q].e32;
      it.f = b->pb[q].f;
      it.r32 = b->pb[q].r32;
      it.nti = nti;
      it.ntj = ntj;
      it.blk0 = blk;
      it.pair = q;
      cr[par].push_back(it);
    }
    b->pair_blk0[q] = blk;
    b->pair_nblk[q] = nb;
    blk += nb;
  }
  b->cr_nitems = b->npairs;
  b->cr_nblocks = blk;
  for (int par = 0; par < 2; ++par) {
    BTRY(hipMalloc((void**)&b->dcr[par], b->npairs * sizeof(GItemCR)));
    BTRY(hipMemcpy(b->dcr[par], cr[par].data(), b->npairs * sizeof(GItemCR),
                   hipMemcpyHostToDevice));
  }
  BTRY(hipMalloc((void**)&b->partials, std::max(blk, 1) * sizeof(double)));
  BTRY(hipMalloc((void**)&b->dstate, b->npairs * sizeof(PairState)));
  BTRY(hipMalloc((void**)&b->dactive, b->npairs * sizeof(int)));
  BTRY(hipHostMalloc((void**)&b->hstate, b->npairs * sizeof(PairState), hipHostMallocDefault));
  BTRY(hipHostMalloc((void**)&b->hactive, b->npairs * sizeof(int), hipHostMallocDefault));
  BTRY(hipStreamSynchronize(s));

  // ---- capture one graph per parity on a private stream ----
  BTRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  for (int par = 0; par < 2; ++par) {
    hipGraph_t g = nullptr;
    BTRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int st = enqueue_step(b, par, b->cap);
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    BTRY(e2);
    hipError_t e3 = hipGraphInstantiate(&b->gexec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BTRY(e3);
  }
  return GMG_OK;
}

}  // namespace

}  // namespace gmg

using gmg::Batch;

extern "C" {

int gmg_batch_setup(const gmg_params* inst, int ninst, int nrhs, void* stream, gmg_ctx** out) {
  if (!out) return gmg::set_error(GMG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!inst || ninst < 1 || nrhs < 1 || (int64_t)ninst * nrhs > (1 << 20))
    return gmg::set_error(GMG_EINVAL, "need inst != NULL, ninst >= 1, nrhs >= 1");
  for (int i = 0; i < ninst; ++i) {
    int st = gmg::validate_params(&inst[i]);
    if (st) return st;
    if (inst[i].rho != inst[0].rho || inst[i].ncoarse != inst[0].ncoarse)
      return gmg::set_error(GMG_EINVAL, "all instances of a batch share rho and ncoarse");
  }
  gmg_ctx* c = new (std::nothrow) gmg_ctx();
  Batch* b = new (std::nothrow) Batch();
  if (!c || !b) {
    delete c;
    delete b;
    return gmg::set_error(GMG_ENOMEM, "host allocation failed");
  }
  c->batch = b;
  c->p = inst[0];
  c->p.zfaces = nullptr;
  c->p.kh = nullptr;
  b->ninst = ninst;
  b->nrhs = nrhs;
  b->npairs = ninst * nrhs;
  b->rho = (float)inst[0].rho;
  b->ncoarse = inst[0].ncoarse;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < ninst; ++i) {
    gmg_params pi = inst[i];
    pi.prec_precond = GMG_F32;
    gmg_ctx* sub = nullptr;
    int st = gmg::setup_impl(&pi, stream, &sub, false);
    if (st) {
      gmg_destroy(c);
      return st;
    }
    b->inst.push_back(sub);
  }
  for (int q = 0; q < b->npairs; ++q) b->pair_inst.push_back(q / nrhs);
  int st = gmg::build(b, s);
  if (st) {
    gmg_destroy(c);
    return st;
  }
  *out = c;
  return GMG_OK;
}

int gmg_batch_layout(const gmg_ctx* c, int instance, int64_t* ldx, int64_t* elems) {
  if (!c || !c->batch) return gmg::set_error(GMG_EINVAL, "not a batched context");
  if (instance < 0 || instance >= c->batch->ninst)
    return gmg::set_error(GMG_EINVAL, "instance out of range");
  return gmg_field_layout(c->batch->inst[instance], 0, ldx, elems);
}

int gmg_batch_solve(gmg_ctx* c, const double* const* f, double* const* u, double rtol, int maxit,
                    int* iters, double* relres, void* stream) {
  if (!c || !c->batch) return gmg::set_error(GMG_EINVAL, "not a batched context");
  Batch* b = c->batch;
  if (!f || !u) return gmg::set_error(GMG_EINVAL, "f and u arrays must not be NULL");
  if (!(rtol > 0.0)) return gmg::set_error(GMG_EINVAL, "rtol must be > 0");
  if (maxit < 0) return gmg::set_error(GMG_EINVAL, "maxit must be >= 0");
  for (int q = 0; q < b->npairs; ++q) {
    if (!f[q] || !u[q] || (reinterpret_cast<uintptr_t>(f[q]) | reinterpret_cast<uintptr_t>(u[q])) % 16)
      return gmg::set_error(GMG_EINVAL, "NULL or misaligned field pointer");
    if (f[q] == u[q]) return gmg::set_error(GMG_EINVAL, "f and u must not overlap");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // inputs into the arenas; e = 0 for the initial residual
  for (int q = 0; q < b->npairs; ++q) {
    const size_t bytes = (size_t)b->inst[b->pair_inst[q]]->lev[0].elems * sizeof(double);
    BTRY(hipMemcpyAsync(b->pb[q].f, f[q], bytes, hipMemcpyDeviceToDevice, s));
    BTRY(hipMemcpyAsync(b->pb[q].uA, u[q], bytes, hipMemcpyDeviceToDevice, s));
  }
  BTRY(gmg::launch_fill<float>(b->e32_all, (int64_t)b->e32_len, 0.0f, s));
  for (int q = 0; q < b->npairs; ++q) {
    gmg::PairState& P = b->hstate[q];
    memset(&P, 0, sizeof(P));
    P.thresh2 = rtol * rtol;
    P.maxit = maxit;
    P.blk0 = b->pair_blk0[q];
    P.nblk = b->pair_nblk[q];
    b->hactive[q] = 1;
  }
  BTRY(hipMemcpyAsync(b->dstate, b->hstate, b->npairs * sizeof(gmg::PairState),
                      hipMemcpyHostToDevice, s));
  BTRY(hipMemcpyAsync(b->dactive, b->hactive, b->npairs * sizeof(int), hipMemcpyHostToDevice, s));
  // initial residual r_0 = f - A u_0 (uA + 0 -> uB)
  BTRY(gmg::launch_grouped_cr(b->dcr[0], b->cr_nitems, b->cr_nblocks, b->dactive, b->partials, s));
  BTRY(gmg::launch_pair_reduce(b->dstate, b->dactive, b->partials, b->npairs, 1, s));
  // iteration n reads the iterate from parity (n-1) and writes parity n:
  // P(0) = uB, P(1) = uA, ...  graph 1 maps uB -> uA, graph 0 uA -> uB
  for (int n = 1; n <= maxit; ++n) {
    BTRY(hipMemcpyAsync(b->hactive, b->dactive, b->npairs * sizeof(int), hipMemcpyDeviceToHost, s));
    BTRY(hipStreamSynchronize(s));
    int live = 0;
    for (int q = 0; q < b->npairs; ++q) live += b->hactive[q];
    if (!live) break;
    BTRY(hipGraphLaunch(b->gexec[(n % 2 == 1) ? 1 : 0], s));
  }
  BTRY(hipMemcpyAsync(b->hstate, b->dstate, b->npairs * sizeof(gmg::PairState),
                      hipMemcpyDeviceToHost, s));
  BTRY(hipMemcpyAsync(b->hactive, b->dactive, b->npairs * sizeof(int), hipMemcpyDeviceToHost, s));
  BTRY(hipStreamSynchronize(s));
  int bad = 0;
  for (int q = 0; q < b->npairs; ++q) {
    const gmg::PairState& P = b->hstate[q];
    const double* res = (P.iters % 2 == 0) ? b->pb[q].uB : b->pb[q].uA;
    const size_t bytes = (size_t)b->inst[b->pair_inst[q]]->lev[0].elems * sizeof(double);
    BTRY(hipMemcpyAsync(u[q], res, bytes, hipMemcpyDeviceToDevice, s));
    if (iters) iters[q] = P.iters;
    if (relres) relres[q] = P.rr0 > 0.0 ? sqrt(P.rr / P.rr0) : 0.0;
    const bool conv = P.status == 0 && (P.rr0 == 0.0 || P.rr < P.thresh2);
    if (!conv || b->hactive[q]) bad++;
  }
  BTRY(hipStreamSynchronize(s));
  if (bad) {
    char m[128];
    snprintf(m, sizeof(m), "%d of %d pairs did not converge to %g in %d cycles", bad, b->npairs,
             rtol, maxit);
    return gmg::set_error(GMG_ENOCONV, m);
  }
  return GMG_OK;
}

}  // extern "C"
