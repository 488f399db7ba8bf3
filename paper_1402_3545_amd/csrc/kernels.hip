// gfx950 kernels of the tensor-product multigrid / line-preconditioned CG path.
//
// Paper: Mueller, Scheichl & Vainikko, arXiv:1402.3545.  Kernel names follow
// Sec. 3.1 (SpMV, Tridiag, Smooth, Residual, ResSmooth, Prolongate).
//
// Layout: x-contiguous (Sec. 3.1): element (i,j,k) at (j*nz + k)*ldx + i, so a
// wavefront reading 32 or 64 consecutive i touches whole 128-byte lines.
//
// Two kernel shapes:
//  * stencil kernels (SpMV, Residual, the CG SpMV step, Prolongate): one thread
//    per column segment of KSEG layers, vertical neighbours rolled through
//    registers; east/west neighbours passed between the lanes of a wavefront
//    (DPP wave shifts, only the two edge lanes load theirs), north/south
//    neighbours loaded directly (they hit L1/L2).
//  * line kernels (Tridiag, Smooth, ResSmooth): the tridiagonal system of each
//    column is solved by two lanes of one wavefront.  Lane l < 32 eliminates
//    upwards from the bottom layer, lane l + 32 downwards from the top layer;
//    they meet in the middle, exchange their last elimination coefficients
//    with one cross-lane swap, solve the 2x2 interface system and
//    back-substitute outwards.  This is Gaussian elimination without pivoting
//    in a twisted order (exact for the diagonally dominant column matrices);
//    each lane keeps only ceil(nz/2) pairs (c', d') in registers, so the whole
//    elimination stays on chip and the kernel streams each field once.
//
// Workgroup ids are remapped so that each of the 8 XCDs (each with its own L2)
// works on a contiguous band of tiles: neighbouring tiles share halo rows.

#include <type_traits>

#include "gmg_internal.h"

namespace gmg {

namespace {

constexpr int KSEG = 32;        // layers per thread in stencil kernels
constexpr int SROWS = 4;        // rows (j) per stencil workgroup, 64 columns wide
constexpr int LROWS = 4;        // rows (j) per line workgroup, 32 columns wide
constexpr int NTHREADS = 256;

__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int x = b & 7, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + (b >> 3);
}

// A gated launch (a solver's iteration enqueued past its convergence)
// returns at once; the flag is uniform, so whole workgroups leave together.
template <typename T>
__device__ __forceinline__ bool gated(const Lvl<T>& L) {
  return L.gate && *L.gate;
}

template <typename T>
struct Col {
  int64_t base;              // index of (i, j, 0)
  int64_t oe, ow, on, os;    // offsets to the four horizontal neighbours
  T ce, cw, cn, cs, S;       // face couplings and their sum
};

template <typename T>
__device__ __forceinline__ Col<T> load_col(const Lvl<T>& L, int i, int j) {
  Col<T> c;
  const int nx = L.nx, ny = L.ny;
  const int ie = (i + 1 == nx) ? 0 : i + 1;
  const int iw = (i == 0) ? nx - 1 : i - 1;
  const int jn = (j + 1 == ny) ? 0 : j + 1;
  const int js = (j == 0) ? ny - 1 : j - 1;
  const int64_t row = (int64_t)j * nx;
  c.ce = L.cx[row + i];
  c.cw = L.cx[row + iw];
  c.cn = L.cy[row + i];
  c.cs = L.cy[(int64_t)js * nx + i];
  c.S = c.ce + c.cw + c.cn + c.cs + L.wall[row + i];
  const int64_t jstride = (int64_t)L.nz * L.ldx;
  c.base = (int64_t)j * jstride + i;
  c.oe = ie - i;
  c.ow = iw - i;
  c.on = (int64_t)(jn - j) * jstride;
  c.os = (int64_t)(js - j) * jstride;
  return c;
}

// Sum NC per-thread values over the workgroup; thread 0 stores them to
// partials[blockIdx.x*NC + c].  Fixed order, so results are reproducible.
template <int NC, int NW = NTHREADS / 64>
__device__ __forceinline__ void block_partials(double (&v)[NC], double* __restrict__ partials) {
  __shared__ double sm[NC][NW];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < NC; ++c) sm[c][w] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += sm[c][q];
      partials[(int64_t)blockIdx.x * NC + c] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Stencil kernels.  A workgroup is SR wavefronts; wavefront w owns grid row
// j = tj*SR + w (wave-uniform, so the row bases of every field are scalar
// registers and each lane needs only 32-bit byte offsets) and 64 consecutive
// columns; each lane walks its column through the KSEG layers of the
// workgroup's segment.  The loads of the next CH layers are issued before the
// current CH layers are computed and stored (a register double buffer): with
// updates in place the compiler may not move a load of layer k+1 above a
// store to layer k itself, and without the buffer every layer would wait for
// the previous layer's stores.  The vertical profiles of the segment are
// staged in LDS.
// ---------------------------------------------------------------------------
struct Geo {
  int j, jn, js;   // the wavefront's grid row and its periodic neighbours
  int ic, ie, iw;  // the lane's column (clamped into the grid) and its neighbours
  bool row, act;   // the row exists (wave-uniform); the lane's column exists
  bool ft;         // all 64 columns of the tile exist (wave-uniform)
  int k0, n;       // first layer and number of layers of the segment (uniform)
};

// Tile coordinates of logical workgroup b (all wave-uniform).  Tiles are
// walked in groups of `group` tile columns: inside a group the tiles of one
// tile row are adjacent and tile rows follow each other, so a tile's
// east/west and north/south neighbours run within a few workgroups of it and
// its halo rows are still in the XCD's L2.  group <= 0 or >= nti: row-major.
// Segments of layers (kb) vary slowest.
__device__ __forceinline__ void tile_coords(int b, int nti, int ntj, int group, int& ti, int& tj,
                                            int& kb) {
  const int per = nti * ntj;
  kb = b / per;
  int r = b - kb * per;
  if (group <= 0 || group >= nti) {
    tj = r / nti;
    ti = r - tj * nti;
    return;
  }
  const int gsize = group * ntj;
  const int gi = r / gsize;
  const int g0 = gi * group;
  const int w = min(group, nti - g0);
  r -= gi * gsize;
  tj = r / w;
  ti = g0 + (r - tj * w);
}

template <int SR, int KS = KSEG>
__device__ __forceinline__ Geo stencil_geo(int nx, int ny, int nz, int nti, int ntj, int group,
                                           int b) {
  Geo g;
  int ti, tj, kb;
  tile_coords(b, nti, ntj, group, ti, tj, kb);
  const int i = ti * 64 + (int)(threadIdx.x & 63);
  const int j = tj * SR + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  g.row = j < ny;
  g.j = min(j, ny - 1);
  g.jn = (g.j + 1 == ny) ? 0 : g.j + 1;
  g.js = (g.j == 0) ? ny - 1 : g.j - 1;
  g.act = i < nx;
  g.ft = ti * 64 + 64 <= nx;
  g.ic = min(i, nx - 1);
  g.ie = (g.ic + 1 == nx) ? 0 : g.ic + 1;
  g.iw = (g.ic == 0) ? nx - 1 : g.ic - 1;
  g.k0 = kb * KS;
  g.n = min(nz - g.k0, KS);
  return g;
}

template <typename T>
struct Prof {
  T sub, sup, dg, dz;
};

// Vertical profiles of layers k0 .. k0+KS-1 (clamped) into LDS.
template <typename T, int KS = KSEG>
__device__ __forceinline__ void stage_prof(const Lvl<T>& L, int k0, Prof<T>* sp) {
  for (int t = threadIdx.x; t < KS; t += blockDim.x) {
    const int k = min(k0 + t, L.nz - 1);
    sp[t] = Prof<T>{L.sub[k], L.sup[k], L.dg[k], L.dz[k]};
  }
  __syncthreads();
}

// Face couplings of the lane's column and their sum.
template <typename T>
struct Cf {
  T ce, cw, cn, cs, S;
};

template <typename T>
__device__ __forceinline__ Cf<T> col_coef(const Lvl<T>& L, const Geo& g) {
  const int64_t row = (int64_t)g.j * L.nx;
  Cf<T> c;
  c.ce = L.cx[row + g.ic];
  c.cw = L.cx[row + g.iw];
  c.cn = L.cy[row + g.ic];
  c.cs = L.cy[(int64_t)g.js * L.nx + g.ic];
  c.S = c.ce + c.cw + c.cn + c.cs + L.wall[row + g.ic];
  return c;
}

// Byte base of grid row j of a field (layer 0, column 0).
template <typename T>
__device__ __forceinline__ const char* rowc(const T* f, int j, int64_t jstride) {
  return reinterpret_cast<const char*>(f + (int64_t)j * jstride);
}
template <typename T>
__device__ __forceinline__ char* roww(T* f, int j, int64_t jstride) {
  return reinterpret_cast<char*>(f + (int64_t)j * jstride);
}

// Load/store through a wave-uniform base and a 32-bit per-lane byte offset
// (the saddr form of the global memory instructions).  Stores are
// non-temporal: every output is written once and read by a later kernel, so
// it should not displace the halo rows the L2 is holding for neighbouring
// tiles.  ldn is the non-temporal load for fields a kernel reads exactly once
// (no halo); fields read with horizontal neighbours use ldo.
template <typename T>
__device__ __forceinline__ T ldo(const char* base, uint32_t off) {
  return *reinterpret_cast<const T*>(base + off);
}
template <typename T>
__device__ __forceinline__ T ldn(const char* base, uint32_t off) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(base + off));
}
// non-temporal load of a pair (double2 / float2) as one 16- or 8-byte access
template <typename V>
__device__ __forceinline__ V ldn2(const char* base, uint32_t off) {
  using E = decltype(V{}.x);
  typedef E N2 __attribute__((ext_vector_type(2)));
  const N2 t = __builtin_nontemporal_load(reinterpret_cast<const N2*>(base + off));
  return V{t.x, t.y};
}
template <typename T>
__device__ __forceinline__ void sto(char* base, uint32_t off, T v) {
  if constexpr (std::is_arithmetic_v<T>)
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(base + off));
  else
    *reinterpret_cast<T*>(base + off) = v;
}

// The layer walk shared by the stencil kernels: P supplies the per-layer
// input record In, load(s, In&) for layer k0+s and step(s, const In&) that
// computes and stores layer k0+s.  FULL: the segment has all KS layers.
template <int CH, bool FULL, int KS = KSEG, typename P>
__device__ __forceinline__ void walk(P& pol, int n) {
  using In = typename P::In;
  static_assert(KS % CH == 0, "whole chunks per segment");
  constexpr int NCH = KS / CH;
  In buf[2][CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) pol.load(t, buf[0][t]);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    if (ch + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) pol.load((ch + 1) * CH + t, buf[(ch + 1) & 1][t]);
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int st = ch * CH + t;
      if (FULL || st < n) pol.step(st, buf[ch & 1][t]);
    }
    // keep later chunks' loads from being hoisted further (registers)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// A value from another lane of the wavefront by a DPP wave shift: CTRL
// kWaveShl1 gives lane l the value of lane l+1, kWaveShr1 that of lane l-1
// (the lane at the end receives 0).  Every lane of the wavefront must be
// active.
constexpr int kWaveShl1 = 0x130;
constexpr int kWaveShr1 = 0x138;
template <int CTRL, typename T>
__device__ __forceinline__ T wave_shift(T v) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf,
                                                              0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL,
                                                              0xf, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
  }
}

// The 7-point operator on one lane's column, rolled through registers:
// (A x)_k = (dg_k + dz_k S) x_k - dz_k (Kh-weighted sum of the four horizontal
// neighbours) + sub_k x_{k-1} + sup_k x_{k+1}, x_{-1} = x_{nz} = 0.
// x is stored as TS (FP32 for the mixed-precision flexible CG), the
// arithmetic is in T.  Byte offsets oc/oe/ow and kb refer to TS elements.
// X (tiles whose 64 columns all exist): the east and west values of layer k
// are the neighbouring lanes' own x_k, passed by wave shifts; one load per
// layer brings lane 0 its west and lane 63 its east value (the tile's halo)
// in the xe slot, and the other lanes their own x_k again (an L1 hit; no
// branch, so the loads of a chunk stay one straight-line batch).
template <typename T, typename TS = T, bool X = false>
struct ColumnOp {
  const char *rx, *rxn, *rxs;
  uint32_t oc, oe, ow, kb, oh;
  int nz, k0;
  bool ew, ee;  // X: the lane is the tile's west / east edge
  Cf<T> c;
  const Prof<T>* sp;
  T xm, xc;

  __device__ __forceinline__ void init(const TS* x, const Geo& g, int64_t jstride,
                                       uint32_t kbytes, const Cf<T>& cf, const Prof<T>* prof,
                                       int nz_) {
    rx = rowc(x, g.j, jstride);
    rxn = rowc(x, g.jn, jstride);
    rxs = rowc(x, g.js, jstride);
    oc = (uint32_t)g.ic * sizeof(TS);
    oe = (uint32_t)g.ie * sizeof(TS);
    ow = (uint32_t)g.iw * sizeof(TS);
    kb = kbytes;
    nz = nz_;
    k0 = g.k0;
    c = cf;
    sp = prof;
    if constexpr (X) {
      const int lane = (int)(threadIdx.x & 63);
      ew = lane == 0;
      ee = lane == 63;
      oh = ew ? ow : ee ? oe : oc;
    }
    xm = k0 > 0 ? (T)ldo<TS>(rx, oc + (uint32_t)(k0 - 1) * kb) : T(0);
    xc = (T)ldo<TS>(rx, oc + (uint32_t)k0 * kb);
  }
  // x at k+1 (clamped address), and the horizontal neighbours at k (X: the
  // edge lanes' halo value in xe, xw unused)
  __device__ __forceinline__ void load(uint32_t ok, uint32_t okp, T& xp, T& xe, T& xw, T& xn,
                                       T& xs) const {
    xp = (T)ldo<TS>(rx, oc + okp);
    if constexpr (X) {
      xe = (T)ldo<TS>(rx, oh + ok);
    } else {
      xe = (T)ldo<TS>(rx, oe + ok);
      xw = (T)ldo<TS>(rx, ow + ok);
    }
    xn = (T)ldo<TS>(rxn, oc + ok);
    xs = (T)ldo<TS>(rxs, oc + ok);
  }
  // (A x) at layer k0+s; advances the rolled column
  __device__ __forceinline__ T apply(int s, T xp_raw, T xe_in, T xw_in, T xn, T xs) {
    const Prof<T> pr = sp[s];
    const T xp = (k0 + s + 1 < nz) ? xp_raw : T(0);
    T xe = xe_in, xw = xw_in;
    if constexpr (X) {
      const T de = wave_shift<kWaveShl1>(xc), dw = wave_shift<kWaveShr1>(xc);
      xe = ee ? xe_in : de;
      xw = ew ? xe_in : dw;
    }
    const T h = c.ce * xe + c.cw * xw + c.cn * xn + c.cs * xs;
    const T ax = (pr.dg + pr.dz * c.S) * xc - pr.dz * h + pr.sub * xm + pr.sup * xp;
    xm = xc;
    xc = xp;
    return ax;
  }
};

// Layer offsets: FULL segments never reach past nz-1; ragged ones clamp.
template <bool FULL>
__device__ __forceinline__ uint32_t layer_off(int k, int nz, uint32_t kb) {
  return (uint32_t)(FULL ? k : min(k, nz - 1)) * kb;
}

// SpMV (y = Ax) and Residual (r = f - Ax, optional ||r||^2 partials and an
// FP32 copy of r for the mixed-precision refinement).
template <typename T, int MODE, bool FULL, bool X>
struct StencilPol {
  struct In {
    T xp, xe, xw, xn, xs, f;
  };
  ColumnOp<T, T, X> op;
  const char* rf;
  char *ry, *rd;
  double nrm;

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = op.k0 + s;
    const uint32_t ok = layer_off<FULL>(k, op.nz, op.kb);
    const uint32_t okp = (uint32_t)min(k + 1, op.nz - 1) * op.kb;
    op.load(ok, okp, v.xp, v.xe, v.xw, v.xn, v.xs);
    if constexpr (MODE != (int)Stencil::SPMV) v.f = ldn<T>(rf, op.oc + ok);
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const uint32_t o = op.oc + layer_off<FULL>(op.k0 + s, op.nz, op.kb);
    const T ax = op.apply(s, v.xp, v.xe, v.xw, v.xn, v.xs);
    if constexpr (MODE == (int)Stencil::SPMV) {
      sto<T>(ry, o, ax);
    } else {
      const T rr = v.f - ax;
      sto<T>(ry, o, rr);
      if constexpr (MODE >= (int)Stencil::RESIDUAL_NORM) nrm += (double)rr * (double)rr;
      if constexpr (MODE == (int)Stencil::RESIDUAL_NORM_DOWN)
        sto<float>(rd, o / sizeof(T) * sizeof(float), (float)rr);
    }
  }
};

template <typename T, int MODE, int SR>
__global__ __launch_bounds__(64 * SR) void k_stencil(Lvl<T> L, const T* __restrict__ x,
                                                     const T* __restrict__ f, T* __restrict__ y,
                                                     float* __restrict__ ydown,
                                                     double* __restrict__ partials, int nti,
                                                     int ntj, int group) {
  constexpr int CH = sizeof(T) == 8 ? 4 : 8;
  if (gated(L)) return;
  const Geo g =
      stencil_geo<SR>(L.nx, L.ny, L.nz, nti, ntj, group, xcd_remap(blockIdx.x, gridDim.x));
  __shared__ Prof<T> sp[KSEG];
  stage_prof(L, g.k0, sp);
  double nrm[1] = {0.0};
  if (g.row && g.act) {
    const int64_t jstride = (int64_t)L.nz * L.ldx;
    const uint32_t kb = (uint32_t)(L.ldx * sizeof(T));
    const Cf<T> cf = col_coef(L, g);
    auto run = [&](auto full, auto xch) {
      constexpr bool F = decltype(full)::value, XC = decltype(xch)::value;
      StencilPol<T, MODE, F, XC> pol;
      pol.op.init(x, g, jstride, kb, cf, sp, L.nz);
      pol.rf = MODE != (int)Stencil::SPMV ? rowc(f, g.j, jstride) : nullptr;
      pol.ry = roww(y, g.j, jstride);
      pol.rd = MODE == (int)Stencil::RESIDUAL_NORM_DOWN ? roww(ydown, g.j, jstride) : nullptr;
      pol.nrm = 0.0;
      walk<CH, F>(pol, g.n);
      nrm[0] = pol.nrm;
    };
    if (g.ft) {
      if (g.n == KSEG)
        run(std::true_type{}, std::true_type{});
      else
        run(std::false_type{}, std::true_type{});
    } else {
      if (g.n == KSEG)
        run(std::true_type{}, std::false_type{});
      else
        run(std::false_type{}, std::false_type{});
    }
  }
  if constexpr (MODE >= (int)Stencil::RESIDUAL_NORM) block_partials<1, SR>(nrm, partials);
}

// u + (9 a + wb b + wc c + wd d) / 16: the cell-centred bilinear correction of
// one fine cell from its coarse parent a, x and y neighbours b, c and diagonal
// d, with the fused multiply-adds spelled out so that every kernel that forms
// it (the prolongation, and the smoother that folds it in) rounds the same way.
template <typename T>
__device__ __forceinline__ T prolong_add(T u, T a, T b, T c, T d, T wb, T wc, T wd) {
  T p = T(9) * a;
  p = fma(wb, b, p);
  p = fma(wc, c, p);
  p = fma(wd, d, p);
  return fma(p, T(0.0625), u);
}

// ---------------------------------------------------------------------------
// Line kernels
// ---------------------------------------------------------------------------
enum LineMode {
  LINE_SOLVE = 0,          // z = rho M^-1 r (rho = 1 for the plain line solve)
  LINE_SMOOTH = 1,         // u' = u + rho M^-1 (f - A u)
  LINE_RESTRICT_SMOOTH = 2,
  LINE_CG = 3,
  LINE_SMOOTH_NORM = 4,    // LINE_SMOOTH plus ||f - A u||^2 partials
  LINE_PROLONG_SMOOTH = 5  // LINE_SMOOTH of u + P u_c: the prolongation folded in
};

template <typename T>
struct LineArgs {
  const T* a;         // SOLVE: r; SMOOTH: u_in; RESTRICT_SMOOTH: fine r; CG: q
  const T* b;         // SMOOTH: f
  T* rw;              // CG: r (updated in place)
  T* o0;              // SOLVE: z; SMOOTH: u_out; RESTRICT_SMOOTH: coarse u; CG: z
  T* o1;              // RESTRICT_SMOOTH: coarse f
  T rho;              // SOLVE: output scale; SMOOTH*, RESTRICT_SMOOTH: damping
  Lvl<T> F;           // RESTRICT_SMOOTH: the fine level
  const CgState* st;  // CG
  int init;           // CG: initial step (alpha = 0)
  double* partials;   // CG: <r,r>, <r,z>; SMOOTH_NORM: ||f - A u||^2 per workgroup
  Lvl<T> C;           // PROLONG_SMOOTH: the coarse level
  const T* uc;        // PROLONG_SMOOTH: the coarse-level correction
};

template <typename T>
struct Vec2;
template <>
struct Vec2<double> { using type = double2; };
template <>
struct Vec2<float> { using type = float2; };

// Reciprocal: hardware estimate refined by Newton-Raphson steps
// r <- r (2 - p r), written as e = 1 - p r, r <- r + r e (two steps in FP64,
// one in FP32 bring the estimate to the last bit or so).  Pivots here are
// positive and well scaled, so no special cases arise.
__device__ __forceinline__ double rcp_nr(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = fma(-p, r, 1.0);
  r = fma(r, e, r);
  e = fma(-p, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float p) {
  const float r = __builtin_amdgcn_rcpf(p);
  const float e = fmaf(-p, r, 1.0f);
  return fmaf(r, e, r);
}

// One elimination step: pivot, its reciprocal and the new c' of this row.
// The line kernels spell out every fused multiply-add, so that each kernel
// (and the back sweep's recomputation of the forward sweep) rounds the same
// way whatever the compiler would contract.
template <typename T>
__device__ __forceinline__ void elim_step(T diag, T cpv, T cnx, T cprev, T& piv, T& inv, T& c) {
  piv = fma(-cpv, cprev, diag);
  inv = rcp_nr(piv);
  c = cnx * inv;
}

// Values one elimination step reads from memory (loaded a chunk ahead).
template <typename T, int MODE>
struct StepIn;
template <typename T>
struct StepIn<T, LINE_SOLVE> { T r; };
template <typename T>
struct StepIn<T, LINE_SMOOTH> { T un, ue, uw, unn, us, f; };
template <typename T>
struct StepIn<T, LINE_SMOOTH_NORM> { T un, ue, uw, unn, us, f; };
template <typename T>
struct StepIn<T, LINE_RESTRICT_SMOOTH> { typename Vec2<T>::type lo, hi; };
template <typename T>
struct StepIn<T, LINE_CG> { T r, q; };
// Smoothers with the horizontal neighbours staged in LDS: the lane's next row
// (un), f, and one value of the workgroup's halo (ex).
template <typename T>
struct StepNb { T un, f, ex; };
// ... and, with the prolongation folded in, one value of the coarse tile (cv).
template <typename T>
struct StepNbP { T un, f, ex, cv; };
// Two wavefronts per column (W2): lanes 0 and 1 also bring the value left or
// right of the tile in the wavefront's row (ew).
template <typename T>
struct StepNb2 { T un, f, ex, ew; };
template <typename T>
struct StepNbP2 { T un, f, ex, cv, ew; };

// Body of the line kernels for tile b of a level (tiles of 32 columns x LROWS
// rows, nti tiles across; wavefront w of the workgroup owns grid row
// tj*LROWS + w).  Block partials go to a.partials[blockIdx.x].
//
// Every column is treated as 2*HALF rows: rows k >= nz are identity rows
// (diagonal 1, no coupling, zero right-hand side) that do not touch the real
// nz x nz block (its last row has no super-diagonal), so one branch-free,
// fully unrolled sweep serves every nz <= 2*HALF.  Addresses of virtual rows
// are clamped to a real row and their results are not stored.  The vertical
// profiles (padded the same way) are staged in LDS once per workgroup.
//
// Registers: the forward sweep keeps d' of its HALF rows and a c' checkpoint
// every G rows; the loads of each chunk of CH steps are issued one chunk
// ahead (double buffer) so that memory latency overlaps the elimination.  The
// back sweep recomputes c' (and the pivots) of each G-row segment from its
// checkpoint and substitutes backwards.
//
// EX (nz == 2*HALF, the column heights of the workloads): no virtual rows, so
// no clamped addresses and no masks; every stream advances by a running byte
// offset per step instead of recomputing its address from the row.
//
// W2 (staged smoothers, EX): the two halves of a column go to two wavefronts
// instead of two lanes of one: wavefront w owns tile row w >> 1 and half
// w & 1 of 64 consecutive columns (tiles of 64 columns x 2 rows), so that
// every load and store instruction covers 64 consecutive values of one layer
// (512 bytes in FP64) instead of two 32-value runs of two layers, which the
// memory system serves measurably faster; the halves swap their last
// elimination coefficients through LDS.  Same arithmetic: the same iterate.
template <typename T, int HALF, int MODE, bool NB = false, bool EX = false, bool W2 = false>
__device__ __forceinline__ void line_body(const Lvl<T>& L, const LineArgs<T>& a, int nti,
                                          int ntj, int group, int b) {
  constexpr int NR = 2 * HALF;
  // the prolongation folded into the post-smoother (staged form only)
  constexpr bool PRO = MODE == LINE_PROLONG_SMOOTH;
  constexpr bool kSmooth = (MODE == LINE_SMOOTH || MODE == LINE_SMOOTH_NORM || PRO);
  static_assert(!PRO || NB, "the prolongation is folded into the staged smoother only");
  // smoothers only: horizontal neighbours through LDS instead of per-lane loads
  constexpr bool NBL = NB && kSmooth;
  static_assert(!NBL || LROWS == 4, "the staged halo assumes four rows per workgroup");
  static_assert(!W2 || (NBL && EX), "two wavefronts per column: staged smoothers, exact heights");
  constexpr int TROWS = W2 ? 2 : LROWS;   // grid rows of a tile
  constexpr int TCOLS = W2 ? 64 : 32;     // columns of a tile
  constexpr int G = HALF < 8 ? HALF : 8;                       // back-sweep segment
  constexpr int NG = HALF / G;
  // prefetch chunk: bounded by the registers the buffered loads take
  // (FP64 with the prolongation folded in: 2, or the coarse values would
  // push the kernel past 256 registers; the FP64 CG step, two values per
  // step: 8, measured 786 -> 773 us at 1024^2 x 128 against 4)
  constexpr int CHW = (MODE == LINE_SOLVE || sizeof(T) == 4) && MODE != LINE_RESTRICT_SMOOTH
                          ? (kSmooth ? 4 : 8)
                          : (PRO ? 2 : MODE == LINE_CG ? 8 : 4);
  constexpr int CH = HALF < CHW ? HALF : CHW;
  constexpr int NCH = HALF / CH;
  constexpr uint32_t ES = sizeof(T);
  using V2 = typename Vec2<T>::type;
  // vertical profiles in each half's elimination order: step s of half h is
  // row k = s (h = 0) or NR-1-s (h = 1), and holds the coupling to the
  // previously eliminated row, the coupling to the next one, the diagonal
  // and dz (identity rows beyond nz), so that a step reads them at a
  // compile-time offset from its half's base, with no selects
  // (the two halves' tables are 4 values apart from 2 HALF x 4, so that the
  // lanes of the two halves, reading step s at once, hit different banks)
  constexpr int PSH = HALF * 4 + 4;
  __shared__ T s_ps[2 * PSH];
  const int nz = L.nz;
  for (int q = threadIdx.x; q < 2 * HALF; q += blockDim.x) {
    const int h = q / HALF, st = q - h * HALF;
    const int k = h ? NR - 1 - st : st;
    const bool real = k < nz;
    const T sub = real ? L.sub[k] : T(0), sup = real ? L.sup[k] : T(0);
    T* pq = s_ps + h * PSH + 4 * st;
    pq[0] = h ? sup : sub;
    pq[1] = h ? sub : sup;
    pq[2] = real ? L.dg[k] : T(1);
    pq[3] = real ? L.dz[k] : T(0);
  }
  __syncthreads();
  int ti, tj, kb_unused;
  tile_coords(b, nti, ntj, group, ti, tj, kb_unused);
  const int lane = threadIdx.x & 63;
  const int wv = (int)(threadIdx.x >> 6);
  // W2: the half is the wavefront's (uniform); otherwise the lane's
  const int half = W2 ? __builtin_amdgcn_readfirstlane(wv & 1) : lane >> 5;
  const int xl = W2 ? lane : (lane & 31);
  const int rt = W2 ? (wv >> 1) : wv;  // tile row of the wavefront
  const int i = ti * TCOLS + xl;
  // the row of the wavefront, made visibly uniform so that row bases live in
  // SGPRs
  const int j = tj * TROWS + __builtin_amdgcn_readfirstlane(rt);
  const bool active = (i < L.nx) && (j < L.ny);
  // inactive lanes compute on a valid column and store nothing; they still
  // take part in the cross-lane exchange.  With the staged neighbours they
  // take the periodic image of their column and row, so that the values they
  // stage are the neighbours the active lanes need across the grid's edge.
  const int ic = NBL ? (i < L.nx ? i : i % L.nx) : min(i, L.nx - 1);
  const int jc = NBL ? (j < L.ny ? j : j % L.ny) : min(j, L.ny - 1);
  const Col<T> c = load_col(L, ic, jc);
  const int jn = (jc + 1 == L.ny) ? 0 : jc + 1;
  const int js = (jc == 0) ? L.ny - 1 : jc - 1;
  const int ie = (ic + 1 == L.nx) ? 0 : ic + 1;
  const int iw = (ic == 0) ? L.nx - 1 : ic - 1;
  const int64_t jstride = (int64_t)nz * L.ldx;
  const uint32_t kbytes = (uint32_t)L.ldx * ES;   // one layer
  const int k0 = half ? NR - 1 : 0;
  const int dir = half ? -1 : 1;

  // Staged neighbours: every chunk of CH steps, the workgroup writes the u
  // values of its 4 rows, the rows above and below them and the columns left
  // and right of its 32 columns, at the layers of both halves, into LDS; each
  // wave contributes its own row (the lanes' current rows) and one halo value
  // per lane and step (wave 0 the row below, wave 3 the row above, waves 1
  // and 2 the side columns of the two halves' layers).
  const char* exbase = nullptr;
  const char* ewbase = nullptr;  // W2: the value left (lane 0) or right (lane 1) of the tile
  int exh = half;
  if constexpr (NBL) {
    const int i0 = ti * TCOLS, j0 = tj * TROWS;
    auto wrapx = [&](int q) { q %= L.nx; return q < 0 ? q + L.nx : q; };
    auto wrapy = [&](int q) { q %= L.ny; return q < 0 ? q + L.ny : q; };
    int exrow, excol;
    if (W2) {
      // every lane: its column in the row below (tile row 0) or above
      // (tile row 1) the tile
      exrow = rt == 0 ? wrapy(j0 - 1) : wrapy(j0 + 2);
      excol = ic;
      // lanes 0 and 1: the value left and right of the tile in the row; the
      // others load their own column (a cache hit) so that no lane branches
      const int ewcol = lane == 0 ? wrapx(i0 - 1) : (lane == 1 ? wrapx(i0 + 64) : ic);
      ewbase = reinterpret_cast<const char*>(a.a + (int64_t)jc * jstride + ewcol);
    } else if (wv == 0) {
      exrow = wrapy(j0 - 1);
      excol = ic;
    } else if (wv == LROWS - 1) {
      exrow = wrapy(j0 + LROWS);
      excol = ic;
    } else {
      const int l = lane % 12;
      exrow = wrapy(j0 - 1 + (l >> 1));
      excol = (l & 1) ? wrapx(i0 + 32) : wrapx(i0 - 1);
      exh = wv - 1;
    }
    exbase = reinterpret_cast<const char*>(a.a + (int64_t)exrow * jstride + excol);
  }
  constexpr int NBW = TCOLS + 2, NBR = TROWS + 2;  // staged tile: rows x columns
  constexpr int NBSTEP = 2 * NBR * NBW;      // one step, both halves
  auto nbi = [&](int buf, int t, int h, int r, int x) {
    return ((buf * CH + t) * 2 + h) * NBR * NBW + r * NBW + x;
  };
  // + 64 slots that the lanes without a halo value write to (no branch)
  __shared__ T s_nb[NBL ? 2 * CH * NBSTEP + 64 : 1];
  // LDS slot of the lane's halo value at step 0 of buffer 0 (or its spare)
  int exslot = 0, ewslot = 0;
  bool exreal = true;
  if constexpr (W2) {
    exslot = nbi(0, 0, half, rt == 0 ? 0 : NBR - 1, xl + 1);
    // lanes 2.. write their value to a spare slot
    ewslot = lane < 2 ? nbi(0, 0, half, rt + 1, lane == 1 ? NBW - 1 : 0) : 2 * CH * NBSTEP + lane;
  } else if constexpr (NBL) {
    const bool rowhalo = wv == 0 || wv == LROWS - 1;
    exreal = rowhalo || lane < 12;
    const int r = wv == 0 ? 0 : (wv == LROWS - 1 ? NBR - 1 : (lane >> 1));
    const int x = rowhalo ? xl + 1 : ((lane & 1) ? NBW - 1 : 0);
    exslot = exreal ? nbi(0, 0, exh, r, x) : 2 * CH * NBSTEP + lane;
  }

  // Prolongation folded in (u + P u_c is smoothed; u + P u_c is never
  // stored): the fine values the workgroup stages (rows j0-1 .. j0+4, columns
  // i0-1 .. i0+32) take their corrections from the coarse columns
  // i0/2-1 .. i0/2+16 and rows j0/2-1 .. j0/2+2 (CNR x CNW).  Every chunk,
  // lanes 0 .. CNS-1 stage one coarse value each for every step of the chunk
  // and for the next chunk's first step (the layer of the last step's next
  // row), for both halves' layers; then each lane adds the 9/3/3/1 sum of
  // its own next rows and its halo value before they go to the fine stage.
  // Fine indices stay unwrapped (F.nx = 2 C.nx, so periodic images of fine
  // and coarse columns line up with the wrapped coarse loads); behind a wall
  // the coarse neighbour is the parent's mirror image with opposite sign.
  constexpr int CNW = W2 ? 34 : 18, CNR = W2 ? 3 : 4, CNS = 2 * CNR * CNW;
  constexpr int CST = CH + 1;
  __shared__ T s_cs[PRO ? CST * CNS + NTHREADS : 1];
  const char* cbase = nullptr;
  uint32_t ckb = 0;
  int chh = 0, cslot = 0;
  bool creal = false;
  // the four coarse slots of a fine cell, packed one per byte (a, b, c, d:
  // parent, x neighbour, y neighbour, diagonal; each < 72), with the mirror
  // signs of the x and y neighbours in bits 15 and 23
  uint32_t po = 0, pe = 0;  // own column (at the lane's half), halo value (at half exh)
  uint32_t pw2 = 0;         // W2: the value left or right of the tile (lanes 0, 1)
  if constexpr (PRO) {
    const int q = (int)threadIdx.x;
    creal = q < CNS;
    const int qq = creal ? q : 0;
    chh = qq / (CNR * CNW);
    const int cr = (qq / CNW) % CNR, cx = qq % CNW;
    const int ib = ti * (TCOLS / 2) - 1, jb = tj * (TROWS / 2) - 1;
    auto wrapn = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
    const int I = wrapn(ib + cx, a.C.nx), J = wrapn(jb + cr, a.C.ny);
    cbase = reinterpret_cast<const char*>(a.uc + (int64_t)J * a.C.nz * a.C.ldx + I);
    ckb = (uint32_t)a.C.ldx * ES;
    cslot = creal ? q : CST * CNS + q;
    // slots (relative to one step and half) of the four coarse values of the
    // fine cell (fi, fj) and the mirror signs
    auto slots = [&](int fi, int fj) -> uint32_t {
      const int I0 = fi >> 1, J0 = fj >> 1;
      int I2 = I0 + ((fi & 1) ? 1 : -1), J2 = J0 + ((fj & 1) ? 1 : -1);
      uint32_t mx = 0, my = 0;
      if (a.C.bch && (I2 < 0 || I2 >= a.C.nx)) {
        I2 = I0;
        mx = 1;
      }
      if (a.C.bch && (J2 < 0 || J2 >= a.C.ny)) {
        J2 = J0;
        my = 1;
      }
      const int x0 = I0 - ib, x2 = I2 - ib, y0 = J0 - jb, y2 = J2 - jb;
      return (uint32_t)(y0 * CNW + x0) | ((uint32_t)(y0 * CNW + x2) << 8) | (mx << 15) |
             ((uint32_t)(y2 * CNW + x0) << 16) | (my << 23) | ((uint32_t)(y2 * CNW + x2) << 24);
    };
    const int i0 = ti * TCOLS, j0 = tj * TROWS;
    po = slots(i, j);
    int hi = i, hj = j;  // lanes without a halo value: any cell of the tile
    if (W2) {
      hj = rt == 0 ? j0 - 1 : j0 + 2;
      pw2 = lane < 2 ? slots(lane == 1 ? i0 + 64 : i0 - 1, j) : po;
    } else if (wv == 0) {
      hj = j0 - 1;
    } else if (wv == LROWS - 1) {
      hj = j0 + LROWS;
    } else if (lane < 12) {
      hj = j0 - 1 + (lane >> 1);
      hi = (lane & 1) ? i0 + 32 : i0 - 1;
    }
    pe = slots(hi, hj);
  }
  // u + P u_c from the coarse stage (step t of the chunk, half h)
  // (the prolongation kernel's arithmetic: prolong_add)
  auto corr = [&](uint32_t ps, int t, int h, T u) {
    const T* cs = s_cs + (t * 2 + h) * (CNR * CNW);
    const T sx = (ps & 0x8000u) ? T(-1) : T(1), sy = (ps & 0x800000u) ? T(-1) : T(1);
    return prolong_add(u, cs[ps & 0x7fu], cs[(ps >> 8) & 0x7fu], cs[(ps >> 16) & 0x7fu],
                       cs[ps >> 24], T(3) * sx, T(3) * sy, sx * sy);
  };

  // wave-uniform row bases
  const char* rA = reinterpret_cast<const char*>(a.a + (int64_t)jc * jstride);
  const char* rAn = reinterpret_cast<const char*>(a.a + (int64_t)jn * jstride);
  const char* rAs = reinterpret_cast<const char*>(a.a + (int64_t)js * jstride);
  const char* rB = reinterpret_cast<const char*>(a.b + (int64_t)jc * jstride);
  char* rW = reinterpret_cast<char*>(a.rw + (int64_t)jc * jstride);
  char* rO0 = reinterpret_cast<char*>(a.o0 + (int64_t)jc * jstride);
  char* rO1 = reinterpret_cast<char*>(a.o1 + (int64_t)jc * jstride);
  const char* rF0 = nullptr;
  const char* rF1 = nullptr;
  uint32_t fkbytes = 0;
  if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
    const int64_t fjs = (int64_t)a.F.nz * a.F.ldx;
    rF0 = reinterpret_cast<const char*>(a.a + (int64_t)(2 * jc) * fjs);
    rF1 = reinterpret_cast<const char*>(a.a + (int64_t)(2 * jc + 1) * fjs);
    fkbytes = (uint32_t)a.F.ldx * ES;
  }

  const T wmu = (T(1) - a.rho) / a.rho;  // smoothers: weight of M u
  T alpha = T(0);
  if constexpr (MODE == LINE_CG) alpha = a.init ? T(0) : (T)a.st->alpha;
  double acc_rr = 0.0, acc_rz = 0.0;

  // Row indices advance as running per-lane counters; the empty asm makes each
  // step's value opaque so the compiler does not precompute (and keep alive)
  // the rows and addresses of the whole unrolled sweep.
  auto next_row = [&](int& kk) {
    asm volatile("" : "+v"(kk));
    const int k = kk;
    kk += dir;
    return k;
  };
  auto kcl = [&](int k) { return (uint32_t)min(k, nz - 1); };
  auto off = [&](int k, int col) { return (uint32_t)col * ES + kcl(k) * kbytes; };
  using SI = std::conditional_t<
      W2, std::conditional_t<PRO, StepNbP2<T>, StepNb2<T>>,
      std::conditional_t<NBL, std::conditional_t<PRO, StepNbP<T>, StepNb<T>>,
                                StepIn<T, MODE>>>;
  // EX: running byte offsets of the next row each stream loads, and their
  // per-step increments (the halo and coarse values may walk their layers in
  // the other half's direction)
  const int32_t dkb = dir * (int32_t)kbytes;
  const uint32_t xo0 = (uint32_t)ic * ES + (uint32_t)k0 * kbytes;
  uint32_t xo = xo0, xe = 0, xc = 0, xf = 0, xw = 0;
  int32_t dex = 0, dcv = 0, dfk = 0;
  [[maybe_unused]] const int32_t dE = (ie - ic) * (int32_t)ES, dW = (iw - ic) * (int32_t)ES;
  if constexpr (EX) {
    if constexpr (NBL) {
      const bool same = exh == half;
      xe = (uint32_t)(same ? k0 : NR - 1 - k0) * kbytes;
      xw = (uint32_t)k0 * kbytes;
      dex = same ? dkb : -dkb;
    }
    if constexpr (PRO) {
      const bool same = chh == half;
      xc = (uint32_t)(same ? k0 : NR - 1 - k0) * ckb;
      dcv = (same ? dir : -dir) * (int32_t)ckb;
    }
    if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
      xf = (uint32_t)(2 * ic) * ES + (uint32_t)k0 * fkbytes;
      dfk = dir * (int32_t)fkbytes;
    }
  }
  // advance a running offset; opaque to the scheduler, like the row
  // counters, so that the unrolled sweep keeps one live offset per stream
  auto adv = [](uint32_t& o, int32_t d) {
    o += (uint32_t)d;
    asm volatile("" : "+v"(o));
  };
  auto load_step_ex = [&](SI& v) {
    if constexpr (NBL) {
      v.un = ldo<T>(rA, xo + (uint32_t)dkb);
      v.f = ldn<T>(rB, xo);
      v.ex = ldo<T>(exbase, xe);
      adv(xe, dex);
      if constexpr (W2) {
        v.ew = ldo<T>(ewbase, xw);
        adv(xw, dkb);
      }
      if constexpr (PRO) {
        v.cv = ldo<T>(cbase, xc);
        adv(xc, dcv);
      }
    } else if constexpr (MODE == LINE_SOLVE) {
      v.r = ldn<T>(rA, xo);
    } else if constexpr (kSmooth) {
      v.un = ldo<T>(rA, xo + (uint32_t)dkb);
      v.ue = ldo<T>(rA, xo + (uint32_t)dE);
      v.uw = ldo<T>(rA, xo + (uint32_t)dW);
      v.unn = ldo<T>(rAn, xo);
      v.us = ldo<T>(rAs, xo);
      v.f = ldn<T>(rB, xo);
    } else if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
      v.lo = ldn2<V2>(rF0, xf);
      v.hi = ldn2<V2>(rF1, xf);
      adv(xf, dfk);
    } else {
      v.r = ldn<T>(rW, xo);
      v.q = ldn<T>(rA, xo);
    }
    adv(xo, dkb);
  };
  auto load_step = [&](int k, SI& v) {
    const uint32_t o = off(k, ic);
    if constexpr (NBL) {
      v.un = ldo<T>(rA, (uint32_t)ic * ES + (uint32_t)min(max(k + dir, 0), nz - 1) * kbytes);
      v.f = ldn<T>(rB, o);
      // the halo value at this step's layer of half exh
      v.ex = ldo<T>(exbase, kcl(exh == half ? k : NR - 1 - k) * kbytes);
      if constexpr (PRO) v.cv = ldo<T>(cbase, kcl(chh == half ? k : NR - 1 - k) * ckb);
    } else if constexpr (MODE == LINE_SOLVE) {
      v.r = ldn<T>(rA, o);
    } else if constexpr (kSmooth) {
      v.un = ldo<T>(rA, (uint32_t)ic * ES + (uint32_t)min(max(k + dir, 0), nz - 1) * kbytes);
      v.ue = ldo<T>(rA, off(k, ie));
      v.uw = ldo<T>(rA, off(k, iw));
      v.unn = ldo<T>(rAn, o);
      v.us = ldo<T>(rAs, o);
      v.f = ldn<T>(rB, o);
    } else if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
      const uint32_t fo = (uint32_t)(2 * ic) * ES + kcl(k) * fkbytes;
      v.lo = ldn2<V2>(rF0, fo);
      v.hi = ldn2<V2>(rF1, fo);
    } else {
      v.r = ldn<T>(rW, o);
      v.q = ldn<T>(rA, o);
    }
  };

  T dp[HALF];
  T ckpt[NG];
  T cprev = T(0), dprev = T(0);
  T uprv = T(0), ucur = T(0);
  if constexpr (kSmooth) ucur = ldo<T>(rA, EX ? xo0 : off(k0, ic));

  SI buf[2][CH];
  int pfo = 0;                // offset of the next step's profiles in the half's table
  T cnext[2] = {T(0), T(0)};  // PRO: coarse value of the next chunk's first step
  int kl = k0, kf = k0;  // next row to load, next row to eliminate
  auto load_cnext = [&](T& cv) {
    if constexpr (PRO) {
      if constexpr (EX)
        cv = ldo<T>(cbase, xc);
      else
        cv = ldo<T>(cbase, kcl(chh == half ? kl : NR - 1 - kl) * ckb);
    }
  };
  auto load_next = [&](SI& v) {
    if constexpr (EX)
      load_step_ex(v);
    else
      load_step(next_row(kl), v);
  };
#pragma unroll
  for (int t = 0; t < CH; ++t) load_next(buf[0][t]);
  load_cnext(cnext[0]);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    if constexpr (PRO) {
      // coarse stage: its previous contents were last read before the
      // previous chunk's fine-stage barrier
#pragma unroll
      for (int t = 0; t < CH; ++t)
        s_cs[creal ? cslot + t * CNS : cslot] = buf[ch & 1][t].cv;
      s_cs[creal ? cslot + CH * CNS : cslot] = cnext[ch & 1];
      __syncthreads();
      if (ch == 0) ucur = corr(po, 0, half, ucur);
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        buf[ch & 1][t].un = corr(po, t + 1, half, buf[ch & 1][t].un);
        buf[ch & 1][t].ex = corr(pe, t, exh, buf[ch & 1][t].ex);
        if constexpr (W2) buf[ch & 1][t].ew = corr(pw2, t, half, buf[ch & 1][t].ew);
      }
    }
    if constexpr (NBL) {
      // stage this chunk's rows: LDS buffer ch&1 was last read two chunks
      // ago, before the barrier of the previous chunk
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const T ctr = t == 0 ? ucur : buf[ch & 1][t - 1].un;
        s_nb[nbi(ch & 1, t, half, rt + 1, xl + 1)] = ctr;
        const int step_off = ((ch & 1) * CH + t) * NBSTEP;
        s_nb[exreal ? exslot + step_off : exslot] = buf[ch & 1][t].ex;
        if constexpr (W2) s_nb[lane < 2 ? ewslot + step_off : ewslot] = buf[ch & 1][t].ew;
      }
      __syncthreads();
    }
    if (ch + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) load_next(buf[(ch + 1) & 1][t]);
      load_cnext(cnext[(ch + 1) & 1]);
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int s = ch * CH + t;
      const SI& v = buf[ch & 1][t];
      bool real = true;
      if constexpr (!EX) real = next_row(kf) < nz;
      // the step's profiles through an offset that the scheduler cannot see
      // ahead of the step (otherwise it hoists the reads of the whole
      // unrolled sweep and runs out of registers)
      const T* ps = s_ps + half * PSH + pfo;
      pfo += 4;
      asm volatile("" : "+v"(pfo));
      const T cpv = ps[0];  // coupling to the previously eliminated row
      const T cnx = ps[1];  // coupling to the next row in this lane's order
      const T dzk = ps[3];
      const T diag = fma(dzk, c.S, ps[2]);
      T rhs;
      if constexpr (MODE == LINE_SOLVE) {
        rhs = real ? v.r : T(0);
      } else if constexpr (kSmooth) {
        // With M u the column's own block and g = f + dz K_h-sum of the
        // neighbours, r = f - A u = g - M u and u' = u + rho M^-1 r solves
        // M (u'/rho) = g + ((1 - rho)/rho) M u: the new iterate comes out of
        // the elimination directly and u is not read again.
        T ue, uw, unn, us;
        if constexpr (NBL) {
          ue = s_nb[nbi(ch & 1, t, half, rt + 1, xl + 2)];
          uw = s_nb[nbi(ch & 1, t, half, rt + 1, xl)];
          unn = s_nb[nbi(ch & 1, t, half, rt + 2, xl + 1)];
          us = s_nb[nbi(ch & 1, t, half, rt, xl + 1)];
        } else {
          ue = v.ue;
          uw = v.uw;
          unn = v.unn;
          us = v.us;
        }
        const T h = fma(c.cs, us, fma(c.cn, unn, fma(c.cw, uw, c.ce * ue)));
        const T mu = fma(cnx, v.un, fma(cpv, uprv, diag * ucur));
        const T g = fma(dzk, h, v.f);
        rhs = real ? fma(wmu, mu, g) : T(0);
        if constexpr (MODE == LINE_SMOOTH_NORM) {
          // EX: every row is real; an inactive lane's sum is dropped at the end
          const double r = (EX || (active && real)) ? (double)(g - mu) : 0.0;
          // pin the running sum to a register at each step: otherwise the
          // scheduler stretches the sum's dependence chain across the sweep
          // and the kernel needs twice the registers (one wave per SIMD)
          asm volatile("" : "+v"(acc_rr));
          acc_rr = fma(r, r, acc_rr);
          asm volatile("" : "+v"(acc_rr));
        }
        uprv = ucur;
        ucur = v.un;
      } else if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
        rhs = real ? v.lo.x + v.lo.y + v.hi.x + v.hi.y : T(0);
      } else {  // LINE_CG
        rhs = real ? fma(-alpha, v.q, v.r) : T(0);
      }
      T piv, inv, cn;
      elim_step(diag, cpv, cnx, cprev, piv, inv, cn);
      dprev = fma(-cpv, dprev, rhs) * inv;
      cprev = cn;
      dp[s] = dprev;
      if (s % G == G - 1) ckpt[s / G] = cprev;
    }
    // keep the scheduler from hoisting later chunks' loads and LDS reads
    // above this point (that would need registers for the whole sweep)
    __builtin_amdgcn_sched_barrier(0);
  }

  // interface between the two halves: lane's last row x_a = d_a - c_a x_b,
  // partner's last row x_b = d_b - c_b x_a
  T cq, dq;
  if constexpr (W2) {
    // the partner half is the other wavefront of the tile row
    __shared__ T s_if[W2 ? 2 : 1][2][64][2];
    s_if[rt][half][xl][0] = cprev;
    s_if[rt][half][xl][1] = dprev;
    __syncthreads();
    cq = s_if[rt][half ^ 1][xl][0];
    dq = s_if[rt][half ^ 1][xl][1];
  } else {
    cq = __shfl_xor(cprev, 32);
    dq = __shfl_xor(dprev, 32);
  }
  T x = fma(-cprev, dq, dprev) / fma(-cprev, cq, T(1));

  // EX: byte offset of the row the back sweep stores next (it walks the
  // lane's rows from the last one back to k0)
  uint32_t bo = xo0 + (uint32_t)((HALF - 1) * dkb);
#pragma unroll
  for (int g = NG - 1; g >= 0; --g) {
    // rows of this segment: k_t = kseg + dir t
    int kseg = k0 + dir * (g * G);
    asm volatile("" : "+v"(kseg));
    // recompute c' (and the pivots) of the segment from its checkpoint
    T cseg[G], pseg[G];
    T cc = g == 0 ? T(0) : ckpt[g - 1];
    int pbo = g * G * 4;  // the segment's profiles (opaque, as in the forward sweep)
    asm volatile("" : "+v"(pbo));
    const T* pseg_p = s_ps + half * PSH + pbo;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const T* ps = pseg_p + 4 * t;
      const T diag = fma(ps[3], c.S, ps[2]);
      T inv;
      elim_step(diag, ps[0], ps[1], cc, pseg[t], inv, cseg[t]);
      cc = cseg[t];
    }
#pragma unroll
    for (int t = G - 1; t >= 0; --t) {
      const int s = g * G + t;
      if (s < HALF - 1) x = fma(-cseg[t], x, dp[s]);
      const int k = kseg + dir * t;
      const bool st = active && (EX || k < nz);
      // modes that need the right-hand side again rebuild it from the
      // elimination: rhs_k = d'_k piv_k + (coupling to the previous row) d'_{k-1}
      // (accurate to a few units of roundoff of the column's largest entry)
      T rk = T(0);
      if constexpr (MODE == LINE_CG || MODE == LINE_RESTRICT_SMOOTH) {
        const T cpv = pseg_p[4 * t];
        rk = s > 0 ? fma(cpv, dp[s > 0 ? s - 1 : 0], dp[s] * pseg[t]) : dp[s] * pseg[t];
      }
      if constexpr (MODE == LINE_CG) {
        // pin both running sums to registers at each step (as in the
        // norm-computing smoother's forward sweep); EX: every row is real,
        // and an inactive lane's sums are dropped at the end
        asm volatile("" : "+v"(acc_rr), "+v"(acc_rz));
        acc_rr += (EX || st) ? (double)rk * (double)rk : 0.0;
        acc_rz += (EX || st) ? (double)rk * (double)x : 0.0;
        asm volatile("" : "+v"(acc_rr), "+v"(acc_rz));
      }
      if (st) {
        const uint32_t o = EX ? bo : off(k, ic);
        if constexpr (MODE == LINE_SOLVE) {
          sto<T>(rO0, o, a.rho * x);
        } else if constexpr (MODE == LINE_RESTRICT_SMOOTH) {
          sto<T>(rO1, o, rk);
          sto<T>(rO0, o, a.rho * x);
        } else if constexpr (kSmooth) {
          sto<T>(rO0, o, a.rho * x);
        } else {
          sto<T>(rW, o, rk);
          sto<T>(rO0, o, x);
        }
      }
      if constexpr (EX) adv(bo, -dkb);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (EX) {
    if (!active) acc_rr = acc_rz = 0.0;
  }
  if constexpr (MODE == LINE_CG) {
    double v[2] = {acc_rr, acc_rz};
    block_partials<2>(v, a.partials);
  }
  if constexpr (MODE == LINE_SMOOTH_NORM) {
    double v[1] = {acc_rr};
    block_partials<1>(v, a.partials);
  }
}

// Occupancy floor of the line kernels: three wavefronts per SIMD in FP32 (at
// most 168 registers), two in FP64 and in the two-wavefront form (at most
// 256): the register allocator keeps the kernels there, where its own choice
// would cross the line by a few registers and lose a wavefront.
template <typename T, int HALF, int MODE, bool NB = false, bool EX = false, bool W2 = false>
__global__ __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !W2 ? 3 : 2))) void k_line(Lvl<T> L, LineArgs<T> a,
                                                                         int nti, int ntj,
                                                                         int group) {
  if (gated(L)) return;
  if constexpr (MODE == LINE_CG) {
    if (a.st->done) return;  // uniform: the solve has already stopped
  }
  line_body<T, HALF, MODE, NB, EX, W2>(L, a, nti, ntj, group,
                                       xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Line solve and smoother by parallel cyclic reduction, one wavefront per
// column, for levels with too few columns to fill the GPU (horizontal-only
// coarsening keeps n_z on every level, so the coarse levels have long columns
// but few of them).  Lane l holds rows 2l and 2l+1 of the column, padded to
// 128 rows with identity rows; each reduction step at distance d eliminates
// the couplings to rows i -+ d with the equations of those rows, so after
// seven steps (d = 1, 2, ..., 64) every equation stands alone and x = y / b.
// All loads of a lane are issued at once: one memory round trip instead of
// the 2 x 64 dependent steps of the twisted elimination.  The arithmetic is
// Gaussian elimination in the cyclic-reduction order, stable for these
// diagonally dominant columns.
// ---------------------------------------------------------------------------
template <typename T>
struct PcrRow {
  T a, b, c, y;
};

template <typename T>
__device__ __forceinline__ PcrRow<T> pcr_fetch(const PcrRow<T>& r, int src, bool valid) {
  PcrRow<T> o;
  o.a = __shfl(r.a, src);
  o.b = __shfl(r.b, src);
  o.c = __shfl(r.c, src);
  o.y = __shfl(r.y, src);
  if (!valid) o = PcrRow<T>{T(0), T(1), T(0), T(0)};
  return o;
}

template <typename T>
__device__ __forceinline__ PcrRow<T> pcr_step(const PcrRow<T>& r, const PcrRow<T>& m,
                                             const PcrRow<T>& p) {
  const T k1 = r.a * rcp_nr(m.b), k2 = r.c * rcp_nr(p.b);
  PcrRow<T> o;
  o.a = -k1 * m.a;
  o.c = -k2 * p.c;
  o.b = r.b - k1 * m.c - k2 * p.a;
  o.y = r.y - k1 * m.y - k2 * p.y;
  return o;
}

template <typename T, int MODE>  // LINE_SOLVE or LINE_SMOOTH
__global__ __launch_bounds__(NTHREADS) void k_line_pcr(Lvl<T> L, LineArgs<T> a, int ncols) {
  if (gated(L)) return;
  constexpr int NR = 128;
  __shared__ T s_sub[NR], s_sup[NR], s_dg[NR], s_dz[NR];
  const int nz = L.nz;
  for (int k = threadIdx.x; k < NR; k += blockDim.x) {
    const bool real = k < nz;
    s_sub[k] = real ? L.sub[k] : T(0);
    s_sup[k] = real ? L.sup[k] : T(0);
    s_dg[k] = real ? L.dg[k] : T(1);
    s_dz[k] = real ? L.dz[k] : T(0);
  }
  __syncthreads();
  const int col = blockIdx.x * (NTHREADS / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (col >= ncols) return;  // wave-uniform; no barrier follows
  const int i = col % L.nx, j = col / L.nx;
  const int lane = threadIdx.x & 63;
  const Col<T> c = load_col(L, i, j);
  const int64_t ldx = L.ldx;
  const T wmu = (T(1) - a.rho) / a.rho;  // smoother: weight of M u
  PcrRow<T> row[2];
  int kr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = 2 * lane + h;
    kr[h] = k;
    const bool real = k < nz;
    const int kc = min(k, nz - 1);
    const int64_t o = c.base + (int64_t)kc * ldx;
    PcrRow<T>& r = row[h];
    r.a = s_sub[k];
    r.c = s_sup[k];
    r.b = s_dg[k] + s_dz[k] * c.S;
    if constexpr (MODE == LINE_SOLVE) {
      r.y = real ? __builtin_nontemporal_load(a.a + o) : T(0);
    } else {
      const T* u = a.a;
      const T um = kc > 0 ? u[o - ldx] : T(0);
      const T up = kc + 1 < nz ? u[o + ldx] : T(0);
      const T uc = u[o];
      const T h4 = c.ce * u[o + c.oe] + c.cw * u[o + c.ow] + c.cn * u[o + c.on] +
                   c.cs * u[o + c.os];
      const T mu = r.b * uc + r.a * um + r.c * up;
      const T g = __builtin_nontemporal_load(a.b + o) + s_dz[k] * h4;
      r.y = real ? g + wmu * mu : T(0);
    }
    if (!real) r = PcrRow<T>{T(0), T(1), T(0), T(0)};
  }
  // d = 1: row 2l couples to 2l-1 (lane l-1, second row) and 2l+1 (own
  // second row); row 2l+1 to 2l (own first row) and 2l+2 (lane l+1, first row)
  {
    const PcrRow<T> m0 = pcr_fetch(row[1], lane - 1 < 0 ? 0 : lane - 1, lane > 0);
    const PcrRow<T> p1 = pcr_fetch(row[0], lane + 1 > 63 ? 63 : lane + 1, lane < 63);
    const PcrRow<T> r0 = pcr_step(row[0], m0, row[1]);
    const PcrRow<T> r1 = pcr_step(row[1], row[0], p1);
    row[0] = r0;
    row[1] = r1;
  }
  // d = 2e: rows 2l -+ 2e live in lanes l -+ e, same slot
#pragma unroll
  for (int e = 1; e < 64; e <<= 1) {
    const int lm = lane - e, lp = lane + e;
    const bool vm = lm >= 0, vp = lp < 64;
    const int sm = vm ? lm : lane, sp = vp ? lp : lane;
    PcrRow<T> nw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const PcrRow<T> m = pcr_fetch(row[h], sm, vm);
      const PcrRow<T> p = pcr_fetch(row[h], sp, vp);
      nw[h] = pcr_step(row[h], m, p);
    }
    row[0] = nw[0];
    row[1] = nw[1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (kr[h] < nz) {
      const T x = row[h].y / row[h].b;
      __builtin_nontemporal_store(a.rho * x, a.o0 + c.base + (int64_t)kr[h] * ldx);
    }
  }
}

// ---------------------------------------------------------------------------
// Residual fused with the restriction: f_c(I,J,k) = sum over the four fine
// children (2I+a, 2J+b) of (f - A u).  One thread per coarse column; the fine
// residual itself is never stored.  A wavefront covers 64 coarse = 128 fine
// columns and reads each fine row pair with 16-byte vector loads.
// ---------------------------------------------------------------------------
template <typename T, bool FULL, bool X>
struct ResRestrictPol {
  using V2 = typename Vec2<T>::type;
  // X (all 64 lanes hold coarse columns): the fine columns west of a / c and
  // east of b / d are the neighbouring lanes' b / d and a / c values of the
  // same layer, passed by wave shifts; uWa and uWc then hold the halo value
  // of the row (lane 0: west, lane 63: east, other lanes their own a / c)
  struct In {
    V2 p0, p1, sS, sN, f0, f1;
    T uWa, uEb, uWc, uEd;
  };
  const char *ra, *rc, *rS, *rN, *fa, *fb;
  char* ro;
  uint32_t o2, ow, oe, oo, fkb, ckb, oh;
  bool lw, le;
  int nz, k0;
  // face couplings of the 2x2 block: a = (i0,j0), b = (i0+1,j0),
  // c = (i0,j0+1), d = (i0+1,j0+1)
  T xab, xbE, xWa, xcd, xdE, xWc, yac, ybd, ycN, ydN, ySa, ySb, Sa, Sb, Sc, Sd;
  const Prof<T>* sp;
  V2 m0, m1, c0, c1;

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = k0 + s;
    const uint32_t ok = layer_off<FULL>(k, nz, fkb);
    const uint32_t okp = (uint32_t)min(k + 1, nz - 1) * fkb;
    v.p0 = ldo<V2>(ra, o2 + okp);
    v.p1 = ldo<V2>(rc, o2 + okp);
    if constexpr (X) {
      v.uWa = ldo<T>(ra, oh + ok);
      v.uWc = ldo<T>(rc, oh + ok);
    } else {
      v.uWa = ldo<T>(ra, ow + ok);
      v.uEb = ldo<T>(ra, oe + ok);
      v.uWc = ldo<T>(rc, ow + ok);
      v.uEd = ldo<T>(rc, oe + ok);
    }
    v.sS = ldo<V2>(rS, o2 + ok);
    v.sN = ldo<V2>(rN, o2 + ok);
    v.f0 = ldn2<V2>(fa, o2 + ok);
    v.f1 = ldn2<V2>(fb, o2 + ok);
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const int k = k0 + s;
    const Prof<T> pr = sp[s];
    const bool top = k + 1 < nz;
    const V2 p0 = top ? v.p0 : V2{T(0), T(0)};
    const V2 p1 = top ? v.p1 : V2{T(0), T(0)};
    const T dzk = pr.dz, dgk = pr.dg, sub = pr.sub, sup = pr.sup;
    T uWa = v.uWa, uEb = v.uEb, uWc = v.uWc, uEd = v.uEd;
    if constexpr (X) {
      const T wa = wave_shift<kWaveShr1>(c0.y), eb = wave_shift<kWaveShl1>(c0.x);
      const T wc = wave_shift<kWaveShr1>(c1.y), ed = wave_shift<kWaveShl1>(c1.x);
      uWa = lw ? v.uWa : wa;
      uEb = le ? v.uWa : eb;
      uWc = lw ? v.uWc : wc;
      uEd = le ? v.uWc : ed;
    }
    // f - A u of one child, with every multiply-add spelled out, so that each
    // instantiation (segment length, tile form, grouped launches) rounds the
    // same way: (dg + dz S) u - dz (sum of the four coupled neighbours)
    //   + sub u_below + sup u_above
    auto res = [&](T f, T S, T uc, T c1_, T n1, T c2_, T n2, T c3_, T n3, T c4_, T n4, T um,
                   T up) {
      T h = c1_ * n1;
      h = fma(c2_, n2, h);
      h = fma(c3_, n3, h);
      h = fma(c4_, n4, h);
      T a = fma(dzk, S, dgk) * uc;
      a = fma(-dzk, h, a);
      a = fma(sub, um, a);
      a = fma(sup, up, a);
      return f - a;
    };
    const T ra_ = res(v.f0.x, Sa, c0.x, xab, c0.y, xWa, uWa, yac, c1.x, ySa, v.sS.x, m0.x, p0.x);
    const T rb_ = res(v.f0.y, Sb, c0.y, xbE, uEb, xab, c0.x, ybd, c1.y, ySb, v.sS.y, m0.y, p0.y);
    const T rc_ = res(v.f1.x, Sc, c1.x, xcd, c1.y, xWc, uWc, ycN, v.sN.x, yac, c0.x, m1.x, p1.x);
    const T rd_ = res(v.f1.y, Sd, c1.y, xdE, uEd, xcd, c1.x, ydN, v.sN.y, ybd, c0.y, m1.y, p1.y);
    sto<T>(ro, oo + layer_off<FULL>(k, nz, ckb), ra_ + rb_ + rc_ + rd_);
    m0 = c0;
    m1 = c1;
    c0 = p0;
    c1 = p1;
  }
};

// Residual of the fine level fused with the restriction (Algorithm 1: the
// residual is only needed restricted): f_c(I,J) = sum over the 2x2 children of
// (f - A u).  One lane per coarse column; its four children are read as two
// 2-vectors per layer.  The fine residual itself is never stored.
// CH: layers loaded ahead; the single-instance kernels take 2 (FP64) and 4
// (FP32), measured 484 -> 477 and 241 -> 238 us at 1024^2 x 128 against 1
// and 2, which the grouped batched kernel keeps
template <typename T, int SR, int KS = KSEG, int CH = (sizeof(T) == 8 ? 1 : 2)>
__device__ __forceinline__ void resrestrict_body(const Lvl<T>& F, const Lvl<T>& C,
                                                 const T* __restrict__ u,
                                                 const T* __restrict__ f, T* __restrict__ fc,
                                                 int nti, int ntj, int group, int b) {
  const Geo g = stencil_geo<SR, KS>(C.nx, C.ny, C.nz, nti, ntj, group, b);
  __shared__ Prof<T> sp[KS];
  stage_prof<T, KS>(F, g.k0, sp);
  if (!(g.row && g.act)) return;
  const int nx = F.nx, ny = F.ny, nz = F.nz;
  const int I = g.ic, J = g.j;
  const int i0 = 2 * I, j0 = 2 * J;
  const int iw = (i0 == 0) ? nx - 1 : i0 - 1;
  const int ie = (i0 + 2 == nx) ? 0 : i0 + 2;
  const int js = (j0 == 0) ? ny - 1 : j0 - 1;
  const int jn = (j0 + 2 == ny) ? 0 : j0 + 2;
  const int64_t jst = (int64_t)nz * F.ldx;
  const uint32_t ES = sizeof(T);
  auto run = [&](auto full, auto xch) {
    constexpr bool FL = decltype(full)::value, XC = decltype(xch)::value;
    ResRestrictPol<T, FL, XC> P;
    const int64_t r0 = (int64_t)j0 * nx, r1c = (int64_t)(j0 + 1) * nx, rs = (int64_t)js * nx;
    P.xab = F.cx[r0 + i0];
    P.xbE = F.cx[r0 + i0 + 1];
    P.xWa = F.cx[r0 + iw];
    P.xcd = F.cx[r1c + i0];
    P.xdE = F.cx[r1c + i0 + 1];
    P.xWc = F.cx[r1c + iw];
    P.yac = F.cy[r0 + i0];
    P.ybd = F.cy[r0 + i0 + 1];
    P.ycN = F.cy[r1c + i0];
    P.ydN = F.cy[r1c + i0 + 1];
    P.ySa = F.cy[rs + i0];
    P.ySb = F.cy[rs + i0 + 1];
    P.Sa = P.xab + P.xWa + P.yac + P.ySa + F.wall[r0 + i0];
    P.Sb = P.xbE + P.xab + P.ybd + P.ySb + F.wall[r0 + i0 + 1];
    P.Sc = P.xcd + P.xWc + P.ycN + P.yac + F.wall[r1c + i0];
    P.Sd = P.xdE + P.xcd + P.ydN + P.ybd + F.wall[r1c + i0 + 1];
    P.ra = rowc(u, j0, jst);
    P.rc = rowc(u, j0 + 1, jst);
    P.rS = rowc(u, js, jst);
    P.rN = rowc(u, jn, jst);
    P.fa = rowc(f, j0, jst);
    P.fb = rowc(f, j0 + 1, jst);
    P.ro = roww(fc, J, (int64_t)C.nz * C.ldx);
    P.o2 = (uint32_t)i0 * ES;
    P.ow = (uint32_t)iw * ES;
    P.oe = (uint32_t)ie * ES;
    if constexpr (XC) {
      const int lane = (int)(threadIdx.x & 63);
      P.lw = lane == 0;
      P.le = lane == 63;
      P.oh = P.lw ? P.ow : P.le ? P.oe : P.o2;
    }
    P.oo = (uint32_t)I * ES;
    P.fkb = (uint32_t)F.ldx * ES;
    P.ckb = (uint32_t)C.ldx * ES;
    P.nz = nz;
    P.k0 = g.k0;
    P.sp = sp;
    using V2 = typename Vec2<T>::type;
    P.m0 = V2{T(0), T(0)};
    P.m1 = V2{T(0), T(0)};
    if (g.k0 > 0) {
      P.m0 = ldo<V2>(P.ra, P.o2 + (uint32_t)(g.k0 - 1) * P.fkb);
      P.m1 = ldo<V2>(P.rc, P.o2 + (uint32_t)(g.k0 - 1) * P.fkb);
    }
    P.c0 = ldo<V2>(P.ra, P.o2 + (uint32_t)g.k0 * P.fkb);
    P.c1 = ldo<V2>(P.rc, P.o2 + (uint32_t)g.k0 * P.fkb);
    walk<CH, FL, KS>(P, g.n);
  };
  if (g.ft) {
    if (g.n == KS)
      run(std::true_type{}, std::true_type{});
    else
      run(std::false_type{}, std::true_type{});
  } else {
    if (g.n == KS)
      run(std::true_type{}, std::false_type{});
    else
      run(std::false_type{}, std::false_type{});
  }
}

template <typename T, int SR, int KS>
__global__ __launch_bounds__(64 * SR) void k_resrestrict(Lvl<T> F, Lvl<T> C,
                                                         const T* __restrict__ u,
                                                         const T* __restrict__ f,
                                                         T* __restrict__ fc, int nti, int ntj,
                                                         int group) {
  if (gated(F)) return;
  resrestrict_body<T, SR, KS, (sizeof(T) == 8 ? 2 : 4)>(F, C, u, f, fc, nti, ntj, group,
                                                       xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Refinement step fused with the next residual: u' = u + e (e FP32),
// r = f - A u', r32 = (float) r, partial ||r||^2.  u' goes to a different
// buffer (neighbouring threads still read u and e).
// ---------------------------------------------------------------------------
// X (all 64 columns of the tile exist): the east and west values of u + e at
// layer k are the neighbouring lanes' own, passed by wave shifts; ue / ee
// then hold the halo column's u and e (lane 0: west, lane 63: east, other
// lanes their own column).
template <bool FULL, bool X>
struct CorrectPol {
  struct In {
    double up, ue, uw, un, us, f;
    float ep, ee, ew, en, es;
  };
  const char *ru, *run, *rus, *re, *ren, *res, *rf;
  char *ruo, *rr32;
  uint32_t oc8, oe8, ow8, oc4, oe4, ow4, kb8, kb4, oh8, oh4;
  bool lw, le;
  int nz, k0;
  Cf<double> c;
  const Prof<double>* sp;
  double xm, xc, nrm;

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = k0 + s;
    const int kc = FULL ? k : min(k, nz - 1);
    const int kp = min(k + 1, nz - 1);
    const uint32_t o8 = (uint32_t)kc * kb8, o4 = (uint32_t)kc * kb4;
    v.up = ldo<double>(ru, oc8 + (uint32_t)kp * kb8);
    v.ep = ldo<float>(re, oc4 + (uint32_t)kp * kb4);
    if constexpr (X) {
      v.ue = ldo<double>(ru, oh8 + o8);
      v.ee = ldo<float>(re, oh4 + o4);
    } else {
      v.ue = ldo<double>(ru, oe8 + o8);
      v.ee = ldo<float>(re, oe4 + o4);
      v.uw = ldo<double>(ru, ow8 + o8);
      v.ew = ldo<float>(re, ow4 + o4);
    }
    v.un = ldo<double>(run, oc8 + o8);
    v.en = ldo<float>(ren, oc4 + o4);
    v.us = ldo<double>(rus, oc8 + o8);
    v.es = ldo<float>(res, oc4 + o4);
    v.f = ldn<double>(rf, oc8 + o8);
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const int k = k0 + s;
    const Prof<double> pr = sp[s];
    const double xp = (k + 1 < nz) ? v.up + (double)v.ep : 0.0;
    double xe, xw;
    if constexpr (X) {
      const double xh = v.ue + (double)v.ee;
      const double de = wave_shift<kWaveShl1>(xc), dw = wave_shift<kWaveShr1>(xc);
      xe = le ? xh : de;
      xw = lw ? xh : dw;
    } else {
      xe = v.ue + (double)v.ee;
      xw = v.uw + (double)v.ew;
    }
    const double h = c.ce * xe + c.cw * xw + c.cn * (v.un + (double)v.en) +
                     c.cs * (v.us + (double)v.es);
    const double au = (pr.dg + pr.dz * c.S) * xc - pr.dz * h + pr.sub * xm + pr.sup * xp;
    const double rr = v.f - au;
    const int kc = FULL ? k : min(k, nz - 1);
    sto<double>(ruo, oc8 + (uint32_t)kc * kb8, xc);
    sto<float>(rr32, oc4 + (uint32_t)kc * kb4, (float)rr);
    nrm += rr * rr;
    xm = xc;
    xc = xp;
  }
};

// CH: layers of each field loaded ahead (4 for the single-instance kernel,
// measured 880 -> 868 us at 1024^2 x 128 at two waves per SIMD; 2 keeps the
// grouped batched kernel at three)
template <int SR, int CH = 2>
__device__ __forceinline__ void correct_residual_body(
    const Lvl<double>& L, const double* __restrict__ u, const float* __restrict__ e,
    const double* __restrict__ f, double* __restrict__ uout, float* __restrict__ r32,
    double* __restrict__ partials, int nti, int ntj, int group, int b) {
  const Geo g = stencil_geo<SR>(L.nx, L.ny, L.nz, nti, ntj, group, b);
  __shared__ Prof<double> sp[KSEG];
  stage_prof(L, g.k0, sp);
  double nrm[1] = {0.0};
  if (g.row && g.act) {
    const int64_t jst = (int64_t)L.nz * L.ldx;
    auto run = [&](auto full, auto xch) {
      constexpr bool FL = decltype(full)::value, XC = decltype(xch)::value;
      CorrectPol<FL, XC> P;
      P.ru = rowc(u, g.j, jst);
      P.run = rowc(u, g.jn, jst);
      P.rus = rowc(u, g.js, jst);
      P.re = rowc(e, g.j, jst);
      P.ren = rowc(e, g.jn, jst);
      P.res = rowc(e, g.js, jst);
      P.rf = rowc(f, g.j, jst);
      P.ruo = roww(uout, g.j, jst);
      P.rr32 = roww(r32, g.j, jst);
      P.oc8 = (uint32_t)g.ic * 8;
      P.oe8 = (uint32_t)g.ie * 8;
      P.ow8 = (uint32_t)g.iw * 8;
      P.oc4 = (uint32_t)g.ic * 4;
      P.oe4 = (uint32_t)g.ie * 4;
      P.ow4 = (uint32_t)g.iw * 4;
      P.kb8 = (uint32_t)L.ldx * 8;
      P.kb4 = (uint32_t)L.ldx * 4;
      if constexpr (XC) {
        const int lane = (int)(threadIdx.x & 63);
        P.lw = lane == 0;
        P.le = lane == 63;
        const int ih = P.lw ? g.iw : P.le ? g.ie : g.ic;
        P.oh8 = (uint32_t)ih * 8;
        P.oh4 = (uint32_t)ih * 4;
      }
      P.nz = L.nz;
      P.k0 = g.k0;
      P.c = col_coef(L, g);
      P.sp = sp;
      P.nrm = 0.0;
      P.xm = g.k0 > 0 ? ldo<double>(P.ru, P.oc8 + (uint32_t)(g.k0 - 1) * P.kb8) +
                            (double)ldo<float>(P.re, P.oc4 + (uint32_t)(g.k0 - 1) * P.kb4)
                      : 0.0;
      P.xc = ldo<double>(P.ru, P.oc8 + (uint32_t)g.k0 * P.kb8) +
             (double)ldo<float>(P.re, P.oc4 + (uint32_t)g.k0 * P.kb4);
      walk<CH, FL>(P, g.n);
      nrm[0] = P.nrm;
    };
    if (g.ft) {
      if (g.n == KSEG)
        run(std::true_type{}, std::true_type{});
      else
        run(std::false_type{}, std::true_type{});
    } else {
      if (g.n == KSEG)
        run(std::true_type{}, std::false_type{});
      else
        run(std::false_type{}, std::false_type{});
    }
  }
  block_partials<1, SR>(nrm, partials);
}

template <int SR>
__global__ __launch_bounds__(64 * SR) void k_correct_residual(
    Lvl<double> L, const double* __restrict__ u, const float* __restrict__ e,
    const double* __restrict__ f, double* __restrict__ uout, float* __restrict__ r32,
    double* __restrict__ partials, int nti, int ntj, int group) {
  if (gated(L)) return;
  correct_residual_body<SR, 4>(L, u, e, f, uout, r32, partials, nti, ntj, group,
                               xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Prolongate: uf += P uc (cell-centred bilinear, 9/3/3/1 over 16, periodic)
// ---------------------------------------------------------------------------
template <typename T, bool FULL>
struct ProlongPol {
  struct In {
    T a, b, c, d, u;
  };
  const char *rc0, *rc1;
  char* rf;
  uint32_t oI, oI2, of, ckb, fkb;
  int nz, k0;
  T wb, wc, wd;  // weights of the x, y and diagonal neighbours (3, 3, 1 inside)

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = k0 + s;
    const uint32_t okc = layer_off<FULL>(k, nz, ckb);
    v.a = ldo<T>(rc0, oI + okc);
    v.b = ldo<T>(rc0, oI2 + okc);
    v.c = ldo<T>(rc1, oI + okc);
    v.d = ldo<T>(rc1, oI2 + okc);
    v.u = ldn<T>(rf, of + layer_off<FULL>(k, nz, fkb));
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    sto<T>(rf, of + layer_off<FULL>(k0 + s, nz, fkb),
           prolong_add(v.u, v.a, v.b, v.c, v.d, wb, wc, wd));
  }
};

// One lane per fine column (i, j); its coarse parent (I, J) = (i/2, j/2) and
// the coarse neighbours on the child's side, I2 = I -+ 1, J2 = J -+ 1, weighted
// 9/3/3/1 over 16.  Periodic boundaries wrap; behind a Dirichlet wall the
// neighbour is the parent's mirror image with opposite sign (the linear
// interpolant that vanishes on the wall).
template <typename T, int SR, int KS = KSEG>
__device__ __forceinline__ void prolongate_body(const Lvl<T>& C, const Lvl<T>& F,
                                                const T* __restrict__ uc, T* __restrict__ uf,
                                                int nti, int ntj, int group, int b) {
  const Geo g = stencil_geo<SR, KS>(F.nx, F.ny, F.nz, nti, ntj, group, b);
  if (!(g.row && g.act)) return;
  const int I = g.ic >> 1, J = g.j >> 1;
  int I2 = I + ((g.ic & 1) ? 1 : -1);
  int J2 = J + ((g.j & 1) ? 1 : -1);
  T sx = T(1), sy = T(1);
  if (I2 < 0 || I2 == C.nx) {
    if (C.bch) {
      I2 = I;
      sx = T(-1);
    } else {
      I2 = (I2 < 0) ? C.nx - 1 : 0;
    }
  }
  if (J2 < 0 || J2 == C.ny) {
    if (C.bch) {
      J2 = J;
      sy = T(-1);
    } else {
      J2 = (J2 < 0) ? C.ny - 1 : 0;
    }
  }
  const uint32_t ES = sizeof(T);
  auto run = [&](auto full) {
    constexpr bool FL = decltype(full)::value;
    ProlongPol<T, FL> P;
    const int64_t cjs = (int64_t)C.nz * C.ldx;
    P.rc0 = rowc(uc, J, cjs);
    P.rc1 = rowc(uc, J2, cjs);
    P.rf = roww(uf, g.j, (int64_t)F.nz * F.ldx);
    P.oI = (uint32_t)I * ES;
    P.oI2 = (uint32_t)I2 * ES;
    P.of = (uint32_t)g.ic * ES;
    P.ckb = (uint32_t)C.ldx * ES;
    P.fkb = (uint32_t)F.ldx * ES;
    P.nz = F.nz;
    P.k0 = g.k0;
    P.wb = T(3) * sx;
    P.wc = T(3) * sy;
    P.wd = sx * sy;
    walk<4, FL, KS>(P, g.n);
  };
  if (g.n == KS)
    run(std::true_type{});
  else
    run(std::false_type{});
}

template <typename T, int SR, int KS>
__global__ __launch_bounds__(64 * SR) void k_prolongate(Lvl<T> C, Lvl<T> F,
                                                        const T* __restrict__ uc,
                                                        T* __restrict__ uf, int nti, int ntj,
                                                        int group) {
  if (gated(F)) return;
  prolongate_body<T, SR, KS>(C, F, uc, uf, nti, ntj, group, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// CG, first fused kernel ("SpMV" of Sec. 3.1):
//   p = z + beta p;  q = A z + beta q;  partial <p, q>  (+ the pending steps
//   of the iterate, u += alpha p, on every other iteration)
// ---------------------------------------------------------------------------
// PAIR (even iterations of line-PCG): the iterate also takes the two steps
// not yet applied, u += alpha_prev p_{i-2} + alpha p_{i-1}, with p_{i-2} read
// from the buffer that p_i then overwrites; odd iterations touch neither u nor
// p_{i-2} (5 words per cell instead of 7; even ones 8).
template <bool FULL, bool PAIR>
struct CgP1Pol {
  struct In {
    double xp, xe, xw, xn, xs, p, q, u, p2;
  };
  ColumnOp<double> op;  // on z
  char *ru, *rw, *rq;
  const char* rp;
  double alpha, alpha_prev, beta, pq;

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = op.k0 + s;
    const uint32_t ok = layer_off<FULL>(k, op.nz, op.kb);
    const uint32_t okp = (uint32_t)min(k + 1, op.nz - 1) * op.kb;
    op.load(ok, okp, v.xp, v.xe, v.xw, v.xn, v.xs);
    v.p = ldn<double>(rp, op.oc + ok);
    v.q = ldn<double>(rq, op.oc + ok);
    if constexpr (PAIR) {
      v.u = ldn<double>(ru, op.oc + ok);
      v.p2 = ldn<double>(rw, op.oc + ok);
    }
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const uint32_t o = op.oc + layer_off<FULL>(op.k0 + s, op.nz, op.kb);
    const double zc = op.xc;
    const double az = op.apply(s, v.xp, v.xe, v.xw, v.xn, v.xs);
    const double pn = zc + beta * v.p;
    const double qn = az + beta * v.q;
    // the two steps in the order of the iterations they belong to
    if constexpr (PAIR) sto<double>(ru, o, fma(alpha, v.p, fma(alpha_prev, v.p2, v.u)));
    sto<double>(rw, o, pn);
    sto<double>(rq, o, qn);
    pq += pn * qn;
  }
};

template <int SR, bool PAIR>
__global__ __launch_bounds__(64 * SR) void k_cg_p1(Lvl<double> L, double* __restrict__ u,
                                                   const double* __restrict__ pr,
                                                   double* __restrict__ pw,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ q,
                                                   const CgState* __restrict__ st,
                                                   double* __restrict__ partials, int nti,
                                                   int ntj, int group) {
  if (st->done || gated(L)) return;  // uniform: the solve has already stopped
  constexpr int CH = 2;
  const double alpha = st->alpha, alpha_prev = st->alpha_prev, beta = st->beta;
  const Geo g =
      stencil_geo<SR>(L.nx, L.ny, L.nz, nti, ntj, group, xcd_remap(blockIdx.x, gridDim.x));
  __shared__ Prof<double> sp[KSEG];
  stage_prof(L, g.k0, sp);
  double pq[1] = {0.0};
  if (g.row && g.act) {
    const int64_t jstride = (int64_t)L.nz * L.ldx;
    const uint32_t kb = (uint32_t)(L.ldx * sizeof(double));
    const Cf<double> cf = col_coef(L, g);
    auto run = [&](auto full) {
      constexpr bool F = decltype(full)::value;
      CgP1Pol<F, PAIR> pol;
      pol.op.init(z, g, jstride, kb, cf, sp, L.nz);
      pol.ru = PAIR ? roww(u, g.j, jstride) : nullptr;
      pol.rp = rowc(pr, g.j, jstride);
      pol.rw = roww(pw, g.j, jstride);
      pol.rq = roww(q, g.j, jstride);
      pol.alpha = alpha;
      pol.alpha_prev = alpha_prev;
      pol.beta = beta;
      pol.pq = 0.0;
      walk<CH, F>(pol, g.n);
      pq[0] = pol.pq;
    };
    if (g.n == KSEG)
      run(std::true_type{});
    else
      run(std::false_type{});
  }
  block_partials<1, SR>(pq, partials);
}

// ---------------------------------------------------------------------------
// Flexible CG with a variable (multigrid) preconditioner z = B(r)
// (Notay, "Flexible conjugate gradients", SIAM J. Sci. Comput. 22, 2000; one
// direction kept):  beta = -<z, q_old>/<p_old, q_old>,  p = z + beta p,
// q = A z + beta q  (= A p),  alpha = <p, r>/<p, q>,  u += alpha p,
// r -= alpha q.  z may be FP32 (mixed precision); everything else is FP64.
// u += alpha p is deferred to the next direction kernel, which reads p anyway
// (so the update kernel does not), and the last one to a final update.
// ---------------------------------------------------------------------------
template <typename TZ>
__global__ __launch_bounds__(NTHREADS) void k_fcg_zq(Lvl<double> L, const TZ* __restrict__ z,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ partials, int nti,
                                                     int ntj) {
  if (gated(L)) return;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int ti = b % nti;
  const int r1 = b / nti;
  const int tj = r1 % ntj;
  const int kb = r1 / ntj;
  const int i = ti * 64 + (threadIdx.x & 63);
  const int j = tj * SROWS + (threadIdx.x >> 6);
  double acc[1] = {0.0};
  if (i < L.nx && j < L.ny) {
    const int64_t base = (int64_t)j * L.nz * L.ldx + i;
    const int k0 = kb * KSEG, k1 = min(L.nz, k0 + KSEG);
    for (int k = k0; k < k1; ++k) {
      const int64_t o = base + (int64_t)k * L.ldx;
      acc[0] += (double)z[o] * q[o];
    }
  }
  block_partials<1>(acc, partials);
}

// PAIR: as in line-PCG, even iterations also apply the two pending steps of
// the iterate (u += alpha_prev p_{i-2} + alpha p_{i-1}, p_{i-2} read from the
// buffer that p_i overwrites); odd ones leave u alone.
template <typename TZ, bool FULL, bool PAIR>
struct FcgDirPol {
  struct In {
    double xp, xe, xw, xn, xs, p, q, r, u, p2;
  };
  ColumnOp<double, TZ> op;  // on z
  char *rw, *rq, *ru;
  const char *rp, *rr;
  uint32_t oc, kb;
  double beta, alpha, alpha_prev, pq, pr;

  __device__ __forceinline__ void load(int s, In& v) {
    const int k = op.k0 + s;
    op.load(layer_off<FULL>(k, op.nz, op.kb), (uint32_t)min(k + 1, op.nz - 1) * op.kb, v.xp,
            v.xe, v.xw, v.xn, v.xs);
    const uint32_t o = oc + layer_off<FULL>(k, op.nz, kb);
    v.p = ldn<double>(rp, o);
    v.q = ldn<double>(rq, o);
    v.r = ldn<double>(rr, o);
    if constexpr (PAIR) {
      v.u = ldn<double>(ru, o);
      v.p2 = ldn<double>(rw, o);
    }
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const uint32_t o = oc + layer_off<FULL>(op.k0 + s, op.nz, kb);
    const double zc = op.xc;
    const double az = op.apply(s, v.xp, v.xe, v.xw, v.xn, v.xs);
    // the two pending steps, in the order of their iterations
    if constexpr (PAIR) sto<double>(ru, o, fma(alpha, v.p, fma(alpha_prev, v.p2, v.u)));
    const double pn = zc + beta * v.p;
    const double qn = az + beta * v.q;
    sto<double>(rw, o, pn);
    sto<double>(rq, o, qn);
    pq += pn * qn;
    pr += pn * v.r;
  }
};

// The updates of the iterate, u += alpha p, are applied here in pairs, where
// the old directions are read anyway (alpha = 0 before the first step); the
// ones still pending after the loop by a final kernel.
template <typename TZ, int SR, bool PAIR>
__global__ __launch_bounds__(64 * SR) void k_fcg_dir(Lvl<double> L, const TZ* __restrict__ z,
                                                     double* __restrict__ u,
                                                     const double* __restrict__ pr,
                                                     double* __restrict__ pw,
                                                     double* __restrict__ q,
                                                     const double* __restrict__ r,
                                                     const CgState* __restrict__ st,
                                                     double* __restrict__ partials, int nti,
                                                     int ntj, int group) {
  if (st->done || gated(L)) return;
  const double beta = st->beta, alpha = st->alpha, alpha_prev = st->alpha_prev;
  const Geo g =
      stencil_geo<SR>(L.nx, L.ny, L.nz, nti, ntj, group, xcd_remap(blockIdx.x, gridDim.x));
  __shared__ Prof<double> sp[KSEG];
  stage_prof(L, g.k0, sp);
  double acc[2] = {0.0, 0.0};
  if (g.row && g.act) {
    const int64_t jst = (int64_t)L.nz * L.ldx;
    auto run = [&](auto full) {
      constexpr bool FL = decltype(full)::value;
      FcgDirPol<TZ, FL, PAIR> P;
      P.op.init(z, g, jst, (uint32_t)(L.ldx * sizeof(TZ)), col_coef(L, g), sp, L.nz);
      P.rp = rowc(pr, g.j, jst);
      P.rw = roww(pw, g.j, jst);
      P.rq = roww(q, g.j, jst);
      P.rr = rowc(r, g.j, jst);
      P.ru = PAIR ? roww(u, g.j, jst) : nullptr;
      P.oc = (uint32_t)g.ic * 8;
      P.kb = (uint32_t)L.ldx * 8;
      P.beta = beta;
      P.alpha = alpha;
      P.alpha_prev = alpha_prev;
      P.pq = 0.0;
      P.pr = 0.0;
      walk<2, FL>(P, g.n);
      acc[0] = P.pq;
      acc[1] = P.pr;
    };
    if (g.n == KSEG)
      run(std::true_type{});
    else
      run(std::false_type{});
  }
  block_partials<2, SR>(acc, partials);
}

template <bool FULL>
struct FcgUpdPol {
  struct In {
    double r, q;
  };
  char* rr;
  const char* rq;
  char* rd;  // FP32 copy of r (mixed precision) or null
  uint32_t oc, kb, oc4, kb4;
  int nz, k0;
  double alpha, rr2;

  __device__ __forceinline__ void load(int s, In& v) {
    const uint32_t o = oc + layer_off<FULL>(k0 + s, nz, kb);
    v.r = ldn<double>(rr, o);
    v.q = ldn<double>(rq, o);
  }
  __device__ __forceinline__ void step(int s, const In& v) {
    const int kc = FULL ? k0 + s : min(k0 + s, nz - 1);
    const uint32_t o = oc + (uint32_t)kc * kb;
    const double rn = v.r - alpha * v.q;
    sto<double>(rr, o, rn);
    if (rd) sto<float>(rd, oc4 + (uint32_t)kc * kb4, (float)rn);
    rr2 += rn * rn;
  }
};

// r -= alpha q (and its FP32 copy), ||r||^2; u is updated by the next
// direction kernel (or after the loop)
template <int SR>
__global__ __launch_bounds__(64 * SR) void k_fcg_update(Lvl<double> L, double* __restrict__ r,
                                                        const double* __restrict__ q,
                                                        float* __restrict__ rdown,
                                                        const CgState* __restrict__ st,
                                                        double* __restrict__ partials, int nti,
                                                        int ntj, int group) {
  // stopped (a breakdown included: r stays the last residual)
  if (st->done || gated(L)) return;
  const double alpha = st->alpha;
  const Geo g =
      stencil_geo<SR>(L.nx, L.ny, L.nz, nti, ntj, group, xcd_remap(blockIdx.x, gridDim.x));
  double acc[1] = {0.0};
  if (g.row && g.act) {
    const int64_t jst = (int64_t)L.nz * L.ldx;
    auto run = [&](auto full) {
      constexpr bool FL = decltype(full)::value;
      FcgUpdPol<FL> P;
      P.rr = roww(r, g.j, jst);
      P.rq = rowc(q, g.j, jst);
      P.rd = rdown ? roww(rdown, g.j, jst) : nullptr;
      P.oc = (uint32_t)g.ic * 8;
      P.kb = (uint32_t)L.ldx * 8;
      P.oc4 = (uint32_t)g.ic * 4;
      P.kb4 = (uint32_t)L.ldx * 4;
      P.nz = L.nz;
      P.k0 = g.k0;
      P.alpha = alpha;
      P.rr2 = 0.0;
      walk<4, FL>(P, g.n);
      acc[0] = P.rr2;
    };
    if (g.n == KSEG)
      run(std::true_type{});
    else
      run(std::false_type{});
  }
  block_partials<1, SR>(acc, partials);
}

// ---------------------------------------------------------------------------
// Grouped launches: one launch covers the work items of many (instance, rhs)
// pairs; each workgroup finds its item by binary search over the items' first
// workgroups (uniform scalar loads) and runs the single-level body.  Items of
// converged pairs return at once.
// ---------------------------------------------------------------------------
template <typename I>
__device__ __forceinline__ int find_item(const I* __restrict__ items, int nitems, int B) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].blk0 <= B) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// EX: every item of the launch has columns of exactly 2 HALF layers (the host
// checks), so the exact-height form serves them all.
template <int HALF, int MODE, bool EX>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_line_grouped(const GItem<float>* __restrict__ items,
                                                           int nitems,
                                                           const int* __restrict__ active,
                                                           float rho) {
  const int B = xcd_remap(blockIdx.x, gridDim.x);
  const GItem<float> it = items[find_item(items, nitems, B)];
  if (!active[it.pair]) return;
  LineArgs<float> a{};
  a.a = it.a;
  a.b = it.b;
  a.o0 = it.o;
  a.rho = rho;
  if constexpr (MODE == LINE_PROLONG_SMOOTH) {
    a.C = it.X;
    a.uc = it.c;
    line_body<float, HALF, MODE, true, EX>(it.L, a, it.nti, it.ntj, 0, B - it.blk0);
  } else {
    // the smoother stages its horizontal neighbours in LDS
    line_body<float, HALF, MODE, MODE == LINE_SMOOTH, EX>(it.L, a, it.nti, it.ntj, 0,
                                                          B - it.blk0);
  }
}

__global__ __launch_bounds__(NTHREADS) void k_resrestrict_grouped(
    const GItem<float>* __restrict__ items, int nitems, const int* __restrict__ active) {
  const int B = xcd_remap(blockIdx.x, gridDim.x);
  const GItem<float> it = items[find_item(items, nitems, B)];
  if (!active[it.pair]) return;
  resrestrict_body<float, SROWS, KSEG, 4>(it.L, it.X, it.a, it.b, it.o, it.nti, it.ntj, 0, B - it.blk0);
}

__global__ __launch_bounds__(NTHREADS) void k_prolongate_grouped(
    const GItem<float>* __restrict__ items, int nitems, const int* __restrict__ active) {
  const int B = xcd_remap(blockIdx.x, gridDim.x);
  const GItem<float> it = items[find_item(items, nitems, B)];
  if (!active[it.pair]) return;
  prolongate_body<float, SROWS>(it.X, it.L, it.a, it.o, it.nti, it.ntj, 0, B - it.blk0);
}

__global__ __launch_bounds__(NTHREADS) void k_correct_residual_grouped(
    const GItemCR* __restrict__ items, int nitems, const int* __restrict__ active,
    double* __restrict__ partials) {
  const int B = xcd_remap(blockIdx.x, gridDim.x);
  const GItemCR it = items[find_item(items, nitems, B)];
  if (!active[it.pair]) return;
  // partial of workgroup B of the item goes to slot B (the pair's segment)
  correct_residual_body<SROWS, 4>(it.L, it.u, it.e, it.f, it.uout, it.r32,
                               partials - blockIdx.x + B, it.nti, it.ntj, 0, B - it.blk0);
}

// ---------------------------------------------------------------------------
// Reductions and scalar updates (single workgroup, fixed summation order)
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void reduce_fixed(const double* __restrict__ partials, int64_t n,
                                             double (&out)[NC]) {
  __shared__ double sm[NC][NTHREADS];
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  // each thread adds its partials in index order; the loads of a batch are
  // issued together (the sums still run in the same order)
  constexpr int BQ = 16;
  for (int64_t q0 = threadIdx.x; q0 < n; q0 += (int64_t)BQ * NTHREADS) {
    double v[BQ][NC];
#pragma unroll
    for (int b = 0; b < BQ; ++b) {
      const int64_t q = q0 + (int64_t)b * NTHREADS;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[b][c] = q < n ? partials[q * NC + c] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < BQ; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += v[b][c];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) sm[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = NTHREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < NC; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = sm[c][0];
}

__global__ __launch_bounds__(NTHREADS) void k_reduce(const double* __restrict__ partials,
                                                     int64_t n, int ncomp,
                                                     double* __restrict__ out) {
  if (ncomp == 1) {
    double r[1];
    reduce_fixed<1>(partials, n, r);
    if (threadIdx.x == 0) out[0] = r[0];
  } else {
    double r[2];
    reduce_fixed<2>(partials, n, r);
    if (threadIdx.x == 0) {
      out[0] = r[0];
      out[1] = r[1];
    }
  }
}

__global__ __launch_bounds__(NTHREADS) void k_cg_fin1(CgState* st,
                                                      const double* __restrict__ partials,
                                                      int64_t n) {
  if (st->done) return;
  double r[1];
  reduce_fixed<1>(partials, n, r);
  if (threadIdx.x == 0) {
    const double sigma = r[0];
    st->sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
      st->status = 3;  // breakdown before the step: keep the previous iterate
      st->done = 1;
    } else {
      st->alpha_prev = st->alpha;
      st->alpha = st->kappa / sigma;
    }
  }
}

__global__ __launch_bounds__(NTHREADS) void k_cg_fin2(CgState* st,
                                                      const double* __restrict__ partials,
                                                      int64_t n, int init,
                                                      double* __restrict__ hist) {
  if (st->done) return;
  double r[2];
  reduce_fixed<2>(partials, n, r);
  if (threadIdx.x == 0) {
    const double rr = r[0], rz = r[1];
    st->rr = rr;
    if (init) {
      st->rr0 = rr;
      st->thresh2 *= rr;
      st->kappa = rz;
      st->iter = 0;
      st->alpha = 0.0;
      st->alpha_prev = 0.0;
      st->beta = 0.0;
      hist[0] = 1.0;
      if (rr == 0.0) st->done = 1;
      else if (!isfinite(rr) || !isfinite(rz)) { st->status = 2; st->done = 1; }
      return;
    }
    const int it = st->iter + 1;
    st->iter = it;
    hist[it] = sqrt(rr / st->rr0);
    if (!isfinite(rr) || !isfinite(rz)) {
      st->status = 2;
      st->done = 1;
    } else if (rr < st->thresh2) {
      st->done = 1;
    } else if (it >= st->maxit) {
      st->status = 1;
      st->done = 1;
    } else {
      st->beta = rz / st->kappa;
      st->kappa = rz;
    }
  }
}

// beta = -<z, q_old> / sigma_old  (0 on the first iteration: q_old = 0)
__global__ __launch_bounds__(NTHREADS) void k_fcg_fin_beta(CgState* st,
                                                           const double* __restrict__ partials,
                                                           int64_t n) {
  if (st->done) return;
  double r[1];
  reduce_fixed<1>(partials, n, r);
  if (threadIdx.x == 0) st->beta = st->iter == 0 ? 0.0 : -r[0] / st->sigma;
}

// sigma = <p, q>, alpha = <p, r> / sigma
__global__ __launch_bounds__(NTHREADS) void k_fcg_fin_alpha(CgState* st,
                                                            const double* __restrict__ partials,
                                                            int64_t n) {
  if (st->done) return;
  double r[2];
  reduce_fixed<2>(partials, n, r);
  if (threadIdx.x == 0) {
    st->sigma = r[0];
    if (!(r[0] > 0.0) || !isfinite(r[0])) {
      // breakdown before the step: alpha keeps the last step taken, which
      // the final update may still owe the iterate
      st->status = 3;
      st->done = 1;
    } else {
      st->alpha_prev = st->alpha;
      st->alpha = r[1] / r[0];
    }
  }
}

// ||r||^2 after the update: history, convergence, iteration count
__global__ __launch_bounds__(NTHREADS) void k_fcg_fin_res(CgState* st,
                                                          const double* __restrict__ partials,
                                                          int64_t n, double* __restrict__ hist) {
  if (st->done) return;  // stopped (a breakdown: keep its status and the count)
  double r[1];
  reduce_fixed<1>(partials, n, r);
  if (threadIdx.x == 0) {
    const double rr = r[0];
    st->rr = rr;
    const int it = st->iter + 1;
    st->iter = it;
    hist[it] = sqrt(rr / st->rr0);
    if (!isfinite(rr)) {
      st->status = 2;
      st->done = 1;
    } else if (rr < st->thresh2) {
      st->done = 1;
    } else if (it >= st->maxit) {
      st->status = 1;
      st->done = 1;
    }
  }
}

// Multigrid and iterative refinement (Sec. 2.2, stopping test): ||f - A u||^2
// of the current iterate from the partials.  init: the initial residual (the
// reference of the relative residual; a zero one ends the solve, a
// non-finite one fails it).  Otherwise the cycle is counted, its relative
// residual goes to the history, and the solve stops below rtol, at maxit or
// on a non-finite norm.  thresh2 = rtol^2 ||r_0||^2 serves the host's
// prediction of the iterations still needed.
__global__ __launch_bounds__(NTHREADS) void k_mg_fin(CgState* st,
                                                     const double* __restrict__ partials,
                                                     int64_t n, int init,
                                                     double* __restrict__ hist) {
  if (st->done) return;
  double r[1];
  reduce_fixed<1>(partials, n, r);
  if (threadIdx.x == 0) {
    const double rr = r[0];
    st->rr = rr;
    if (init) {
      st->rr0 = rr;
      st->thresh2 = st->rtol * st->rtol * rr;
      st->iter = 0;
      hist[0] = 1.0;
      if (!isfinite(rr)) {
        st->status = 2;
        st->done = 1;
      } else if (rr == 0.0) {
        st->done = 1;
      } else if (st->maxit <= 0) {
        st->status = 1;
        st->done = 1;
      }
      return;
    }
    const int it = st->iter + 1;
    st->iter = it;
    const double rel = sqrt(rr / st->rr0);
    hist[it] = rel;
    if (!isfinite(rel)) {
      st->status = 2;
      st->done = 1;
    } else if (rel < st->rtol) {
      st->done = 1;
    } else if (it >= st->maxit) {
      st->status = 1;
      st->done = 1;
    }
  }
}

// One workgroup per pair: sum the pair's partials (fixed order) and update
// its state.  init: record ||r_0||^2.  Otherwise count the iteration and stop
// the pair on convergence, maxit or a non-finite norm.
__global__ __launch_bounds__(NTHREADS) void k_pair_reduce(PairState* __restrict__ ps,
                                                          int* __restrict__ active,
                                                          const double* __restrict__ partials,
                                                          int init) {
  const int p = blockIdx.x;
  if (!active[p]) return;
  double r[1];
  reduce_fixed<1>(partials + ps[p].blk0, ps[p].nblk, r);
  if (threadIdx.x == 0) {
    const double rr = r[0];
    PairState& q = ps[p];
    q.rr = rr;
    if (init) {
      q.rr0 = rr;
      q.thresh2 *= rr;
      q.iters = 0;
      if (!isfinite(rr)) { q.status = 2; active[p] = 0; }
      else if (rr == 0.0) active[p] = 0;
      return;
    }
    q.iters += 1;
    if (!isfinite(rr)) { q.status = 2; active[p] = 0; }
    else if (rr < q.thresh2) active[p] = 0;
    else if (q.iters >= q.maxit) { q.status = 1; active[p] = 0; }
  }
}

// Line-PCG and flexible CG with paired updates: after n completed
// iterations (n = iter) the
// directions j <= n not yet in u are applied, in order.  The last direction
// step kernel that ran is iteration n + 1 after a breakdown before its step
// (status 3), else n; an even one (m) applied the directions up to m - 1, so
// one or two remain: n alone, or n - 1 and n.  Direction j lives in p_{j & 1}
// (an even step m overwrote p_{(m) & 1} only after reading it).
__global__ __launch_bounds__(NTHREADS) void k_pcg_final_update(Lvl<double> L,
                                                               double* __restrict__ u,
                                                               const double* __restrict__ p0,
                                                               const double* __restrict__ p1,
                                                               const CgState* __restrict__ st) {
  const int n = st->iter;
  if (n <= 0) return;
  const int last = n + (st->status == 3 ? 1 : 0);
  const int applied = (last & 1) ? last - 2 : last - 1;
  if (applied >= n) return;
  const double* pn = (n & 1) ? p1 : p0;
  const double* pm = (n & 1) ? p0 : p1;  // direction n - 1
  const double an = st->alpha, am = st->alpha_prev;
  const bool two = applied < n - 1;
  // the grid's cells only: the padding columns of the direction buffers are
  // never written
  const int64_t cnt = (int64_t)L.ny * L.nz * L.ldx;
  for (int64_t g = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; g < cnt;
       g += (int64_t)gridDim.x * NTHREADS) {
    if (g % L.ldx >= L.nx) continue;
    const double v = two ? fma(am, pm[g], u[g]) : u[g];
    u[g] = fma(an, pn[g], v);
  }
}

// dst = src over a level's field (both in its layout), gated like the
// iteration it belongs to
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_copy_level(Lvl<T> L, const T* __restrict__ src,
                                                         T* __restrict__ dst) {
  if (gated(L)) return;
  const int64_t n = (int64_t)L.ny * L.nz * L.ldx;
  for (int64_t g = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * NTHREADS)
    dst[g] = src[g];
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t g = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * NTHREADS)
    p[g] = v;
}

__global__ __launch_bounds__(NTHREADS) void k_add_f32_to_f64(double* __restrict__ u,
                                                             const float* __restrict__ e,
                                                             int64_t n) {
  for (int64_t g = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * NTHREADS)
    u[g] += (double)e[g];
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

inline int grid_stride_blocks(int64_t n) {
  int64_t b = (n + NTHREADS - 1) / NTHREADS;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// The two-wavefront staged smoother (launch shape rows = 3) needs columns of
// exactly 32, 64 or 128 layers and whole tiles of 64 columns x 2 rows.
template <typename T>
bool line_w2_fits(const Lvl<T>& L) {
  return L.nx % 64 == 0 && L.ny % 2 == 0 && (L.nz == 32 || L.nz == 64 || L.nz == 128);
}

template <typename T, int MODE>
hipError_t line_dispatch(const Lvl<T>& L, const LineArgs<T>& a, hipStream_t s, int group,
                         int rows = 4) {
  if constexpr (MODE == LINE_SOLVE || MODE == LINE_SMOOTH) {
    // one wavefront per column (parallel cyclic reduction) when asked for
    if (rows == 1 && L.nz <= 128) {
      const int ncols = L.nx * L.ny;
      hipLaunchKernelGGL((k_line_pcr<T, MODE>), dim3(cdiv(ncols, NTHREADS / 64)),
                         dim3(NTHREADS), 0, s, L, a, ncols);
      return hipGetLastError();
    }
  }
  const int nti = cdiv(L.nx, 32), ntj = cdiv(L.ny, LROWS);
  const dim3 grid(nti * ntj), block(NTHREADS);
  const int half = (L.nz + 1) / 2;
  if constexpr (MODE == LINE_SMOOTH || MODE == LINE_SMOOTH_NORM || MODE == LINE_PROLONG_SMOOTH) {
    // staged smoothers with two wavefronts per column where the level fits
    if (rows == 3 && line_w2_fits(L)) {
      const int nti2 = L.nx / 64, ntj2 = L.ny / 2;
      const dim3 grid2(nti2 * ntj2);
      if (L.nz == 128)
        hipLaunchKernelGGL((k_line<T, 64, MODE, true, true, true>), grid2, block, 0, s, L, a,
                           nti2, ntj2, group);
      else if (L.nz == 64)
        hipLaunchKernelGGL((k_line<T, 32, MODE, true, true, true>), grid2, block, 0, s, L, a,
                           nti2, ntj2, group);
      else
        hipLaunchKernelGGL((k_line<T, 16, MODE, true, true, true>), grid2, block, 0, s, L, a,
                           nti2, ntj2, group);
      return hipGetLastError();
    }
  }
  auto go = [&](auto nb) -> hipError_t {
    constexpr bool NB = decltype(nb)::value;
    // columns of exactly 32, 64 or 128 layers take the exact-height form
    if (L.nz == 32)
      hipLaunchKernelGGL((k_line<T, 16, MODE, NB, true>), grid, block, 0, s, L, a, nti, ntj,
                         group);
    else if (L.nz == 64)
      hipLaunchKernelGGL((k_line<T, 32, MODE, NB, true>), grid, block, 0, s, L, a, nti, ntj,
                         group);
    else if (L.nz == 128)
      hipLaunchKernelGGL((k_line<T, 64, MODE, NB, true>), grid, block, 0, s, L, a, nti, ntj,
                         group);
    else if (half <= 4)
      hipLaunchKernelGGL((k_line<T, 4, MODE, NB>), grid, block, 0, s, L, a, nti, ntj, group);
    else if (half <= 8)
      hipLaunchKernelGGL((k_line<T, 8, MODE, NB>), grid, block, 0, s, L, a, nti, ntj, group);
    else if (half <= 16)
      hipLaunchKernelGGL((k_line<T, 16, MODE, NB>), grid, block, 0, s, L, a, nti, ntj, group);
    else if (half <= 32)
      hipLaunchKernelGGL((k_line<T, 32, MODE, NB>), grid, block, 0, s, L, a, nti, ntj, group);
    else if (half <= 64)
      hipLaunchKernelGGL((k_line<T, 64, MODE, NB>), grid, block, 0, s, L, a, nti, ntj, group);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  };
  if constexpr (MODE == LINE_PROLONG_SMOOTH) {
    return go(std::true_type{});  // staged form only
  } else {
    // smoothers: horizontal neighbours staged in LDS when asked for (rows = 2,
    // and rows = 3 where the two-wavefront form does not fit the level)
    if constexpr (MODE == LINE_SMOOTH || MODE == LINE_SMOOTH_NORM) {
      if (rows == 2 || rows == 3) return go(std::true_type{});
    }
    return go(std::false_type{});
  }
}

}  // namespace

int64_t line_tiles_x(int nx) { return cdiv(nx, 32); }
int64_t line_tiles_y(int ny) { return cdiv(ny, LROWS); }
int64_t stencil_tiles_x(int nx) { return cdiv(nx, 64); }
int64_t stencil_tiles_y(int ny) { return cdiv(ny, SROWS); }
int64_t stencil_tiles_k(int nz) { return cdiv(nz, KSEG); }

hipError_t launch_grouped_f32(GKind kind, int half, bool exact, const GItem<float>* items,
                              int nitems, int nblocks, const int* active, float rho,
                              hipStream_t s) {
  const dim3 grid(nblocks), block(NTHREADS);
  switch (kind) {
    case GKind::LINE_SOLVE:
    case GKind::SMOOTH:
    case GKind::PROLONG_SMOOTH: {
      const bool sm = kind == GKind::SMOOTH;
      const bool ps = kind == GKind::PROLONG_SMOOTH;
#define GMG_GLINE(H, EX)                                                                     \
  if (half == H && exact == EX) {                                                            \
    if (ps)                                                                                  \
      hipLaunchKernelGGL((k_line_grouped<H, LINE_PROLONG_SMOOTH, EX>), grid, block, 0, s,    \
                         items, nitems, active, rho);                                        \
    else if (sm)                                                                             \
      hipLaunchKernelGGL((k_line_grouped<H, LINE_SMOOTH, EX>), grid, block, 0, s, items,     \
                         nitems, active, rho);                                               \
    else                                                                                     \
      hipLaunchKernelGGL((k_line_grouped<H, LINE_SOLVE, EX>), grid, block, 0, s, items,      \
                         nitems, active, rho);                                               \
    return hipGetLastError();                                                                \
  }
      GMG_GLINE(4, false)
      GMG_GLINE(8, false)
      GMG_GLINE(16, false)
      GMG_GLINE(32, false)
      GMG_GLINE(64, false)
      GMG_GLINE(16, true)
      GMG_GLINE(32, true)
      GMG_GLINE(64, true)
#undef GMG_GLINE
      return hipErrorInvalidValue;
    }
    case GKind::RESRESTRICT:
      hipLaunchKernelGGL(k_resrestrict_grouped, grid, block, 0, s, items, nitems, active);
      return hipGetLastError();
    case GKind::PROLONGATE:
      hipLaunchKernelGGL(k_prolongate_grouped, grid, block, 0, s, items, nitems, active);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_grouped_cr(const GItemCR* items, int nitems, int nblocks, const int* active,
                             double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_correct_residual_grouped, dim3(nblocks), dim3(NTHREADS), 0, s, items,
                     nitems, active, partials);
  return hipGetLastError();
}

hipError_t launch_pair_reduce(PairState* ps, int* active, const double* partials, int npairs,
                              int init, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_reduce, dim3(npairs), dim3(NTHREADS), 0, s, ps, active, partials,
                     init);
  return hipGetLastError();
}

int64_t stencil_blocks(int nx, int ny, int nz) {
  return (int64_t)cdiv(nx, 64) * cdiv(ny, SROWS) * cdiv(nz, KSEG);
}

int64_t line_blocks(int nx, int ny) { return (int64_t)cdiv(nx, 32) * cdiv(ny, LROWS); }

// Instantiate f with the compile-time rows of a stencil launch shape.
template <typename F>
hipError_t with_rows(int rows, F&& f) {
  switch (rows) {
    case 8:
      f(std::integral_constant<int, 8>{});
      break;
    case 16:
      f(std::integral_constant<int, 16>{});
      break;
    default:
      f(std::integral_constant<int, 4>{});
      break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Lvl<T>& L, Stencil mode, const T* x, const T* f, T* y,
                          float* ydown, double* partials, int64_t* nblocks, hipStream_t s,
                          Shape sh) {
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SR), nkb = cdiv(L.nz, KSEG);
    const dim3 grid(nti * ntj * nkb), block(64 * SR);
    if (nblocks) *nblocks = (int64_t)nti * ntj * nkb;
    switch (mode) {
      case Stencil::SPMV:
        hipLaunchKernelGGL((k_stencil<T, 0, SR>), grid, block, 0, s, L, x, f, y, ydown,
                           partials, nti, ntj, sh.group);
        break;
      case Stencil::RESIDUAL:
        hipLaunchKernelGGL((k_stencil<T, 1, SR>), grid, block, 0, s, L, x, f, y, ydown,
                           partials, nti, ntj, sh.group);
        break;
      case Stencil::RESIDUAL_NORM:
        hipLaunchKernelGGL((k_stencil<T, 2, SR>), grid, block, 0, s, L, x, f, y, ydown,
                           partials, nti, ntj, sh.group);
        break;
      case Stencil::RESIDUAL_NORM_DOWN:
        hipLaunchKernelGGL((k_stencil<T, 3, SR>), grid, block, 0, s, L, x, f, y, ydown,
                           partials, nti, ntj, sh.group);
        break;
    }
  });
}

template <typename T>
hipError_t launch_line_solve(const Lvl<T>& L, const T* r, T* z, hipStream_t s, Shape sh) {
  LineArgs<T> a{};
  a.a = r;
  a.o0 = z;
  a.rho = T(1);
  return line_dispatch<T, LINE_SOLVE>(L, a, s, sh.group, sh.rows);
}

template <typename T>
hipError_t launch_smooth(const Lvl<T>& L, const T* f, const T* uin, T* uout, T rho,
                         hipStream_t s, Shape sh) {
  LineArgs<T> a{};
  a.a = uin;
  a.b = f;
  a.o0 = uout;
  a.rho = rho;
  return line_dispatch<T, LINE_SMOOTH>(L, a, s, sh.group, sh.rows);
}

template <typename T>
hipError_t launch_prolong_smooth(const Lvl<T>& F, const Lvl<T>& C, const T* f, const T* uin,
                                 const T* uc, T* uout, T rho, hipStream_t s, Shape sh) {
  if (F.nx != 2 * C.nx || F.ny != 2 * C.ny || F.nz != C.nz) return hipErrorInvalidValue;
  LineArgs<T> a{};
  a.a = uin;
  a.b = f;
  a.o0 = uout;
  a.rho = rho;
  a.C = C;
  a.uc = uc;
  return line_dispatch<T, LINE_PROLONG_SMOOTH>(F, a, s, sh.group, sh.rows == 3 ? 3 : 2);
}

template <typename T>
hipError_t launch_restrict_smooth(const Lvl<T>& C, const Lvl<T>& F, const T* rf, T* fc, T* uc,
                                  T rho, hipStream_t s, Shape sh) {
  LineArgs<T> a{};
  a.a = rf;
  a.o0 = uc;
  a.o1 = fc;
  a.rho = rho;
  a.F = F;
  return line_dispatch<T, LINE_RESTRICT_SMOOTH>(C, a, s, sh.group);
}

template <typename T>
hipError_t launch_line_solve_scaled(const Lvl<T>& L, const T* r, T* z, T scale, hipStream_t s,
                                    Shape sh) {
  LineArgs<T> a{};
  a.a = r;
  a.o0 = z;
  a.rho = scale;
  return line_dispatch<T, LINE_SOLVE>(L, a, s, sh.group, sh.rows);
}

template <typename T>
hipError_t launch_smooth_norm(const Lvl<T>& L, const T* f, const T* uin, T* uout, T rho,
                              double* partials, int64_t* nblocks, hipStream_t s, Shape sh) {
  LineArgs<T> a{};
  a.a = uin;
  a.b = f;
  a.o0 = uout;
  a.rho = rho;
  a.partials = partials;
  *nblocks = (sh.rows == 3 && line_w2_fits(L)) ? (int64_t)(L.nx / 64) * (L.ny / 2)
                                                : line_blocks(L.nx, L.ny);
  return line_dispatch<T, LINE_SMOOTH_NORM>(L, a, s, sh.group, sh.rows);
}

// Levels with at most kShortSegCols lane columns walk segments of KSHORT
// layers instead of KSEG: their kernels are bound by the chain of dependent
// loads along a segment, not by bandwidth, and shorter segments give more
// workgroups to overlap those waits (the FP64 residual-restriction onto
// 64^2 and 32^2: 23 -> 12 and 19 -> 10 us; onto 128^2, which reads a 256^2
// level, they cost 10 %).
constexpr int KSHORT = 8;
constexpr int64_t kShortSegCols = 64 * 64;

template <typename T>
hipError_t launch_resrestrict(const Lvl<T>& F, const Lvl<T>& C, const T* u, const T* f, T* fc,
                              hipStream_t s, Shape sh) {
  const bool shortseg = (int64_t)C.nx * C.ny <= kShortSegCols;
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int ks = shortseg ? KSHORT : KSEG;
    const int nti = cdiv(C.nx, 64), ntj = cdiv(C.ny, SR), nkb = cdiv(C.nz, ks);
    if (shortseg)
      hipLaunchKernelGGL((k_resrestrict<T, SR, KSHORT>), dim3(nti * ntj * nkb), dim3(64 * SR), 0,
                         s, F, C, u, f, fc, nti, ntj, sh.group);
    else
      hipLaunchKernelGGL((k_resrestrict<T, SR, KSEG>), dim3(nti * ntj * nkb), dim3(64 * SR), 0,
                         s, F, C, u, f, fc, nti, ntj, sh.group);
  });
}

hipError_t launch_correct_residual(const Lvl<double>& L, const double* u, const float* e,
                                   const double* f, double* uout, float* r32, double* partials,
                                   int64_t* nblocks, hipStream_t s, Shape sh) {
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SR), nkb = cdiv(L.nz, KSEG);
    *nblocks = (int64_t)nti * ntj * nkb;
    hipLaunchKernelGGL(k_correct_residual<SR>, dim3(nti * ntj * nkb), dim3(64 * SR), 0, s, L, u,
                       e, f, uout, r32, partials, nti, ntj, sh.group);
  });
}

template <typename T>
hipError_t launch_prolongate(const Lvl<T>& C, const Lvl<T>& F, const T* uc, T* uf,
                             hipStream_t s, Shape sh) {
  const bool shortseg = (int64_t)F.nx * F.ny <= kShortSegCols;
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int ks = shortseg ? KSHORT : KSEG;
    const int nti = cdiv(F.nx, 64), ntj = cdiv(F.ny, SR), nkb = cdiv(F.nz, ks);
    if (shortseg)
      hipLaunchKernelGGL((k_prolongate<T, SR, KSHORT>), dim3(nti * ntj * nkb), dim3(64 * SR), 0,
                         s, C, F, uc, uf, nti, ntj, sh.group);
    else
      hipLaunchKernelGGL((k_prolongate<T, SR, KSEG>), dim3(nti * ntj * nkb), dim3(64 * SR), 0, s,
                         C, F, uc, uf, nti, ntj, sh.group);
  });
}

hipError_t launch_cg_p1(const Lvl<double>& L, double* u, const double* pr, double* pw,
                        const double* z, double* q, const CgState* st, bool paired,
                        double* partials, int64_t* nblocks, hipStream_t s, Shape sh) {
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SR), nkb = cdiv(L.nz, KSEG);
    *nblocks = (int64_t)nti * ntj * nkb;
    if (paired)
      hipLaunchKernelGGL((k_cg_p1<SR, true>), dim3(nti * ntj * nkb), dim3(64 * SR), 0, s, L, u,
                         pr, pw, z, q, st, partials, nti, ntj, sh.group);
    else
      hipLaunchKernelGGL((k_cg_p1<SR, false>), dim3(nti * ntj * nkb), dim3(64 * SR), 0, s, L, u,
                         pr, pw, z, q, st, partials, nti, ntj, sh.group);
  });
}

hipError_t launch_cg_p2(const Lvl<double>& L, double* r, const double* q, double* z,
                        const CgState* st, int init, double* partials, int64_t* nblocks,
                        hipStream_t s, Shape sh) {
  LineArgs<double> a{};
  a.a = q;
  a.rw = r;
  a.o0 = z;
  a.st = st;
  a.init = init;
  a.partials = partials;
  *nblocks = line_blocks(L.nx, L.ny);
  return line_dispatch<double, LINE_CG>(L, a, s, sh.group);
}

template <typename TZ>
hipError_t launch_fcg_zq(const Lvl<double>& L, const TZ* z, const double* q, double* partials,
                         int64_t* nblocks, hipStream_t s) {
  const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SROWS), nkb = cdiv(L.nz, KSEG);
  *nblocks = (int64_t)nti * ntj * nkb;
  hipLaunchKernelGGL((k_fcg_zq<TZ>), dim3(nti * ntj * nkb), dim3(NTHREADS), 0, s, L, z, q,
                     partials, nti, ntj);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fcg_dir(const Lvl<double>& L, const TZ* z, double* u, const double* pr,
                          double* pw, double* q, const double* r, const CgState* st, bool paired,
                          double* partials, int64_t* nblocks, hipStream_t s, Shape sh) {
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SR), nkb = cdiv(L.nz, KSEG);
    *nblocks = (int64_t)nti * ntj * nkb;
    if (paired)
      hipLaunchKernelGGL((k_fcg_dir<TZ, SR, true>), dim3(nti * ntj * nkb), dim3(64 * SR), 0, s, L,
                         z, u, pr, pw, q, r, st, partials, nti, ntj, sh.group);
    else
      hipLaunchKernelGGL((k_fcg_dir<TZ, SR, false>), dim3(nti * ntj * nkb), dim3(64 * SR), 0, s,
                         L, z, u, pr, pw, q, r, st, partials, nti, ntj, sh.group);
  });
}

hipError_t launch_fcg_update(const Lvl<double>& L, double* r, const double* q, float* rdown,
                             const CgState* st, double* partials, int64_t* nblocks,
                             hipStream_t s, Shape sh) {
  return with_rows(sh.rows, [&](auto R) {
    constexpr int SR = decltype(R)::value;
    const int nti = cdiv(L.nx, 64), ntj = cdiv(L.ny, SR), nkb = cdiv(L.nz, KSEG);
    *nblocks = (int64_t)nti * ntj * nkb;
    hipLaunchKernelGGL(k_fcg_update<SR>, dim3(nti * ntj * nkb), dim3(64 * SR), 0, s, L, r, q,
                       rdown, st, partials, nti, ntj, sh.group);
  });
}

hipError_t launch_fcg_fin(int which, CgState* st, const double* partials, int64_t nblocks,
                          double* hist, hipStream_t s) {
  if (which == 0)
    hipLaunchKernelGGL(k_fcg_fin_beta, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks);
  else if (which == 1)
    hipLaunchKernelGGL(k_fcg_fin_alpha, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks);
  else
    hipLaunchKernelGGL(k_fcg_fin_res, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks,
                       hist);
  return hipGetLastError();
}

template hipError_t launch_fcg_zq<double>(const Lvl<double>&, const double*, const double*,
                                          double*, int64_t*, hipStream_t);
template hipError_t launch_fcg_zq<float>(const Lvl<double>&, const float*, const double*,
                                         double*, int64_t*, hipStream_t);
template hipError_t launch_fcg_dir<double>(const Lvl<double>&, const double*, double*,
                                           const double*, double*, double*, const double*,
                                           const CgState*, bool, double*, int64_t*, hipStream_t,
                                           Shape);
template hipError_t launch_fcg_dir<float>(const Lvl<double>&, const float*, double*,
                                          const double*, double*, double*, const double*,
                                          const CgState*, bool, double*, int64_t*, hipStream_t,
                                          Shape);

hipError_t launch_cg_fin1(CgState* st, const double* partials, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_fin1, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks);
  return hipGetLastError();
}

hipError_t launch_cg_fin2(CgState* st, const double* partials, int64_t nblocks, int init,
                          double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_fin2, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks, init,
                     hist);
  return hipGetLastError();
}

hipError_t launch_pcg_final_update(const Lvl<double>& L, double* u, const double* p0,
                                   const double* p1, const CgState* st, hipStream_t s) {
  const int64_t n = (int64_t)L.ny * L.nz * L.ldx;
  hipLaunchKernelGGL(k_pcg_final_update, dim3(grid_stride_blocks(n)), dim3(NTHREADS), 0, s, L,
                     u, p0, p1, st);
  return hipGetLastError();
}

hipError_t launch_mg_fin(CgState* st, const double* partials, int64_t nblocks, int init,
                         double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_fin, dim3(1), dim3(NTHREADS), 0, s, st, partials, nblocks, init, hist);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int64_t nblocks, int ncomp, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NTHREADS), 0, s, partials, nblocks, ncomp, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_level(const Lvl<T>& L, const T* src, T* dst, hipStream_t s) {
  const int64_t n = (int64_t)L.ny * L.nz * L.ldx;
  hipLaunchKernelGGL((k_copy_level<T>), dim3(grid_stride_blocks(n)), dim3(NTHREADS), 0, s, L,
                     src, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_stride_blocks(n)), dim3(NTHREADS), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_add_f32_to_f64(double* u, const float* e, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f32_to_f64, dim3(grid_stride_blocks(n)), dim3(NTHREADS), 0, s, u, e,
                     n);
  return hipGetLastError();
}

#define GMG_INSTANTIATE(T)                                                                    \
  template hipError_t launch_stencil<T>(const Lvl<T>&, Stencil, const T*, const T*, T*,       \
                                        float*, double*, int64_t*, hipStream_t, Shape);       \
  template hipError_t launch_line_solve<T>(const Lvl<T>&, const T*, T*, hipStream_t, Shape);  \
  template hipError_t launch_smooth<T>(const Lvl<T>&, const T*, const T*, T*, T, hipStream_t, \
                                       Shape);                                                \
  template hipError_t launch_prolong_smooth<T>(const Lvl<T>&, const Lvl<T>&, const T*,        \
                                               const T*, const T*, T*, T, hipStream_t, Shape);\
  template hipError_t launch_restrict_smooth<T>(const Lvl<T>&, const Lvl<T>&, const T*, T*,   \
                                                T*, T, hipStream_t, Shape);                   \
  template hipError_t launch_prolongate<T>(const Lvl<T>&, const Lvl<T>&, const T*, T*,        \
                                           hipStream_t, Shape);                               \
  template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                            \
  template hipError_t launch_copy_level<T>(const Lvl<T>&, const T*, T*, hipStream_t);         \
  template hipError_t launch_line_solve_scaled<T>(const Lvl<T>&, const T*, T*, T, hipStream_t, \
                                                  Shape);                                     \
  template hipError_t launch_smooth_norm<T>(const Lvl<T>&, const T*, const T*, T*, T, double*, \
                                            int64_t*, hipStream_t, Shape);                    \
  template hipError_t launch_resrestrict<T>(const Lvl<T>&, const Lvl<T>&, const T*, const T*, \
                                            T*, hipStream_t, Shape);

GMG_INSTANTIATE(double)
GMG_INSTANTIATE(float)

}  // namespace gmg
