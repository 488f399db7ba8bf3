// The residual with its FP64 norm for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): the per-workgroup partial sums of ||r||^2 go to a
// file-scope device array instead of the context's scratch, and the norm is
// written to a device double of the caller, so the call neither allocates nor
// synchronises.
//
// The array is one per GPU and lives until the process ends.  Its device
// address is looked up once per device, with that device current (at context
// setup, or at the first call on a device), and only that address is handed to
// kernels: in host code the array's own name is a host-side stand-in.

#include <stdio.h>

#include <mutex>

#include "gmg_internal.h"

namespace {

// 1 MiB: the partial sums of a residual launch (one FP64 value per workgroup;
// the smallest stencil workgroup covers 64 columns x 4 rows x 32 layers).
constexpr int64_t kScratchDoubles = 131072;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

int err(int code, const char* what, hipError_t e) {
  char msg[256];
  snprintf(msg, sizeof(msg), "%s: %s", what, hipGetErrorString(e));
  return gmg::set_error(code, msg);
}

}  // namespace

namespace gmg {

int scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return err(GMG_EHIP, "hipGetDevice", e);
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GMG_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return err(GMG_EHIP, "hipGetSymbolAddress(scratch)", e);
    g_scratch[dev] = static_cast<double*>(p);
  }
  if (out) *out = g_scratch[dev];
  return GMG_OK;
}

}  // namespace gmg

extern "C" {

int gmg_residual_noalloc(gmg_ctx* c, int level, int prec, const void* f, const void* u, void* r,
                         double* norm2, void* stream) {
  if (!c || c->batch || level < 0 || level >= c->nlevels)
    return gmg::set_error(GMG_EINVAL, "bad context or level");
  if (prec != GMG_F64 && prec != GMG_F32) return gmg::set_error(GMG_EINVAL, "prec must be 0 or 1");
  for (const void* q : {f, u, (const void*)r}) {
    if (!q) return gmg::set_error(GMG_EINVAL, "NULL field pointer");
    if (reinterpret_cast<uintptr_t>(q) % 16)
      return gmg::set_error(GMG_EINVAL, "field pointer not 16-byte aligned");
  }
  if (r == u || r == f) return gmg::set_error(GMG_EINVAL, "r must not overlap f or u");
  if (norm2 && reinterpret_cast<uintptr_t>(norm2) % 8)
    return gmg::set_error(GMG_EINVAL, "norm2 not 8-byte aligned");
  const gmg::LevelBuf& B = c->lev[level];
  // every stencil launch shape has at least 4 rows, so this bounds the
  // workgroup count of the residual launch
  if (norm2 && gmg::stencil_blocks(B.nx, B.ny, B.nz) > kScratchDoubles)
    return gmg::set_error(GMG_EINVAL,
                          "level too large for the static scratch (more than 131072 residual "
                          "workgroups)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* part = nullptr;
  if (norm2) {
    const int st = gmg::scratch_address(&part);
    if (st) return st;
  }
  const gmg::Stencil mode = norm2 ? gmg::Stencil::RESIDUAL_NORM : gmg::Stencil::RESIDUAL;
  const gmg::Shape sh = c->shape[gmg::tslot(GMG_K_RESIDUAL, level, prec)];
  int64_t nb = 0;
  hipError_t e;
  if (prec == GMG_F64)
    e = gmg::launch_stencil<double>(gmg::view<double>(c, level), mode, (const double*)u,
                                    (const double*)f, (double*)r, nullptr, part, &nb, s, sh);
  else
    e = gmg::launch_stencil<float>(gmg::view<float>(c, level), mode, (const float*)u,
                                   (const float*)f, (float*)r, nullptr, part, &nb, s, sh);
  if (e != hipSuccess) return err(GMG_EHIP, "residual launch", e);
  if (norm2) {
    // the launch wrote every one of its nb partials, so nothing an earlier
    // call left in the array is read
    if ((e = gmg::launch_reduce(part, nb, 1, norm2, s)) != hipSuccess)
      return err(GMG_EHIP, "reduction launch", e);
  }
  return GMG_OK;
}

}  // extern "C"
