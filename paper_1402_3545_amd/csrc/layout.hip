// Layout conversion kernels (the host-transfer side of the path).

#include "gmg_internal.h"

namespace gmg {

namespace {

constexpr int NTHREADS = 256;

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Layout conversion between the canonical z-contiguous order
// (j*nx + i)*nz + k of host data and the x-contiguous device order
// (j*nz + k)*ldx + i (Sec. 3.1 stores fields x-contiguous; Sec. 5.1 times the
// host transfer and this transpose separately).  A workgroup moves one
// 32 x 32 (i, k) tile of one grid row j through LDS, so the reads and the
// writes both run along contiguous memory.  Padding columns i >= nx of the
// x-contiguous field are not touched.
// ---------------------------------------------------------------------------
template <typename T, bool TO_X>
__global__ __launch_bounds__(NTHREADS) void k_transpose(const T* __restrict__ src,
                                                        T* __restrict__ dst, int nx, int nz,
                                                        int64_t ldx, int ntx, int ntz) {
  __shared__ T tile[32][33];
  int b = blockIdx.x;
  const int tz = b % ntz;
  b /= ntz;
  const int tx = b % ntx;
  const int j = b / ntx;
  const int i0 = tx * 32, k0 = tz * 32;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8 threads
  const int64_t zrow = (int64_t)j * nx;        // z-contiguous: column index base
  const int64_t xrow = (int64_t)j * nz * ldx;  // x-contiguous: row slab base
  if constexpr (TO_X) {
    for (int r = ly; r < 32; r += 8) {  // r: column i0+r, lx: layer k0+lx
      const int i = i0 + r, k = k0 + lx;
      if (i < nx && k < nz) tile[r][lx] = src[(zrow + i) * nz + k];
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {  // r: layer k0+r, lx: column i0+lx
      const int k = k0 + r, i = i0 + lx;
      if (i < nx && k < nz) dst[xrow + (int64_t)k * ldx + i] = tile[lx][r];
    }
  } else {
    for (int r = ly; r < 32; r += 8) {  // r: layer k0+r, lx: column i0+lx
      const int k = k0 + r, i = i0 + lx;
      if (i < nx && k < nz) tile[lx][r] = src[xrow + (int64_t)k * ldx + i];
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {  // r: column i0+r, lx: layer k0+lx
      const int i = i0 + r, k = k0 + lx;
      if (i < nx && k < nz) dst[(zrow + i) * nz + k] = tile[r][lx];
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_transpose(const T* src, T* dst, int nx, int ny, int nz, int64_t ldx,
                            bool to_x, hipStream_t s) {
  const int ntx = cdiv(nx, 32), ntz = cdiv(nz, 32);
  const int64_t nb = (int64_t)ny * ntx * ntz;
  if (nb <= 0 || nb > INT32_MAX) return hipErrorInvalidValue;
  if (to_x)
    hipLaunchKernelGGL((k_transpose<T, true>), dim3((unsigned)nb), dim3(NTHREADS), 0, s, src,
                       dst, nx, nz, ldx, ntx, ntz);
  else
    hipLaunchKernelGGL((k_transpose<T, false>), dim3((unsigned)nb), dim3(NTHREADS), 0, s, src,
                       dst, nx, nz, ldx, ntx, ntz);
  return hipGetLastError();
}
template hipError_t launch_transpose<double>(const double*, double*, int, int, int, int64_t, bool,
                                             hipStream_t);
template hipError_t launch_transpose<float>(const float*, float*, int, int, int, int64_t, bool,
                                            hipStream_t);

// Streaming copy for measuring the achievable HBM bandwidth: 8-byte
// non-temporal loads and stores, grid-stride, 1024-thread workgroups (up to
// 16384 of them), the fastest plain-copy form measured on gfx950.
__global__ __launch_bounds__(1024) void k_copy_probe(const double* __restrict__ src,
                                                     double* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 1024;
  for (int64_t g = (int64_t)blockIdx.x * 1024 + threadIdx.x; g < n; g += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + g), dst + g);
}

hipError_t launch_copy_probe(const double* src, double* dst, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(16384, (n + 1023) / 1024);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)blocks), dim3(1024), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace gmg
