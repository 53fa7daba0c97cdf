// Mode reconstruction Phi = V B (Algorithm 1 steps 25 and 28): the panel-layout
// basis W (n x k columns in use, FP32 or FP64) times the k x r coefficient
// matrix B (FP64, sigma folded in, packed real columns).
#include "foa_internal.h"

namespace foa {

// Reference kernel: one thread per row, 16 output columns per block column,
// the block's 16 columns of B staged in LDS, FP64 accumulation.
template <typename TV, typename TO>
__global__ __launch_bounds__(256) void k_modes_rowwise(const TV *W, int64_t n, int n_max, int k,
                                                       const double *B, int r, TO *out, int64_t ld) {
  __shared__ double sB[512 * 16];
  const int c0 = blockIdx.y * 16;
  const int nc = min(16, r - c0);
  for (int idx = threadIdx.x; idx < k * 16; idx += 256) {
    const int l = idx / 16, cc = idx % 16;
    sB[idx] = cc < nc ? B[(size_t)(c0 + cc) * k + l] : 0.0;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  const TV *base = W + (size_t)(row / PANEL) * n_max * PANEL + (row % PANEL);
  double acc[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) acc[cc] = 0.0;
  for (int l = 0; l < k; ++l) {
    const double w = (double)base[(size_t)l * PANEL];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc[cc] = fma(w, sB[l * 16 + cc], acc[cc]);
  }
  for (int cc = 0; cc < nc; ++cc) out[(size_t)(c0 + cc) * ld + row] = (TO)acc[cc];
}

hipError_t launch_modes_gemm(bool tv_f64, const void *W, int64_t n, int n_max, int k, const double *B, int r,
                             void *out, int64_t ld, bool out_f64, hipStream_t s) {
  if (r <= 0 || k <= 0) return hipSuccess;
  if (k > 512) return hipErrorInvalidValue;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((r + 15) / 16));
  if (tv_f64) {
    if (out_f64)
      hipLaunchKernelGGL((k_modes_rowwise<double, double>), grid, dim3(256), 0, s, (const double *)W, n, n_max, k,
                         B, r, (double *)out, ld);
    else
      hipLaunchKernelGGL((k_modes_rowwise<double, float>), grid, dim3(256), 0, s, (const double *)W, n, n_max, k,
                         B, r, (float *)out, ld);
  } else {
    if (out_f64)
      hipLaunchKernelGGL((k_modes_rowwise<float, double>), grid, dim3(256), 0, s, (const float *)W, n, n_max, k,
                         B, r, (double *)out, ld);
    else
      hipLaunchKernelGGL((k_modes_rowwise<float, float>), grid, dim3(256), 0, s, (const float *)W, n, n_max, k, B,
                         r, (float *)out, ld);
  }
  return hipGetLastError();
}

}  // namespace foa
