// Mode reconstruction Phi = V B (the modes of Algorithm 1): the panel-layout
// basis W (n x k columns in use, FP32 or FP64) times the k x r coefficient
// matrix B (FP64, sigma folded in, packed real columns).  An FP32 basis with
// FP32 output runs on FP32 MFMA; every other combination uses the FP64-
// accumulating row kernel.
#include <algorithm>

#include "foa_buffer.h"
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

// MFMA kernel (FP32 basis, FP32 output): Phi^T = B^T W^T on 32x32x2 FP32 MFMA
// with FP32 accumulation.  Tile: 128 data rows (two panels) x 32*NB mode
// columns per workgroup; wavefront w owns data rows 32w..32w+31 and all NB
// 32-mode blocks, so for r <= 256 the basis is read exactly once.  k advances
// in chunks of 32 staged through LDS, the next chunk's global loads in flight
// in registers while the current one is multiplied: W as As[k][row] (rows
// contiguous, as in the panel layout), B as Bs[k][mode], both with row strides
// that put the two half-wavefronts of a fragment read 32 banks apart.  B
// arrives as FP32, k-major and zero-padded to whole chunks and mode blocks, so
// its loads need no masks.  Operands: A = B^T (lane l holds mode l%32,
// k-offset l/32), B = W^T (lane l holds data row l%32, k-offset l/32); the
// result D[i][j] has j = lane % 32, so each store instruction writes 32
// consecutive rows of one mode column.
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int MT_ROWS = 128, MT_K = 32, MT_LDA = 160;

__host__ __device__ constexpr int mfma_nb(int r) { return r <= 32 ? 1 : (r + 31) / 32 < 8 ? (r + 31) / 32 : 8; }

bool modes_use_mfma(bool tv_f64, bool out_f64) { return !tv_f64 && !out_f64; }
int modes_kpad(int k) { return (k + MT_K - 1) / MT_K * MT_K; }
int modes_rpad(int r) {
  const int t = 32 * mfma_nb(r);
  return (r + t - 1) / t * t;
}

// Up to NB = 5 the registers fit three wavefronts per SIMD (three workgroups
// per CU), so one workgroup's staging and epilogue overlap the others' MFMA.
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB <= 5 ? 3 : 2))) void k_modes_mfma(const float *W, int64_t n, int64_t P, int n_max, int kdim,
                                                    const float *Bt, int rpad, int r, float *out, int64_t ld) {
  constexpr int LDB = 32 * NB + (NB % 2 == 0 ? 32 : 0);
  constexpr int GPR = 8 * NB;  // 16-byte groups per staged B row
  __shared__ float As[MT_K * MT_LDA];
  __shared__ float Bs[MT_K * LDB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * MT_ROWS;
  const int64_t p0 = m0 / PANEL;
  const int npan = (int)(P - p0 < 2 ? P - p0 : 2);
  const int n0 = blockIdx.y * 32 * NB;
  // This tile's (at most two) panels of W: rows of a missing second panel and
  // basis columns >= kdim read as 0.
  const unsigned pbytes = (unsigned)n_max * PANEL * 4;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(W + (size_t)p0 * n_max * PANEL, npan * pbytes);
  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[b][t] = 0.f;

  f32x4v ra[4], rb[NB];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = (tid + u * 256) * 4;  // first of 4 consecutive rows
      const int c = e / MT_ROWS, row = e % MT_ROWS;
      const unsigned off = k0 + c < kdim ? (row / PANEL) * pbytes + ((k0 + c) * PANEL + row % PANEL) * 4u : kOOR;
      ra[u] = __builtin_bit_cast(f32x4v, __builtin_amdgcn_raw_buffer_load_b128(rw, (int)off, 0, kTileLoad));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * 256;
      rb[u] = *reinterpret_cast<const f32x4v *>(Bt + (size_t)(k0 + e / GPR) * rpad + n0 + (e % GPR) * 4);
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = (tid + u * 256) * 4;
      *reinterpret_cast<f32x4v *>(&As[(e / MT_ROWS) * MT_LDA + e % MT_ROWS]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * 256;
      *reinterpret_cast<f32x4v *>(&Bs[(e / GPR) * LDB + (e % GPR) * 4]) = rb[u];
    }
  };
  // operand fragments of k-step kk
  float wf[2], bf[2][NB];
  auto read_frag = [&](int kk, float &w, float (&b)[NB]) {
    const int kr = kk + (lane >> 5);
    w = As[kr * MT_LDA + wave * 32 + (lane & 31)];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = Bs[kr * LDB + i * 32 + (lane & 31)];
  };

  load_chunk(0);
  for (int k0 = 0; k0 < kdim; k0 += MT_K) {
    store_chunk();
    __syncthreads();
    if (k0 + MT_K < kdim) load_chunk(k0 + MT_K);
    // the fragments of step kk + 2 are read while step kk's products run
    read_frag(0, wf[0], bf[0]);
#pragma unroll
    for (int kk = 0; kk < MT_K; kk += 2) {
      const int cur = (kk / 2) & 1;
      if (kk + 2 < MT_K) read_frag(kk + 2, wf[cur ^ 1], bf[cur ^ 1]);
      // keep the scheduler from sinking those reads next to their use
      __builtin_amdgcn_sched_barrier(0);
      if (k0 + kk < kdim) {  // ragged last chunk (uniform branch)
#pragma unroll
        for (int i = 0; i < NB; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(bf[cur][i], wf[cur], acc[i], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
  // D[i][j]: j = lane % 32 (data row), i = 8 (t / 4) + 4 (lane / 32) + t % 4 (mode)
  const int64_t row = m0 + wave * 32 + (lane & 31);
  if (row >= n) return;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int mode = n0 + b * 32 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
      if (mode < r) out[(size_t)mode * ld + row] = acc[b][t];
    }
  }
}

template <int NB>
static void launch_mfma_nb(const float *W, int64_t n, int n_max, int k, const float *Bt, int r, float *out,
                           int64_t ld, hipStream_t s) {
  const int64_t P = (n + PANEL - 1) / PANEL;
  dim3 g((unsigned)((n + MT_ROWS - 1) / MT_ROWS), (unsigned)((r + 32 * NB - 1) / (32 * NB)));
  hipLaunchKernelGGL((k_modes_mfma<NB>), g, dim3(256), 0, s, W, n, P, n_max, k, Bt, modes_rpad(r), r, out, ld);
}

static void launch_mfma(const float *W, int64_t n, int n_max, int k, const float *Bt, int r, float *out,
                        int64_t ld, hipStream_t s) {
  switch (mfma_nb(r)) {
    case 1: launch_mfma_nb<1>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 2: launch_mfma_nb<2>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 3: launch_mfma_nb<3>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 4: launch_mfma_nb<4>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 5: launch_mfma_nb<5>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 6: launch_mfma_nb<6>(W, n, n_max, k, Bt, r, out, ld, s); break;
    case 7: launch_mfma_nb<7>(W, n, n_max, k, Bt, r, out, ld, s); break;
    default: launch_mfma_nb<8>(W, n, n_max, k, Bt, r, out, ld, s); break;
  }
}

hipError_t launch_modes_gemm(bool tv_f64, const void *W, int64_t n, int n_max, int k, const void *Bv, int r,
                             void *out, int64_t ld, bool out_f64, hipStream_t s) {
  if (r <= 0 || k <= 0) return hipSuccess;
  if (k > 512) return hipErrorInvalidValue;
  if (modes_use_mfma(tv_f64, out_f64)) {
    launch_mfma((const float *)W, n, n_max, k, (const float *)Bv, r, (float *)out, ld, s);
    return hipGetLastError();
  }
  const double *B = (const double *)Bv;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((r + 15) / 16));
  if (tv_f64) {
    if (out_f64)
      hipLaunchKernelGGL((k_modes_rowwise<double, double>), grid, dim3(256), 0, s, (const double *)W, n, n_max, k,
                         B, r, (double *)out, ld);
    else
      hipLaunchKernelGGL((k_modes_rowwise<double, float>), grid, dim3(256), 0, s, (const double *)W, n, n_max, k,
                         B, r, (float *)out, ld);
  } else {
    hipLaunchKernelGGL((k_modes_rowwise<float, double>), grid, dim3(256), 0, s, (const float *)W, n, n_max, k, B,
                       r, (double *)out, ld);
  }
  return hipGetLastError();
}

}  // namespace foa
