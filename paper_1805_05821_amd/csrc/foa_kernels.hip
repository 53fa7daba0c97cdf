// HIP kernels (gfx950) of one FOA push: one iteration of the snapshot loop of
// Algorithm 1 of Anantharamu & Mahesh, restructured as three fused row passes
// over the basis.
//
// The paper's literal schedule sweeps V five times per snapshot (forming w,
// the projection, the first orthogonalisation, the reprojection and the
// second orthogonalisation).  Each pair -- w and its projection, the first
// orthogonalisation and the reprojection, the second orthogonalisation and
// the norm -- is "apply a row-local update with coefficients known before the
// pass, then reduce over the rows", so one pass over V serves both halves;
// the two projections must finish globally before the next update, so three
// sweeps is the minimum for classical Gram-Schmidt with one
// reorthogonalisation.
//
//   pass A : w = (psi - V b) / beta_jj ; partial V^T w ; partial ||psi||^2
//   reduce : h = V^T w
//   pass B : w = w - V h ; partial V^T w
//   reduce : s = V^T w ; h = h + s
//   pass C : w = w - V s ; v_{j+1} <- w ; partial ||w||^2
//   finalize: h_{j+1,j} = ||w||, breakdown test, H_bar column, beta
//             completion, then the next push's partial beta column
//             (eq. betacolumnupdate) in a small multi-block kernel.
//
// The basis is stored unnormalised: column c holds fl(w_c) and
// v_c = sigma_c * column_c with sigma_c = 1 / h_{c,c-1} (sigma_1 = 1/beta_11).
// Every coefficient vector handed to a pass is pre-multiplied by sigma and every
// projection is post-multiplied by sigma, so the normalisation's division
// never needs its own sweep over n.  All dot products, norms and small-matrix arithmetic are FP64.
//
// Reductions are deterministic: every partial sum has a fixed association
// (per-lane register sums in panel order, butterfly within a wavefront, fixed
// per-block order); no floating-point atomics are used.

#include "foa_device.h"


namespace foa {

template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(pass_waves<TV, QW>()))) void k_pass(PassArgs a) {
  if (a.st->status != ST_ACTIVE) return;
  __shared__ double lds[pass_lds_doubles<TV, NW, QW, MODE>()];
  row_pass_body<TV, TX, NW, QW, MODE, PREF>(a, blockIdx.x, a.P, gridDim.x, blockIdx.x, lds);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(SmallArgs a) {
  if (a.st->status != ST_ACTIVE) return;
  reduce_body<MODE>(a, blockIdx.x * 4);
}

__global__ __launch_bounds__(256) void k_finalize(SmallArgs a) { finalize_body(a); }
__global__ __launch_bounds__(256) void k_finalize_init(SmallArgs a) { finalize_init_body(a); }
__global__ __launch_bounds__(256) void k_nextb(SmallArgs a) { nextb_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_init_state(SmallArgs a, double tol) { init_state_body(a, tol); }

template <typename TV, typename TO>
__global__ __launch_bounds__(256) void k_copy_basis(const TV *W, const double *sigma, int64_t r0,
                                                    int64_t nrows, int n_max, int ncols, TO *out,
                                                    int64_t ld) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nrows || c >= ncols) return;
  const int64_t r = r0 + i;
  const int64_t p = r / PANEL;
  const double v = (double)W[((size_t)p * n_max + c) * PANEL + (r % PANEL)];
  out[(size_t)c * ld + i] = (TO)(sigma[c] * v);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Smallest QW in {1, 2, 4, 8, 16} whose instance covers j columns when one
// QW step spans cols_per_qw columns.
int pick_qw(int j, int cols_per_qw) {
  int qw = 1;
  while (qw < 16 && qw * cols_per_qw < j) qw *= 2;
  return qw;
}

int tile_slot(int qw) {
  switch (qw) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
    case 6: return 5;
    default: return 6;
  }
}

// The FP32 pass has 6- and 12-group tiles where the power-of-two tile would
// be a third to a half empty and the narrower one measured faster at
// n = 2^24: 8 x 6 for 129-192 columns (about 2%), 8 x 12 for 257-320 (about
// 2%) and 16 x 6 for 321-384 (about 5%; 16 x 6 for 257-320 was 6% slower
// than 8 x 16, and 8 x 12 for 321-384 no faster than 16 x 6).
int pass_qw(bool tv_f64, int nw, int j) {
  if (!tv_f64 && ((nw == 8 && j > 128 && j <= 192) || (nw == 16 && j > 320 && j <= 384))) return 6;
  if (!tv_f64 && nw == 8 && j > 256 && j <= 320) return 12;
  return pick_qw(j > 0 ? j : 1, tv_f64 ? 32 : nw * 4);
}

template <typename TV, typename TX, int NW, int MODE, bool PREF>
static hipError_t launch_pass_q(int qw, int grid, const PassArgs &a, hipStream_t s) {
  constexpr int NT = NW * 64;
  switch (qw) {
    case 1: hipLaunchKernelGGL((k_pass<TV, TX, NW, 1, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pass<TV, TX, NW, 2, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pass<TV, TX, NW, 4, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_pass<TV, TX, NW, 8, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 6:
      if constexpr (sizeof(TV) == 4 && NW >= 8) {
        hipLaunchKernelGGL((k_pass<TV, TX, NW, 6, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case 12:
      if constexpr (sizeof(TV) == 4 && NW == 8) {
        hipLaunchKernelGGL((k_pass<TV, TX, NW, 12, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default:
      if constexpr (NW * 16 * Vec<TV>::EPL <= 512)
        hipLaunchKernelGGL((k_pass<TV, TX, NW, 16, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a);
      else
        return hipErrorInvalidValue;
      break;
  }
  return hipGetLastError();
}

// Register budget: a 16-group FP64 tile (64 VGPRs) cannot be double buffered
// within the 128 VGPRs a 16-wavefront workgroup allows.
template <typename TV, int NW>
static bool prefetch_fits(int qw) {
  return !(sizeof(TV) == 8 && NW == 16 && qw >= 16);
}

template <typename TV, typename TX, int NW>
static hipError_t launch_pass_m(int mode, bool pref, int grid, const PassArgs &a, hipStream_t s) {
  const int qw = pass_qw(sizeof(TV) == 8, NW, a.j);
  if (qw * NW * Vec<TV>::EPL < a.j) return hipErrorInvalidValue;  // tile narrower than the basis
  pref = pref && prefetch_fits<TV, NW>(qw);
  switch (mode) {
    case PM_INIT: return launch_pass_q<TV, TX, NW, PM_INIT, false>(1, grid, a, s);
    case PM_A:
      return pref ? launch_pass_q<TV, TX, NW, PM_A, true>(qw, grid, a, s)
                  : launch_pass_q<TV, TX, NW, PM_A, false>(qw, grid, a, s);
    case PM_B:
      return pref ? launch_pass_q<TV, TX, NW, PM_B, true>(qw, grid, a, s)
                  : launch_pass_q<TV, TX, NW, PM_B, false>(qw, grid, a, s);
    default:
      return pref ? launch_pass_q<TV, TX, NW, PM_C, true>(qw, grid, a, s)
                  : launch_pass_q<TV, TX, NW, PM_C, false>(qw, grid, a, s);
  }
}

// Wavefronts per row-pass workgroup.  An FP64 basis always uses 16.  For an
// FP32 basis nw_opt (4, 8 or 16) if set, else 4 up to 128 columns, 8 up to
// 320 and 16 beyond: at small basis sizes a panel carries little data and
// the pass is bound by the per-panel barrier and LDS round trips, which
// smaller, independent workgroups overlap better; above 320 columns 16
// wavefronts of 8 groups (128 VGPRs, 4 wavefronts per SIMD) beat 8 of 16
// groups (one workgroup of 8 per CU).  Between 257 and 320 columns the
// 8-group tile is half empty and the n = 1e8 run was 2.5% slower with it.
int pass_nw(bool tv_f64, int nw_opt, int j) {
  if (tv_f64) return 16;
  if (nw_opt == 4 && j > 256) return 8;  // 4 wavefronts cover at most 256 columns
  if (nw_opt > 0) return nw_opt;
  return j <= 128 ? 4 : (j <= 320 ? 8 : 16);
}

hipError_t launch_pass(int mode, bool tv_f64, bool tx_f64, bool prefetch, int nw, int grid,
                       const PassArgs &a, hipStream_t s) {
  if (tv_f64) {
    return tx_f64 ? launch_pass_m<double, double, 16>(mode, prefetch, grid, a, s)
                  : launch_pass_m<double, float, 16>(mode, prefetch, grid, a, s);
  }
  if (nw == 4)
    return tx_f64 ? launch_pass_m<float, double, 4>(mode, prefetch, grid, a, s)
                  : launch_pass_m<float, float, 4>(mode, prefetch, grid, a, s);
  if (nw == 8)
    return tx_f64 ? launch_pass_m<float, double, 8>(mode, prefetch, grid, a, s)
                  : launch_pass_m<float, float, 8>(mode, prefetch, grid, a, s);
  return tx_f64 ? launch_pass_m<float, double, 16>(mode, prefetch, grid, a, s)
                : launch_pass_m<float, float, 16>(mode, prefetch, grid, a, s);
}

// Resident workgroups per CU of the pass-A kernel for tile width qw (the
// widest register footprint of the three passes at that width).
template <typename TV, typename TX, int NW, int QW>
static int occ_q(bool pref) {
  int nb = 0;
  const void *f = pref ? reinterpret_cast<const void *>(&k_pass<TV, TX, NW, QW, PM_A, true>)
                       : reinterpret_cast<const void *>(&k_pass<TV, TX, NW, QW, PM_A, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, NW * 64, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <typename TV, typename TX, int NW>
static int occ_m(int qw, bool pref) {
  pref = pref && prefetch_fits<TV, NW>(qw);
  switch (qw) {
    case 1: return occ_q<TV, TX, NW, 1>(pref);
    case 2: return occ_q<TV, TX, NW, 2>(pref);
    case 4: return occ_q<TV, TX, NW, 4>(pref);
    case 8: return occ_q<TV, TX, NW, 8>(pref);
    case 6:
      if constexpr (sizeof(TV) == 4 && NW >= 8) return occ_q<TV, TX, NW, 6>(pref);
      return 1;
    case 12:
      if constexpr (sizeof(TV) == 4 && NW == 8) return occ_q<TV, TX, NW, 12>(pref);
      return 1;
    default:
      if constexpr (NW * 16 * Vec<TV>::EPL <= 512) return occ_q<TV, TX, NW, 16>(pref);
      return 1;
  }
}

int pass_occupancy(bool tv_f64, bool tx_f64, bool prefetch, int nw, int qw) {
  if (tv_f64) return tx_f64 ? occ_m<double, double, 16>(qw, prefetch) : occ_m<double, float, 16>(qw, prefetch);
  if (nw == 4) return tx_f64 ? occ_m<float, double, 4>(qw, prefetch) : occ_m<float, float, 4>(qw, prefetch);
  if (nw == 8) return tx_f64 ? occ_m<float, double, 8>(qw, prefetch) : occ_m<float, float, 8>(qw, prefetch);
  return tx_f64 ? occ_m<float, double, 16>(qw, prefetch) : occ_m<float, float, 16>(qw, prefetch);
}

hipError_t launch_reduce(int mode, const SmallArgs &a, hipStream_t s) {
  const int waves = a.j + (mode == 1 ? 1 : 0);
  const int blocks = (waves + 3) / 4;
  if (mode == 1)
    hipLaunchKernelGGL(k_reduce<1>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_reduce<2>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const SmallArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize_init(const SmallArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_init, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nextb(const SmallArgs &a, hipStream_t s) {
  // J = q after the push is at most j + 1 (host expectation).
  const int J = a.j + 1;
  const int blocks = (J + 63) / 64;
  hipLaunchKernelGGL(k_nextb, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_state(const SmallArgs &a, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(64), dim3(256), 0, s, a, tol);
  return hipGetLastError();
}

hipError_t launch_copy_basis(bool tv_f64, const void *W, const double *sigma, int64_t r0, int64_t nrows,
                             int n_max, int ncols, void *out, int64_t ld, bool out_f64, hipStream_t s) {
  if (ncols <= 0 || nrows <= 0) return hipSuccess;
  dim3 grid((unsigned)((nrows + 255) / 256), (unsigned)ncols);
  if (tv_f64) {
    if (out_f64)
      hipLaunchKernelGGL((k_copy_basis<double, double>), grid, dim3(256), 0, s, (const double *)W, sigma, r0,
                         nrows, n_max, ncols, (double *)out, ld);
    else
      hipLaunchKernelGGL((k_copy_basis<double, float>), grid, dim3(256), 0, s, (const double *)W, sigma, r0,
                         nrows, n_max, ncols, (float *)out, ld);
  } else {
    if (out_f64)
      hipLaunchKernelGGL((k_copy_basis<float, double>), grid, dim3(256), 0, s, (const float *)W, sigma, r0,
                         nrows, n_max, ncols, (double *)out, ld);
    else
      hipLaunchKernelGGL((k_copy_basis<float, float>), grid, dim3(256), 0, s, (const float *)W, sigma, r0,
                         nrows, n_max, ncols, (float *)out, ld);
  }
  return hipGetLastError();
}

}  // namespace foa
