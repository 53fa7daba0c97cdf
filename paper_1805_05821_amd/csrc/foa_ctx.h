// Host-side context of one FOA stream (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdarg>
#include <string>
#include <vector>

#include "foa.h"
#include "foa_internal.h"

namespace foa {

// Byte offsets of the pieces of one stream's device workspace.
struct Layout {
  int64_t P = 0, n_pad = 0;
  int ldg = 0, ldH = 0, ldB = 0;
  size_t W = 0, w = 0, part = 0, partn = 0, H = 0, beta = 0, sigma = 0, bvec = 0, h = 0, s = 0;
  size_t coefA = 0, coefB = 0, coefC = 0, st = 0, mcoef = 0;
  size_t ls_part1 = 0, ls_red = 0, ls_xpre = 0;  // one-reduction form
  size_t ls_part2 = 0, ls_E = 0, ls_what = 0;     // one-reduction form, FP32 basis
  size_t total = 0;
};

// Eigen-decomposition of the projected matrix and everything derived from it
// (cached until the next push, reset or truncation change).
struct DmdCache {
  bool valid = false;
  int m = 0;        // order of H_m
  int r = 0;        // truncation rank (0: untruncated)
  int k = 0;        // order of the eigenproblem (m or r)
  std::vector<std::complex<double>> lam;   // k eigenvalues
  std::vector<std::complex<double>> B;     // m x k: mode coefficients in the V_{1:m} basis
  std::vector<std::complex<double>> coef;  // k coefficients of psi_1
  std::vector<double> ind;                 // k error indicators
  std::vector<int> is_real;                // k
  std::vector<int> entries;                // eigen indices, one per real / pair, in mode order
};

// ldg: leading dimension (slots) of the partial-sum arrays.
Layout make_layout(int64_t n, int n_max, foa_prec prec, int ldg = kStreamSlots);

}  // namespace foa

struct foa_ctx_s {
  int64_t n = 0;
  int n_max = 0;
  foa_prec prec = FOA_PREC_F64;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0, cus = 0;
  foa::Layout L;
  // device pointers (inside ws)
  void *W = nullptr;
  double *w = nullptr, *part = nullptr, *partn = nullptr;
  foa::SmallArgs sa{};
  // launch configuration
  int grid_auto = 0, grid_opt = 0;
  int occ_cache[2][3][7] = {};  // resident pass-A workgroups per CU [x_f64][nw 4/8/16][tile_slot]
  bool prefetch = false;
  int nw = 16;  // wavefronts per row-pass workgroup (FP32 basis: 8 or 16)
  double tol = 0.0;
  // host view of the state
  int q_host = 0;     // expected q (exact after a synchronising call)
  int dev_status = 0; // device status at the last synchronising call
  int pushes = 0;
  bool is_view = false;
  bool mirror_valid = false;
  std::vector<double> hH, hB, hsigma;
  // truncation (foa_truncate)
  int trunc_r = 0;
  int trunc_m = 0;            // m the truncation was computed for
  foa::DmdCache dmd;
  std::vector<double> Ur;     // m x r, column-major
  std::vector<double> hsv;    // singular values of beta_m
  std::string err;
  // one-reduction form (foa_set_form): 0 = three-sweep CGS2, 1 = one reduction;
  // the host's model of the pending columns (exact unless the device found a
  // dependent or non-finite snapshot, which the next synchronising call reads)
  int form = 0;
  int ls_hu = 0, ls_hx = 0;
  int ls_occ[2][2][3][7] = {};  // resident sweep workgroups per CU [v64][x64][nw][tile_slot]
  int ls_nw_opt = 0;            // option "ls_nw": 0 automatic, 16 = 16-wavefront sweeps above 128 columns
  // row-pass timing (foa_profile)
  bool profile = false;
  // kind 0: row pass (work = algorithmic bytes); kind 1: mode GEMM (work = flops)
  struct EvPair { hipEvent_t a, b; double work; int kind; };
  std::vector<EvPair> ev_pending;
  std::vector<hipEvent_t> ev_free;
  double prof_launches = 0, prof_ms = 0, prof_bytes = 0;
  double prof_gemm_launches = 0, prof_gemm_ms = 0, prof_gemm_flops = 0;
};

namespace foa {

void bind_pointers(foa_ctx_s *c);
foa_status set_err(foa_ctx_s *c, foa_status st, const char *fmt, ...);
foa_status hip_err(foa_ctx_s *c, hipError_t e, const char *where);
foa_status map_status(int s);
foa_status sync_state(foa_ctx_s *c);
foa_status refresh_mirror(foa_ctx_s *c);
foa_status reset_device_state(foa_ctx_s *c);
foa_status enqueue_push(foa_ctx_s *c, const void *x, bool x_f64);
// one-reduction form (foa_lowsync.cpp)
foa_status enqueue_ls_push(foa_ctx_s *c, const void *x, bool x_f64);
foa_status enqueue_ls_flush(foa_ctx_s *c);
int projected_order(const foa_ctx_s *c);
int pass_grid(foa_ctx_s *c, int j, bool x_f64);
foa_status collect_profile(foa_ctx_s *c);
void release_events(foa_ctx_s *c);
hipEvent_t take_event(foa_ctx_s *c);

}  // namespace foa
