// Host side of the C ABI declared in include/foa.h: workspace layout,
// argument validation, the per-push kernel sequence, status readback and the
// host FP64 post-processing (truncation, eigenpairs, indicators, modes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "foa.h"
#include "foa_ctx.h"
#include "foa_internal.h"


using foa::DevState;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxGrid = foa::kStreamSlots;  // leading dimension of the partial-sum arrays

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool valid_prec(int p) { return p == FOA_PREC_F64 || p == FOA_PREC_F32; }
bool valid_dtype(int d) { return d == FOA_F32 || d == FOA_F64; }

}  // namespace

namespace foa {

Layout make_layout(int64_t n, int n_max, foa_prec prec, int ldg) {
  Layout L{};
  const int64_t P = (n + PANEL - 1) / PANEL;
  const size_t sV = prec == FOA_PREC_F64 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.P = P;
  L.n_pad = P * PANEL;
  L.ldg = ldg;
  L.ldH = n_max + 1;
  L.ldB = n_max + 1;
  L.W = take((size_t)P * PANEL * (size_t)n_max * sV);
  L.w = take((size_t)L.n_pad * 8);
  L.part = take((size_t)n_max * L.ldg * 8);
  L.partn = take((size_t)L.ldg * 8);
  L.H = take((size_t)L.ldH * (n_max + 1) * 8);
  L.beta = take((size_t)L.ldB * (n_max + 1) * 8);
  const size_t vec = (size_t)(n_max + 1) * 8;
  L.sigma = take(vec);
  L.bvec = take(vec);
  L.h = take(vec);
  L.s = take(vec);
  L.coefA = take(vec);
  L.coefB = take(vec);
  L.coefC = take(vec);
  L.st = take(sizeof(DevState));
  // mode coefficients: FP64 k x r, or the padded FP32 layout of the MFMA path
  L.mcoef = take(std::max((size_t)n_max * n_max * 8, (size_t)modes_kpad(n_max) * modes_rpad(n_max) * 4));
  // one-reduction form: second partial-sum array (with the scalar rows), the
  // reduced sums and the prefix sums of the snapshot norms; with an FP32
  // basis also the partial sums of the finished column's rounding error, the
  // Gram deviation E of the final columns and the corrected coefficients
  L.ls_part1 = take((size_t)(n_max + LS_NSC) * L.ldg * 8);
  L.ls_red = take((size_t)(3 * n_max + LS_NSC) * 8);
  L.ls_xpre = take((size_t)(n_max + 1) * 8);
  L.ls_what = take((size_t)(n_max + 1) * 8);
  if (prec == FOA_PREC_F32) {
    L.ls_part2 = take((size_t)n_max * L.ldg * 8);
    L.ls_E = take((size_t)n_max * n_max * 8);
  }
  L.total = off;
  return L;
}

void bind_pointers(foa_ctx_s *c) {
  const Layout &L = c->L;
  char *b = static_cast<char *>(c->ws);
  c->W = b + L.W;
  c->w = reinterpret_cast<double *>(b + L.w);
  c->part = reinterpret_cast<double *>(b + L.part);
  c->partn = reinterpret_cast<double *>(b + L.partn);
  SmallArgs &s = c->sa;
  s.st = reinterpret_cast<DevState *>(b + L.st);
  s.H = reinterpret_cast<double *>(b + L.H);
  s.beta = reinterpret_cast<double *>(b + L.beta);
  s.sigma = reinterpret_cast<double *>(b + L.sigma);
  s.bvec = reinterpret_cast<double *>(b + L.bvec);
  s.h = reinterpret_cast<double *>(b + L.h);
  s.s = reinterpret_cast<double *>(b + L.s);
  s.coefA = reinterpret_cast<double *>(b + L.coefA);
  s.coefB = reinterpret_cast<double *>(b + L.coefB);
  s.coefC = reinterpret_cast<double *>(b + L.coefC);
  s.part = c->part;
  s.partn = c->partn;
  s.ldH = L.ldH;
  s.ldB = L.ldB;
  s.n_max = c->n_max;
  s.ldg = L.ldg;
}

foa_status set_err(foa_ctx_s *c, foa_status st, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return st;
}

foa_status hip_err(foa_ctx_s *c, hipError_t e, const char *where) {
  if (e == hipSuccess) return FOA_OK;
  return set_err(c, FOA_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

foa_status map_status(int s) {
  switch (s) {
    case ST_ACTIVE: return FOA_OK;
    case ST_INVARIANT: return FOA_INVARIANT;
    case ST_NONFINITE: return FOA_E_NONFINITE;
    case ST_ZERO: return FOA_E_ZERO;
    default: return FOA_E_DEVICE;
  }
}

// Row-pass grid of a push at basis size j: the "grid" option if set, else
// one full complement of resident workgroups for the pass kernel at this tile
// width (at least grid_auto); bounded by the partial-sum slots and the panels.
int pass_grid(foa_ctx_s *c, int j, bool x_f64) {
  int g = c->grid_opt;
  if (g <= 0) {
    const bool v64 = c->prec == FOA_PREC_F64;
    const int nw = pass_nw(v64, c->nw, j);
    const int qw = pass_qw(v64, nw, j);
    const int qi = tile_slot(qw);
    const int ni = nw == 4 ? 0 : (nw == 8 ? 1 : 2);
    int &occ = c->occ_cache[x_f64 ? 1 : 0][ni][qi];
    if (occ <= 0) occ = pass_occupancy(v64, x_f64, c->prefetch, nw, qw);
    g = std::max(c->grid_auto, occ * c->cus);
  }
  if (g > kMaxGrid) g = kMaxGrid;
  if ((int64_t)g > c->L.P) g = (int)c->L.P;
  return g < 1 ? 1 : g;
}

hipEvent_t take_event(foa_ctx_s *c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one row pass, bracketed by timing events when profiling is on.
static hipError_t timed_pass(foa_ctx_s *c, int mode, bool v64, bool x64, bool pref, int G,
                             const PassArgs &pa, double alg_bytes) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, c->stream);
  }
  hipError_t e = launch_pass(mode, v64, x64, pref, pass_nw(v64, c->nw, pa.j), G, pa, c->stream);
  if (c->profile && e0 && e1) {
    (void)hipEventRecord(e1, c->stream);
    c->ev_pending.push_back({e0, e1, alg_bytes, 0});
  }
  return e;
}

foa_status collect_profile(foa_ctx_s *c) {
  for (auto &p : c->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      if (p.kind == 0) {
        c->prof_launches += 1;
        c->prof_ms += ms;
        c->prof_bytes += p.work;
      } else {
        c->prof_gemm_launches += 1;
        c->prof_gemm_ms += ms;
        c->prof_gemm_flops += p.work;
      }
    }
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.b);
  }
  c->ev_pending.clear();
  return FOA_OK;
}

void release_events(foa_ctx_s *c) {
  for (auto &p : c->ev_pending) {
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.b);
  }
  c->ev_pending.clear();
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  c->ev_free.clear();
}

// Enqueue one push of snapshot x (Algorithm 1: the first-snapshot
// normalisation for q = 0, else one iteration of its snapshot loop).
foa_status enqueue_push(foa_ctx_s *c, const void *x, bool x_f64) {
  if (c->form == 1) return enqueue_ls_push(c, x, x_f64);
  const bool v64 = c->prec == FOA_PREC_F64;
  const int j = c->q_host;
  const int G = pass_grid(c, j, x_f64);
  PassArgs pa{};
  pa.W = c->W;
  pa.x = x;
  pa.w = c->w;
  pa.coef[0] = c->sa.coefA;
  pa.coef[1] = c->sa.coefB;
  pa.coef[2] = c->sa.coefC;
  pa.st = c->sa.st;
  pa.part = c->part;
  pa.partn = c->partn;
  pa.n = c->n;
  pa.P = c->L.P;
  pa.j = j;
  pa.n_max = c->n_max;
  pa.ldg = c->L.ldg;
  SmallArgs sa = c->sa;
  sa.G = G;
  sa.j = j;
  hipStream_t s = c->stream;
  hipError_t e;
  const double nv = (double)c->n, sV = v64 ? 8.0 : 4.0, sX = x_f64 ? 8.0 : 4.0;
  const double vbytes = nv * j * sV;  // the j basis columns, read once per pass
  if (j == 0) {
    if ((e = timed_pass(c, PM_INIT, v64, x_f64, false, G, pa, nv * (sX + sV))) != hipSuccess)
      return hip_err(c, e, "pass init");
    if ((e = launch_finalize_init(sa, s)) != hipSuccess) return hip_err(c, e, "finalize init");
  } else {
    if ((e = timed_pass(c, PM_A, v64, x_f64, c->prefetch, G, pa, vbytes + nv * sX)) != hipSuccess)
      return hip_err(c, e, "pass A");
    if ((e = launch_reduce(1, sa, s)) != hipSuccess) return hip_err(c, e, "reduce A");
    if ((e = timed_pass(c, PM_B, v64, x_f64, c->prefetch, G, pa, vbytes)) != hipSuccess)
      return hip_err(c, e, "pass B");
    if ((e = launch_reduce(2, sa, s)) != hipSuccess) return hip_err(c, e, "reduce B");
    if ((e = timed_pass(c, PM_C, v64, x_f64, c->prefetch, G, pa, vbytes + nv * sV)) != hipSuccess)
      return hip_err(c, e, "pass C");
    if ((e = launch_finalize(sa, s)) != hipSuccess) return hip_err(c, e, "finalize");
  }
  if ((e = launch_nextb(sa, s)) != hipSuccess) return hip_err(c, e, "next b");
  c->q_host = j + 1;
  c->mirror_valid = false;
  c->dmd.valid = false;
  return FOA_OK;
}

// Synchronise and read the device scalar state (the one-reduction form first
// finishes its pending columns).
foa_status sync_state(foa_ctx_s *c) {
  if (c->form == 1 && (c->ls_hu || c->ls_hx)) {
    foa_status r = enqueue_ls_flush(c);
    if (r != FOA_OK) return r;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
  DevState st;
  e = hipMemcpy(&st, c->sa.st, sizeof st, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_err(c, e, "hipMemcpy state");
  c->q_host = st.q;
  c->dev_status = st.status;
  c->pushes = st.pushes;
  collect_profile(c);
  return FOA_OK;
}

int projected_order(const foa_ctx_s *c) {
  if (c->q_host == 0) return 0;
  return c->dev_status == ST_INVARIANT ? c->q_host : c->q_host - 1;
}

// Synchronise and copy H_bar, beta and sigma of the used extent to the host.
foa_status refresh_mirror(foa_ctx_s *c) {
  foa_status r = sync_state(c);
  if (r != FOA_OK) return r;
  if (c->mirror_valid) return FOA_OK;
  const int q = c->q_host;
  const int cols = std::min(q + 1, c->n_max);
  c->hH.assign((size_t)c->L.ldH * cols, 0.0);
  c->hB.assign((size_t)c->L.ldB * cols, 0.0);
  c->hsigma.assign((size_t)c->n_max + 1, 0.0);
  if (cols > 0) {
    hipError_t e = hipMemcpy(c->hH.data(), c->sa.H, c->hH.size() * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(c->hB.data(), c->sa.beta, c->hB.size() * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(c->hsigma.data(), c->sa.sigma, c->hsigma.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(c, e, "hipMemcpy mirror");
  }
  c->mirror_valid = true;
  return FOA_OK;
}

foa_status reset_device_state(foa_ctx_s *c) {
  hipError_t e = launch_init_state(c->sa, c->tol, c->stream);
  if (e != hipSuccess) return hip_err(c, e, "init state");
  c->q_host = 0;
  c->dev_status = ST_ACTIVE;
  c->pushes = 0;
  c->ls_hu = c->ls_hx = 0;
  c->mirror_valid = false;
  c->trunc_r = 0;
  c->trunc_m = 0;
  c->Ur.clear();
  c->dmd.valid = false;
  return FOA_OK;
}

}  // namespace foa

using namespace foa;

extern "C" {

const char *foa_status_str(foa_status s) {
  switch (s) {
    case FOA_OK: return "ok";
    case FOA_INVARIANT: return "invariant subspace reached (dependent snapshot)";
    case FOA_E_ARG: return "invalid argument";
    case FOA_E_CAPACITY: return "snapshot capacity exceeded";
    case FOA_E_STATE: return "call not valid in this state";
    case FOA_E_NONFINITE: return "non-finite snapshot";
    case FOA_E_DEVICE: return "HIP runtime error";
    case FOA_E_NOMEM: return "workspace or host memory too small";
    case FOA_E_NUMERIC: return "host eigen/SVD iteration did not converge";
    case FOA_E_ZERO: return "first snapshot has zero norm";
  }
  return "unknown status";
}

const char *foa_last_error(foa_ctx ctx) { return ctx ? ctx->err.c_str() : ""; }

foa_status foa_workspace_bytes(int64_t n, int32_t n_max, foa_prec prec, size_t *bytes) {
  if (!bytes || n < 1 || n_max < 1 || n_max > FOA_MAX_CAPACITY || !valid_prec(prec)) return FOA_E_ARG;
  *bytes = make_layout(n, n_max, prec).total;
  return FOA_OK;
}

foa_status foa_init(foa_ctx *out, int64_t n, int32_t n_max, foa_prec prec, void *d_workspace,
                    size_t ws_bytes, void *hip_stream, double breakdown_tol) {
  if (!out) return FOA_E_ARG;
  *out = nullptr;
  if (n < 1 || n_max < 1 || n_max > FOA_MAX_CAPACITY || !valid_prec(prec) || !d_workspace) return FOA_E_ARG;
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return FOA_E_ARG;
  if (std::isnan(breakdown_tol)) return FOA_E_ARG;
  const Layout L = make_layout(n, n_max, prec);
  if (ws_bytes < L.total) return FOA_E_NOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FOA_E_DEVICE;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return FOA_E_DEVICE;
  foa_ctx_s *c = new (std::nothrow) foa_ctx_s();
  if (!c) return FOA_E_NOMEM;
  c->n = n;
  c->n_max = n_max;
  c->prec = prec;
  c->ws = d_workspace;
  c->ws_bytes = ws_bytes;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->L = L;
  c->device = dev;
  {
    // set-up of foa_push_blocked_static on this device (once per device); an
    // error is kept and reported by that entry point, not here
    char *scratch_addr = nullptr;
    (void)block_static_scratch(dev, &scratch_addr);
  }
  c->cus = cus;
  c->grid_auto = 2 * cus;
  c->prefetch = true;  // register double buffering wherever the tile fits
  c->nw = 0;           // FP32 basis: wavefronts per row-pass workgroup chosen per basis size
  c->tol = breakdown_tol < 0 ? (double)n_max * std::ldexp(1.0, -52) : breakdown_tol;
  bind_pointers(c);
  foa_status r = reset_device_state(c);
  if (r != FOA_OK) {
    delete c;
    return r;
  }
  *out = c;
  return FOA_OK;
}

foa_status foa_set_option(foa_ctx c, const char *key, int64_t value) {
  if (!c || !key) return FOA_E_ARG;
  if (!std::strcmp(key, "grid")) {
    if (value < 0 || value > kMaxGrid) return set_err(c, FOA_E_ARG, "grid must be in [0, %d]", kMaxGrid);
    c->grid_opt = (int)value;
    return FOA_OK;
  }
  if (!std::strcmp(key, "prefetch")) {
    c->prefetch = value != 0;
    std::memset(c->occ_cache, 0, sizeof c->occ_cache);
    return FOA_OK;
  }
  if (!std::strcmp(key, "nw")) {
    if (value != 0 && value != 4 && value != 8 && value != 16)
      return set_err(c, FOA_E_ARG, "nw must be 0 (automatic), 4, 8 or 16");
    c->nw = (int)value;
    std::memset(c->occ_cache, 0, sizeof c->occ_cache);
    return FOA_OK;
  }
  if (!std::strcmp(key, "ls_nw")) {
    if (value != 0 && value != 8 && value != 16) return set_err(c, FOA_E_ARG, "ls_nw must be 0, 8 or 16");
    c->ls_nw_opt = (int)value;
    std::memset(c->ls_occ, 0, sizeof c->ls_occ);
    return FOA_OK;
  }
  if (!std::strcmp(key, "profile")) {
    c->profile = value != 0;
    return FOA_OK;
  }
  return set_err(c, FOA_E_ARG, "unknown option '%s'", key);
}

static foa_status push_checks(foa_ctx c) {
  if (c->is_view) return set_err(c, FOA_E_STATE, "pushes to a batch stream go through foa_batch_push");
  if (c->dev_status != ST_ACTIVE)
    return set_err(c, FOA_E_STATE, "stream is no longer active (%s)", foa_status_str(map_status(c->dev_status)));
  if (c->q_host >= c->n_max) return set_err(c, FOA_E_CAPACITY, "capacity %d reached", c->n_max);
  return FOA_OK;
}

foa_status foa_push_snapshot(foa_ctx c, const void *d_x, foa_dtype x_dtype) {
  if (!c) return FOA_E_ARG;
  if (!d_x || !valid_dtype(x_dtype)) return set_err(c, FOA_E_ARG, "null snapshot or bad dtype");
  foa_status r = push_checks(c);
  if (r != FOA_OK) return r;
  return enqueue_push(c, d_x, x_dtype == FOA_F64);
}

foa_status foa_push_block(foa_ctx c, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype) {
  if (!c) return FOA_E_ARG;
  if (!d_X || !valid_dtype(x_dtype) || p < 0 || (p > 0 && ld < c->n))
    return set_err(c, FOA_E_ARG, "bad block arguments");
  const size_t es = x_dtype == FOA_F64 ? 8 : 4;
  if (c->q_host + p > c->n_max) return set_err(c, FOA_E_CAPACITY, "block exceeds capacity");
  for (int k = 0; k < p; ++k) {
    foa_status r = push_checks(c);
    if (r != FOA_OK) return r;
    r = enqueue_push(c, static_cast<const char *>(d_X) + (size_t)k * ld * es, x_dtype == FOA_F64);
    if (r != FOA_OK) return r;
  }
  return FOA_OK;
}

foa_status foa_sync(foa_ctx c, int32_t *q) {
  if (!c) return FOA_E_ARG;
  foa_status r = sync_state(c);
  if (r != FOA_OK) return r;
  if (q) *q = c->q_host;
  return map_status(c->dev_status);
}

foa_status foa_get_state(foa_ctx c, double *h_Hbar, double *h_beta, int32_t ld, int32_t *q, int32_t *m_out) {
  if (!c) return FOA_E_ARG;
  foa_status r = refresh_mirror(c);
  if (r != FOA_OK) return r;
  const int qq = c->q_host;
  const int m = projected_order(c);
  if ((h_Hbar || h_beta) && ld < qq + 1) return set_err(c, FOA_E_ARG, "ld must be >= q+1 = %d", qq + 1);
  if (h_Hbar) {
    for (int col = 0; col < m; ++col)
      for (int row = 0; row <= qq && row <= col + 1; ++row)
        h_Hbar[(size_t)col * ld + row] = c->hH[(size_t)col * c->L.ldH + row];
  }
  if (h_beta) {
    const int bcols = (c->dev_status == ST_INVARIANT) ? qq + 1 : qq;
    for (int col = 0; col < bcols && col < c->n_max; ++col)
      for (int row = 0; row <= col && row <= qq; ++row)
        h_beta[(size_t)col * ld + row] = c->hB[(size_t)col * c->L.ldB + row];
  }
  if (q) *q = qq;
  if (m_out) *m_out = m;
  return FOA_OK;
}

foa_status foa_copy_basis(foa_ctx c, void *d_V, int64_t ld, foa_dtype dtype, int32_t ncols) {
  if (!c) return FOA_E_ARG;
  if (!d_V || !valid_dtype(dtype) || ld < c->n || ncols < 0 || ncols > c->q_host)
    return set_err(c, FOA_E_ARG, "bad basis copy arguments (ncols %d, q %d)", ncols, c->q_host);
  hipError_t e = launch_copy_basis(c->prec == FOA_PREC_F64, c->W, c->sa.sigma, 0, c->n, c->n_max, ncols, d_V,
                                   ld, dtype == FOA_F64, c->stream);
  return hip_err(c, e, "copy basis");
}

foa_status foa_copy_basis_rows(foa_ctx c, int64_t r0, int64_t nrows, void *d_V, int64_t ld, foa_dtype dtype,
                               int32_t ncols) {
  if (!c) return FOA_E_ARG;
  if (!d_V || !valid_dtype(dtype) || r0 < 0 || nrows < 0 || r0 + nrows > c->n || ld < nrows || ncols < 0 ||
      ncols > c->q_host)
    return set_err(c, FOA_E_ARG, "bad basis row-copy arguments");
  hipError_t e = launch_copy_basis(c->prec == FOA_PREC_F64, c->W, c->sa.sigma, r0, nrows, c->n_max, ncols, d_V,
                                   ld, dtype == FOA_F64, c->stream);
  return hip_err(c, e, "copy basis rows");
}

foa_status foa_profile(foa_ctx c, double out[3]) {
  if (!c || !out) return FOA_E_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
  collect_profile(c);
  out[0] = c->prof_launches;
  out[1] = c->prof_ms;
  out[2] = c->prof_bytes;
  c->prof_launches = c->prof_ms = c->prof_bytes = 0;
  return FOA_OK;
}

foa_status foa_next_column(foa_ctx c, void **d_col) {
  if (!c || !d_col) return FOA_E_ARG;
  if (c->form == 1) return set_err(c, FOA_E_STATE, "the one-reduction form has no in-place snapshot buffer");
  *d_col = c->w;
  return FOA_OK;
}

foa_status foa_set_form(foa_ctx c, foa_form form) {
  if (!c) return FOA_E_ARG;
  if (form != FOA_FORM_CGS2 && form != FOA_FORM_ONE_REDUCTION) return set_err(c, FOA_E_ARG, "unknown form");
  if (c->is_view) return set_err(c, FOA_E_STATE, "batch streams use the three-sweep form");
  if (c->q_host != 0 || c->pushes != 0 || c->ls_hu || c->ls_hx)
    return set_err(c, FOA_E_STATE, "the form is chosen before the first push (after foa_init or foa_reset)");
  if (form == FOA_FORM_ONE_REDUCTION && !ls_supported(c->prec == FOA_PREC_F64, c->n_max - 1))
    return set_err(c, FOA_E_ARG, "the one-reduction form holds at most %d snapshots with this basis precision",
                   c->prec == FOA_PREC_F64 ? 257 : 513);
  c->form = form == FOA_FORM_ONE_REDUCTION ? 1 : 0;
  return FOA_OK;
}

foa_status foa_flush(foa_ctx c) {
  if (!c) return FOA_E_ARG;
  if (c->form != 1 || (!c->ls_hu && !c->ls_hx)) return FOA_OK;
  return enqueue_ls_flush(c);
}

foa_status foa_profile_modes(foa_ctx c, double out[3]) {
  if (!c || !out) return FOA_E_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
  collect_profile(c);
  out[0] = c->prof_gemm_launches;
  out[1] = c->prof_gemm_ms;
  out[2] = c->prof_gemm_flops;
  c->prof_gemm_launches = c->prof_gemm_ms = c->prof_gemm_flops = 0;
  return FOA_OK;
}

foa_status foa_reset(foa_ctx c) {
  if (!c) return FOA_E_ARG;
  if (c->is_view) return set_err(c, FOA_E_STATE, "reset a batch through the batch");
  return reset_device_state(c);
}

foa_status foa_destroy(foa_ctx c) {
  if (!c) return FOA_E_ARG;
  if (c->is_view) return set_err(c, FOA_E_STATE, "views are owned by their batch");
  (void)hipStreamSynchronize(c->stream);
  release_events(c);
  delete c;
  return FOA_OK;
}

}  // extern "C"
