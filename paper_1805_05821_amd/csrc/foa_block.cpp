// Blocked push (host side): foa_block_workspace_bytes, foa_push_blocked.
// The kernels and the method are described in foa_block.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "foa.h"
#include "foa_ctx.h"
#include "foa_internal.h"

using namespace foa;

namespace {

constexpr size_t kAlign = 256;
constexpr int kGramGrid = 1024;    // workgroups of the block Gram passes (partial slots)
constexpr int kBlockSlots = 1024;  // partial slots of the block passes (their largest grid)
constexpr int kNarrowCols = 128;   // FP32 basis sizes that take 4-wavefront block passes
constexpr int kWindowCols = 256;   // widest column window of an FP64-basis block pass

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct BlockLayout {
  size_t Z = 0, coef = 0, partb = 0, partg = 0, partq = 0, dnext = 0, sm = 0, flag = 0, gate = 0, total = 0;
};

BlockLayout block_layout(int64_t n, int n_max, int ldg) {
  BlockLayout B;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  const int64_t P = (n + PANEL - 1) / PANEL;
  B.Z = take((size_t)P * PANEL * BPK * 8);
  B.coef = take((size_t)n_max * BPK * 8);
  B.partb = take((size_t)n_max * BPK * ldg * 8);
  B.partg = take((size_t)kGramGrid * BPK * BPK * 8);
  B.partq = take((size_t)kGramGrid * BPK * BPK * 8);
  B.dnext = take((size_t)n_max * BPK * 8);
  B.sm = take((size_t)SM_TOTAL * 8);
  B.flag = take(sizeof(int));
  B.gate = take(sizeof(int));
  B.total = o;
  return B;
}

// All kernels of one block of BPK snapshots starting at basis size j.  xn:
// the next block's snapshots when it follows in the same run (its first
// projection over these j columns then rides on this block's last sweep);
// have_d: this block's V^T Y over its first j - BPK columns was formed so
// by the block before.
hipError_t enqueue_block(foa_ctx_s *c, const BlockLayout &L, char *bws, const void *x, int64_t ldx, bool x64,
                         int j, const void *xn, bool have_d) {
  const bool v64 = c->prec == FOA_PREC_F64;
  BlockArgs a{};
  a.W = c->W;
  a.x = x;
  a.ldx = ldx;
  a.Z = reinterpret_cast<double *>(bws + L.Z);
  a.coef = reinterpret_cast<double *>(bws + L.coef);
  a.partb = reinterpret_cast<double *>(bws + L.partb);
  a.partg = reinterpret_cast<double *>(bws + L.partg);
  a.partq = reinterpret_cast<double *>(bws + L.partq);
  a.dnext = reinterpret_cast<double *>(bws + L.dnext);
  a.qy = have_d ? 1 : 0;
  a.sm = reinterpret_cast<double *>(bws + L.sm);
  a.flag = reinterpret_cast<int *>(bws + L.flag);
  a.st = c->sa.st;
  a.H = c->sa.H;
  a.beta = c->sa.beta;
  a.sigma = c->sa.sigma;
  a.n = c->n;
  a.P = c->L.P;
  a.j = j;
  a.n_max = c->n_max;
  a.ldg = kBlockSlots;
  a.ldH = c->L.ldH;
  a.ldB = c->L.ldB;
  // FP32 basis up to 128 columns: 4-wavefront workgroups, four per CU (the
  // panels carry little data and the per-panel chain of barriers and LDS
  // round trips dominates; smaller independent workgroups overlap it)
  const bool narrow = !v64 && j <= kNarrowCols;
  const int nw = v64 ? 16 : (narrow ? 4 : 8);
  a.G = (int)std::min<int64_t>({(int64_t)kBlockSlots, c->L.P, (int64_t)(narrow ? 4 : 2) * c->cus});
  a.Gz = (int)std::min<int64_t>(kGramGrid, std::max<int64_t>(1, (c->L.P * PANEL + 255) / 256));
  // FP32 basis: a 12-group tile for 257-384 columns (the 16-group one is up to
  // a half empty there; the blocked run measured 4-7% faster) and a 14-group
  // one for 385-448 (the 16-group both-phase sweep spills)
  const int qw = narrow ? pick_qw(j, 16)
                        : ((!v64 && j > 256 && j <= 384) ? 12 : ((!v64 && j > 384 && j <= 448) ? 14 : pick_qw(j, 32)));
  hipStream_t s = c->stream;
  hipError_t e;
  // An FP64 basis above kWindowCols columns goes through the row passes in
  // column windows (the accumulators of a wider one do not fit a
  // workgroup's registers): the first window takes what the others, of
  // kWindowCols each, leave.  Column sums (D) of the windows are
  // independent.  Z = Y - W C goes window by window: Z = Y - W_0 C_0, then
  // Z -= W_i C_i, the last window forming its D = W_i^T Z in the same pass;
  // the other windows' D follow in passes of their own (with the narrow
  // window first, the widest one is read once).
  const int nwin = v64 ? (j + kWindowCols - 1) / kWindowCols : 1;
  auto window = [&](const BlockArgs &b, int i) {
    BlockArgs w = b;
    const int first = j - (nwin - 1) * kWindowCols;
    w.c0 = i == 0 ? 0 : first + (i - 1) * kWindowCols;
    w.j = i == 0 ? first : kWindowCols;
    return w;
  };
  auto bpass = [&](int mode, bool src64, const BlockArgs &b) -> hipError_t {
    if (nwin == 1) return launch_bpass(mode, v64, src64, nw, qw, b.G, b, s);
    hipError_t r = hipSuccess;
    for (int i = 0; i < nwin && r == hipSuccess; ++i) {
      const BlockArgs w = window(b, i);
      r = launch_bpass(mode, v64, src64, nw, pick_qw(w.j, 32), w.G, w, s);
    }
    return r;
  };
  auto bpass_z1 = [&](const BlockArgs &b) -> hipError_t {
    if (nwin == 1) return launch_bpass(1, v64, x64, nw, qw, b.G, b, s);
    BlockArgs w = window(b, 0);
    hipError_t r = launch_bpass(4, v64, x64, nw, pick_qw(w.j, 32), w.G, w, s);  // Z = Y - W_0 C_0
    for (int i = 1; i < nwin && r == hipSuccess; ++i) {
      w = window(b, i);                                                          // Z -= W_i C_i
      r = launch_bpass(i == nwin - 1 ? 5 : 2, v64, true, nw, pick_qw(w.j, 32), w.G, w, s);
    }
    for (int i = 0; i < nwin - 1 && r == hipSuccess; ++i) {
      w = window(b, i);                                                          // D_i = W_i^T Z
      r = launch_bpass(3, v64, true, nw, pick_qw(w.j, 32), w.G, w, s);
    }
    return r;
  };
  if (have_d) {
    if ((e = launch_zgram(3, v64, x64, a.Gz, a, s)) != hipSuccess) return e;        // ||y_k||^2, q^T y_k
  } else {
    if ((e = launch_zgram(0, v64, x64, a.Gz, a, s)) != hipSuccess) return e;        // ||y_k||^2
    if ((e = bpass(0, x64, a)) != hipSuccess) return e;                             // D = W^T Y
  }
  if ((e = launch_breduce(1, a, s)) != hipSuccess) return e;                         // R1, coef
  if ((e = bpass_z1(a)) != hipSuccess) return e;                                    // Z = Y - W C, D
  if ((e = launch_breduce(2, a, s)) != hipSuccess) return e;                         // R2, R += R2, coef
  if (xn) {
    BlockArgs r = a;
    r.xn = xn;
    if ((e = bpass(6, x64, r)) != hipSuccess) return e;                             // Z = Z - W C, D' = W^T Y'
    if ((e = launch_breduce(4, r, s)) != hipSuccess) return e;                       // D' -> dnext
  } else {
    if ((e = bpass(2, true, a)) != hipSuccess) return e;                            // Z = Z - W C
  }
  if ((e = launch_zgram(1, v64, x64, a.Gz, a, s)) != hipSuccess) return e;          // Z^T Z
  // third projection, where the test asks for it (the gated kernels return
  // at once otherwise)
  int *gate = reinterpret_cast<int *>(bws + L.gate);
  if ((e = launch_bthird(a, gate, v64 ? 0x1p-53 : 0x1p-24, s)) != hipSuccess) return e;
  BlockArgs g = a;
  g.gate = gate;
  if ((e = bpass(3, true, g)) != hipSuccess) return e;                              // D = W^T Z
  if ((e = launch_breduce(3, g, s)) != hipSuccess) return e;                         // R3, R += R3, coef
  if ((e = bpass(2, true, g)) != hipSuccess) return e;                              // Z = Z - W C
  if ((e = launch_zgram(1, v64, x64, g.Gz, g, s)) != hipSuccess) return e;          // Z^T Z
  // shifted CholeskyQR3: each Gram pass forms Z T_0 .. T_{t-1} row by row
  // from the unchanged Z, the last one writes Z T_0 T_1 T_2 into V
  BlockArgs q = a;
  if ((e = launch_bchol(0, a, s)) != hipSuccess) return e;                           // shifted: T_0
  q.tlev = 1;
  if ((e = launch_zgram(1, v64, x64, q.Gz, q, s)) != hipSuccess) return e;          // Gram of Z T_0
  if ((e = launch_bchol(1, a, s)) != hipSuccess) return e;                           // T_1
  q.tlev = 2;
  if ((e = launch_zgram(1, v64, x64, q.Gz, q, s)) != hipSuccess) return e;          // Gram of Z T_0 T_1
  if ((e = launch_bchol(2, a, s)) != hipSuccess) return e;                           // T_2
  q.tlev = 3;
  if ((e = launch_zgram(2, v64, x64, q.Gz, q, s)) != hipSuccess) return e;          // V <- Z T_0 T_1 T_2
  if ((e = launch_bcommit(a, s)) != hipSuccess) return e;
  SmallArgs sa = c->sa;
  sa.j = j + BPK;  // nextb sizes its grid from j + 1 and reads the committed q itself
  return launch_nextb(sa, s);
}

foa_status push_blocked_impl(foa_ctx_s *c, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype,
                             char *bws, const BlockLayout &L);

}  // namespace

extern "C" {

foa_status foa_block_workspace_bytes(int64_t n, int32_t n_max, foa_prec prec, size_t *bytes) {
  if (!bytes || n < 1 || n_max < 1 || n_max > FOA_MAX_CAPACITY ||
      (prec != FOA_PREC_F32 && prec != FOA_PREC_F64))
    return FOA_E_ARG;
  *bytes = block_layout(n, n_max, kBlockSlots).total;
  return FOA_OK;
}

foa_status foa_push_blocked(foa_ctx c, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype, void *d_bws,
                            size_t bws_bytes) {
  if (!c) return FOA_E_ARG;
  if (!d_X || (x_dtype != FOA_F32 && x_dtype != FOA_F64) || p < 0 || (p > 0 && ld < c->n) || !d_bws)
    return set_err(c, FOA_E_ARG, "bad blocked-push arguments");
  if (c->is_view) return set_err(c, FOA_E_STATE, "blocked pushes go to a single stream, not a batch view");
  const BlockLayout L = block_layout(c->n, c->n_max, kBlockSlots);
  if (bws_bytes < L.total || reinterpret_cast<uintptr_t>(d_bws) % kAlign)
    return set_err(c, FOA_E_NOMEM, "block workspace of %zu bytes needed", L.total);
  return push_blocked_impl(c, d_X, ld, p, x_dtype, static_cast<char *>(d_bws), L);
}

foa_status foa_push_blocked_static(foa_ctx c, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype) {
  if (!c) return FOA_E_ARG;
  if (!d_X || (x_dtype != FOA_F32 && x_dtype != FOA_F64) || p < 0 || (p > 0 && ld < c->n))
    return set_err(c, FOA_E_ARG, "bad blocked-push arguments");
  if (c->is_view) return set_err(c, FOA_E_STATE, "blocked pushes go to a single stream, not a batch view");
  const BlockLayout L = block_layout(c->n, c->n_max, kBlockSlots);
  if (L.total > FOA_BLOCK_STATIC_BYTES)
    return set_err(c, FOA_E_NOMEM,
                   "the static block workspace holds %zu bytes; this stream needs %zu (n or n_max too large)",
                   (size_t)FOA_BLOCK_STATIC_BYTES, L.total);
  char *bws = nullptr;
  const hipError_t e = block_static_scratch(c->device, &bws);
  if (e != hipSuccess || !bws) return hip_err(c, e != hipSuccess ? e : hipErrorUnknown, "static block workspace");
  return push_blocked_impl(c, d_X, ld, p, x_dtype, bws, L);
}

}  // extern "C"

namespace {

// Everything of a blocked push after argument checks; bws is the block
// workspace (the caller's, or the static one).
foa_status push_blocked_impl(foa_ctx_s *c, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype,
                             char *bws, const BlockLayout &L) {
  if (c->form == 1) return set_err(c, FOA_E_STATE, "the blocked form is not available on a one-reduction stream");
  foa_status r = sync_state(c);
  if (r != FOA_OK) return r;
  if (c->dev_status != ST_ACTIVE) return set_err(c, FOA_E_STATE, "stream is not active");
  if (c->q_host + p > c->n_max) return set_err(c, FOA_E_CAPACITY, "block exceeds capacity");
  const bool x64 = x_dtype == FOA_F64;
  const size_t es = x64 ? 8 : 4;
  const char *X = static_cast<const char *>(d_X);
  int *flag = reinterpret_cast<int *>(bws + L.flag);
  // the block passes address a block through one 32-bit buffer range
  const bool range_ok = (double)(BPK * ld + PANEL) * es < 4294967295.0;
  auto push_one = [&](int k) -> foa_status {
    foa_status rr = enqueue_push(c, X + (size_t)k * ld * es, x64);
    return rr;
  };
  int k = 0;
  if (p > 0 && c->q_host == 0) {
    if ((r = push_one(0)) != FOA_OK) return r;
    ++k;
    if ((r = sync_state(c)) != FOA_OK) return r;
  }
  // the part that does not fill whole blocks goes first, one snapshot at a
  // time, while the basis is smallest (a single push sweeps it three times)
  const int lead = (p - k) % BPK;
  if (lead > 0 && c->dev_status == ST_ACTIVE) {
    for (int i = 0; i < lead; ++i, ++k)
      if ((r = push_one(k)) != FOA_OK) return r;
    if ((r = sync_state(c)) != FOA_OK) return r;
  }
  while (k < p) {
    if (c->dev_status != ST_ACTIVE) break;
    // blocks that can go now: the whole ones
    int nblk = 0;
    while (k + (nblk + 1) * BPK <= p && range_ok) ++nblk;
    if (nblk == 0) {
      while (k < p) {
        if ((r = push_one(k)) != FOA_OK) return r;
        ++k;
      }
      break;
    }
    const int q0 = c->q_host;
    hipError_t e = launch_bflag_clear(flag, c->stream);
    for (int b = 0; b < nblk && e == hipSuccess; ++b)
      e = enqueue_block(c, L, bws, X + (size_t)(k + b * BPK) * ld * es, ld, x64, q0 + b * BPK,
                        b + 1 < nblk ? X + (size_t)(k + (b + 1) * BPK) * ld * es : nullptr, b > 0);
    if (e != hipSuccess) return hip_err(c, e, "blocked push");
    c->mirror_valid = false;
    c->dmd.valid = false;
    if ((r = sync_state(c)) != FOA_OK) return r;
    int rejected = 0;
    if (hipMemcpy(&rejected, flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return hip_err(c, hipErrorUnknown, "hipMemcpy block flag");
    const int done = (c->q_host - q0) / BPK;
    k += done * BPK;
    if (rejected && c->dev_status == ST_ACTIVE && k < p) {
      // the first block that did not go: its snapshots one at a time
      const int m = std::min(BPK, p - k);
      for (int i = 0; i < m; ++i) {
        if ((r = push_one(k)) != FOA_OK) return r;
        ++k;
      }
      if ((r = sync_state(c)) != FOA_OK) return r;
    }
  }
  // snapshots offered after the stream stopped are ignored by the device (and
  // counted as offered), as in foa_push_block
  for (; k < p; ++k)
    if ((r = push_one(k)) != FOA_OK) return r;
  return sync_state(c);
}


}  // namespace

