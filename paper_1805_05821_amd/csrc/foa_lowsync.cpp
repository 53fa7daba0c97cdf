// Host side of the one-reduction form (foa_set_form with
// FOA_FORM_ONE_REDUCTION): the per-push kernel sequence -- one sweep over the
// rows, one fixed-order reduction, one finalize -- and the flush that
// finishes the pending columns.  The method and the kernels are described
// in foa_lowsync.hip.
//
// The host keeps a model of the pending columns (a column under its second
// projection, a snapshot copy awaiting its first) to pick the sweep's tile
// width and the number of flush sweeps.  The model is exact while the
// stream is active; when the device finds a dependent or non-finite
// snapshot, later kernels see the device status and leave the state alone,
// and the next synchronising call reads the device's q and status.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "foa.h"
#include "foa_ctx.h"
#include "foa_internal.h"

namespace foa {

namespace {

LsSmall ls_small(foa_ctx_s *c, int G, bool flush) {
  char *b = static_cast<char *>(c->ws);
  LsSmall a{};
  a.st = c->sa.st;
  a.H = c->sa.H;
  a.beta = c->sa.beta;
  a.sigma = c->sa.sigma;
  a.w = c->sa.h;
  a.z = c->sa.s;
  a.coefW = c->sa.coefA;
  a.coefZ = c->sa.coefB;
  a.red = reinterpret_cast<double *>(b + c->L.ls_red);
  a.bvec = c->sa.bvec;
  a.xpre = reinterpret_cast<double *>(b + c->L.ls_xpre);
  a.part0 = c->part;
  a.part1 = reinterpret_cast<double *>(b + c->L.ls_part1);
  a.what = reinterpret_cast<double *>(b + c->L.ls_what);
  if (c->prec == FOA_PREC_F32) {
    a.gram = 1;
    a.part2 = reinterpret_cast<double *>(b + c->L.ls_part2);
    a.E = reinterpret_cast<double *>(b + c->L.ls_E);
  }
  a.ldH = c->L.ldH;
  a.ldB = c->L.ldB;
  a.n_max = c->n_max;
  a.ldg = c->L.ldg;
  a.G = G;
  a.nt = c->q_host;
  a.flush = flush ? 1 : 0;
  return a;
}

// Workgroups of the sweep: every workgroup the kernel of this tile width
// keeps resident (at least two per CU), bounded by the partial-sum slots and
// the panels; the "grid" option overrides.
int ls_grid(foa_ctx_s *c, int q, bool x64) {
  int g = c->grid_opt;
  if (g <= 0) {
    const bool v64 = c->prec == FOA_PREC_F64;
    const int nw = ls_nw(v64, q, c->ls_nw_opt), qw = ls_qw(v64, q, c->ls_nw_opt);
    const int qi = tile_slot(qw);
    const int ni = nw == 4 ? 0 : (nw == 8 ? 1 : 2);
    int &occ = c->ls_occ[v64 ? 1 : 0][x64 ? 1 : 0][ni][qi];
    if (occ <= 0) occ = ls_occupancy(v64, x64, q, c->ls_nw_opt);
    g = std::max(c->grid_auto, occ * c->cus);
  }
  g = std::min<int64_t>({(int64_t)g, (int64_t)c->L.ldg, c->L.P});
  return g < 1 ? 1 : g;
}

// One sweep + reduction + finalize; x == nullptr: a flush sweep.
foa_status enqueue_ls_sweep(foa_ctx_s *c, const void *x, bool x64) {
  const bool v64 = c->prec == FOA_PREC_F64;
  const bool flush = x == nullptr;
  const int q = c->q_host;
  if (!ls_supported(v64, q)) return set_err(c, FOA_E_STATE, "basis too wide for the one-reduction sweep");
  const int G = ls_grid(c, q, x64);
  LsArgs a{};
  a.W = c->W;
  a.x = x;
  a.coefW = c->sa.coefA;
  a.coefZ = c->sa.coefB;
  a.st = c->sa.st;
  a.part0 = c->part;
  a.part1 = reinterpret_cast<double *>(static_cast<char *>(c->ws) + c->L.ls_part1);
  if (c->prec == FOA_PREC_F32) a.part2 = reinterpret_cast<double *>(static_cast<char *>(c->ws) + c->L.ls_part2);
  a.n = c->n;
  a.P = c->L.P;
  a.n_max = c->n_max;
  a.ldg = c->L.ldg;
  a.flush = flush ? 1 : 0;
  const LsSmall sm = ls_small(c, G, flush);
  hipStream_t s = c->stream;
  // algorithmic bytes: the q final columns once, the pending columns read and
  // written, the new snapshot read and stored
  const double nv = (double)c->n, sV = v64 ? 8.0 : 4.0, sX = x64 ? 8.0 : 4.0;
  const int pend = c->ls_hu + c->ls_hx, nn = flush ? 0 : 1;
  const double bytes = nv * (q * sV + pend * sV + (pend + nn) * sV + nn * sX);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, s);
  }
  hipError_t e = launch_ls_pass(v64, x64, q, c->ls_nw_opt, G, a, s);
  if (c->profile && e0 && e1) {
    (void)hipEventRecord(e1, s);
    c->ev_pending.push_back({e0, e1, bytes, 0});
  }
  if (e != hipSuccess) return hip_err(c, e, "one-reduction sweep");
  if ((e = launch_ls_reduce(sm, s)) != hipSuccess) return hip_err(c, e, "one-reduction reduce");
  if ((e = launch_ls_finalize(sm, s)) != hipSuccess) return hip_err(c, e, "one-reduction finalize");
  // the host model of the pending columns
  if (c->ls_hu) {
    c->q_host += 1;
    c->ls_hu = 0;
  }
  if (c->ls_hx) {
    c->ls_hu = 1;
    c->ls_hx = 0;
  }
  if (!flush) c->ls_hx = 1;
  c->mirror_valid = false;
  c->dmd.valid = false;
  return FOA_OK;
}

}  // namespace

foa_status enqueue_ls_push(foa_ctx_s *c, const void *x, bool x64) {
  if (c->q_host + c->ls_hu + c->ls_hx >= c->n_max)
    return set_err(c, FOA_E_CAPACITY, "capacity %d reached", c->n_max);
  return enqueue_ls_sweep(c, x, x64);
}

foa_status enqueue_ls_flush(foa_ctx_s *c) {
  while (c->ls_hu || c->ls_hx) {
    foa_status r = enqueue_ls_sweep(c, nullptr, false);
    if (r != FOA_OK) return r;
  }
  return FOA_OK;
}

}  // namespace foa
