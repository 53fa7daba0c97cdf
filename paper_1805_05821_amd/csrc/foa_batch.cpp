// Batched form of the C ABI: many independent FOA streams of uneven n and
// capacity in one caller-owned workspace, all advanced by one snapshot per
// foa_batch_push as a single graph launch.  Each stream is exactly the single
// stream of foa_api.cpp (same layout, same kernels' arithmetic); per-stream
// context views give access to its state, basis, truncation and modes.
//
// Work decomposition of the row passes, rebuilt on the device every step: the
// active streams are bucketed by basis size (one pass kernel per column-tile
// width) and each bucket's panels are cut into equal contiguous ranges, one
// per workgroup.  The grid and the smallest range ("unit_panels") are chosen
// by timing candidates (autotuner) and cached in a JSON table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "foa.h"
#include "foa_ctx.h"
#include "foa_internal.h"

using namespace foa;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinUnitPanels = 4;                 // smallest range: sizes the partial slots
constexpr int kUnitCandidates[] = {4, 16, 64};    // bucket mode: smallest range (panels)
constexpr int kTuneSamples = 8;                      // basis sizes timed per configuration

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct BatchLayout {
  std::vector<size_t> off;       // per-stream Layout base
  std::vector<Layout> L;
  size_t states = 0, streams = 0, xptrs = 0, rblk_s = 0, rblk_c = 0, tune_x = 0, total = 0;
  size_t plist = 0, ppre = 0, pfirst = 0, pmeta = 0, pspos = 0;
  size_t qlist = 0, qpre = 0, qsgrp = 0, qfirst = 0, qctl = 0;  // persistent step
  size_t rblocks = 0;
  int64_t max_n = 0;
  int max_nmax = 0;
};

BatchLayout batch_layout(int S, const int64_t *n, const int32_t *n_max, foa_prec prec) {
  BatchLayout B;
  size_t o = 0;
  for (int s = 0; s < S; ++s) {
    const int64_t P = (n[s] + PANEL - 1) / PANEL;
    // ranges are >= kMinUnitPanels panels, so at most P / kMinUnitPanels + 2 touch a stream
    const int slots = (int)((P + kMinUnitPanels - 1) / kMinUnitPanels) + 2;
    Layout L = make_layout(n[s], n_max[s], prec, slots);
    B.off.push_back(o);
    B.L.push_back(L);
    o = align_up(o + L.total);
    B.rblocks += (size_t)(n_max[s] + 1 + 3) / 4;
    B.max_n = std::max<int64_t>(B.max_n, n[s]);
    B.max_nmax = std::max<int>(B.max_nmax, n_max[s]);
  }
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  B.states = take((size_t)S * sizeof(DevState));
  B.streams = take((size_t)S * sizeof(BatchStream));
  B.plist = take((size_t)NBUCKET * S * sizeof(int));
  B.ppre = take((size_t)NBUCKET * (S + 1) * sizeof(int64_t));
  B.pfirst = take((size_t)NBUCKET * kMaxBatchGrid * sizeof(int));
  B.pmeta = take((size_t)NBUCKET * 2 * sizeof(int));
  B.pspos = take((size_t)S * sizeof(int));
  B.qlist = take((size_t)S * sizeof(int));
  B.qpre = take((size_t)(S + 1) * sizeof(int64_t));
  B.qsgrp = take((size_t)S * sizeof(int));
  B.qfirst = take((size_t)kMaxGroups * kMaxRanks * sizeof(int));
  B.qctl = take(kCtlInts * sizeof(int));
  B.xptrs = take((size_t)S * sizeof(void *));
  B.rblk_s = take(B.rblocks * sizeof(int));
  B.rblk_c = take(B.rblocks * sizeof(int));
  B.tune_x = take((size_t)B.max_n * sizeof(float));
  B.total = o;
  return B;
}

}  // namespace

struct foa_batch_s {
  int S = 0;
  foa_prec prec = FOA_PREC_F32;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  int device = 0, cus = 0;
  double tol = 0.0;
  BatchLayout B;
  std::vector<int64_t> n;
  std::vector<int> nmax;
  std::vector<foa_ctx_s *> views;
  BatchArgs args{};
  int unit_panels = 16, grid = 0;
  bool persist = false;  // one persistent launch for the streams of up to kPersistCols columns
  int pgrid = 0;         // its workgroups (resident complement)
  int occ[NBUCKET] = {};  // resident row-pass workgroups per CU, per bucket
  double tuned_ms = 0.0;
  // one captured step per snapshot dtype and widest bucket that can be in use
  hipGraph_t graph[2][NBUCKET] = {};
  hipGraphExec_t exec[2][NBUCKET] = {};
  // one-reduction form (foa_batch_set_form): flush steps, one graph per widest bucket
  int form = 0;
  hipGraph_t graph_flush[NBUCKET] = {};
  hipGraphExec_t exec_flush[NBUCKET] = {};
  bool ls_pending = false;  // pushes since the last flush
  int pushes = 0;  // foa_batch_push calls since the last reset
  std::string tune_path, tune_key;
  std::vector<DevState> hstates;
};

namespace {

foa_status upload_config(foa_batch_s *b, int unit_panels) {
  std::vector<BatchStream> ds(b->S);
  for (int s = 0; s < b->S; ++s) {
    foa_ctx_s *v = b->views[s];
    BatchStream &d = ds[s];
    d.W = v->W;
    d.w = v->w;
    d.part = v->part;
    d.partn = v->partn;
    d.st = v->sa.st;
    d.H = v->sa.H;
    d.beta = v->sa.beta;
    d.sigma = v->sa.sigma;
    d.bvec = v->sa.bvec;
    d.h = v->sa.h;
    d.s = v->sa.s;
    d.coefA = v->sa.coefA;
    d.coefB = v->sa.coefB;
    d.coefC = v->sa.coefC;
    d.part1 = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_part1);
    d.red = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_red);
    d.xpre = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_xpre);
    d.what = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_what);
    if (v->prec == FOA_PREC_F32) {
      d.part2 = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_part2);
      d.E = reinterpret_cast<double *>(static_cast<char *>(v->ws) + v->L.ls_E);
    } else {
      d.part2 = nullptr;
      d.E = nullptr;
    }
    d.n = v->n;
    d.P = v->L.P;
    d.n_max = v->n_max;
    d.ldg = v->L.ldg;
    d.ldH = v->L.ldH;
    d.ldB = v->L.ldB;
  }
  hipError_t e = hipMemcpy(b->ws + b->B.streams, ds.data(), ds.size() * sizeof(BatchStream), hipMemcpyHostToDevice);
  if (e != hipSuccess) return FOA_E_DEVICE;
  b->unit_panels = unit_panels;
  b->args.min_seg = unit_panels;
  b->args.p_unit = std::max(unit_panels, kMinUnitPanels);
  // every bucket gets at least the tuned grid, and at least one workgroup
  // per resident slot of its kernel
  for (int k = 0; k < NBUCKET; ++k) {
    if (b->occ[k] <= 0)
      b->occ[k] = b->form == 1 ? ls_batch_occupancy(b->prec == FOA_PREC_F64, k)
                               : batch_pass_occupancy(b->prec == FOA_PREC_F64, k);
    b->args.gridb[k] = std::min(kMaxBatchGrid, std::max(b->grid, b->occ[k] * b->cus));
  }
  return FOA_OK;
}

// All kernels of one step, enqueued on stream s (direct launches or capture).
// Bucket mode: per pass one row-pass launch per tile bucket up to kmax, then
// the reductions, finalize and next b.  Persistent mode (FP32 basis): the
// streams of up to kPersistCols columns run in one persistent launch; first
// pushes and wider bases take the bucket launches, which skip the others.
hipError_t enqueue_ls_step(foa_batch_s *b, bool x_f64, hipStream_t s, int kmax) {
  const bool v64 = b->prec == FOA_PREC_F64;
  const BatchArgs &a = b->args;
  hipError_t e;
  if ((e = launch_batch_plan(a, s)) != hipSuccess) return e;
  for (int k = 0; k <= kmax && k < NBUCKET; ++k)
    if (ls_batch_supported(v64, k) && (e = launch_ls_batch_pass(v64, x_f64, k, a.gridb[k], a, s)) != hipSuccess)
      return e;
  return launch_ls_batch_small(a, s);
}

hipError_t enqueue_step(foa_batch_s *b, bool x_f64, hipStream_t s, int kmax) {
  if (b->form == 1) return enqueue_ls_step(b, x_f64, s, kmax);
  const bool v64 = b->prec == FOA_PREC_F64;
  const int cols = batch_cols_per_qw(v64);
  const int qmax = pick_qw(std::max(b->B.max_nmax - 1, 1), cols);
  const bool pers = b->persist && !v64;
  // buckets run by launches: all, or in persistent mode only those wider than kPersistCols
  int kfirst = 1;
  if (pers)
    for (int qw = 1; qw * cols <= kPersistCols; qw *= 2) ++kfirst;
  const BatchArgs &a = b->args;
  hipError_t e;
  if ((e = launch_batch_plan(a, s)) != hipSuccess) return e;
  if (pers && (e = launch_persist_plan(a, s)) != hipSuccess) return e;
  if ((e = launch_batch_pass(PM_INIT, v64, x_f64, 1, a.gridb[0], a, s)) != hipSuccess) return e;
  if (pers && (e = launch_step_persist(x_f64, b->pgrid, a, s)) != hipSuccess) return e;
  for (int qw = 1, k = 1; qw <= qmax && k <= kmax; qw *= 2, ++k)
    if (k >= kfirst && (e = launch_batch_pass(PM_A, v64, x_f64, k, a.gridb[k], a, s)) != hipSuccess) return e;
  if ((e = launch_batch_reduce(1, a, s)) != hipSuccess) return e;
  for (int qw = 1, k = 1; qw <= qmax && k <= kmax; qw *= 2, ++k)
    if (k >= kfirst && (e = launch_batch_pass(PM_B, v64, x_f64, k, a.gridb[k], a, s)) != hipSuccess) return e;
  if ((e = launch_batch_reduce(2, a, s)) != hipSuccess) return e;
  for (int qw = 1, k = 1; qw <= qmax && k <= kmax; qw *= 2, ++k)
    if (k >= kfirst && (e = launch_batch_pass(PM_C, v64, x_f64, k, a.gridb[k], a, s)) != hipSuccess) return e;
  if ((e = launch_batch_finalize(a, s)) != hipSuccess) return e;
  return launch_batch_nextb(a, s);
}

void drop_graphs(foa_batch_s *b) {
  for (int x = 0; x < 2; ++x)
    for (int k = 0; k < NBUCKET; ++k) {
      if (b->exec[x][k]) (void)hipGraphExecDestroy(b->exec[x][k]);
      if (b->graph[x][k]) (void)hipGraphDestroy(b->graph[x][k]);
      b->exec[x][k] = nullptr;
      b->graph[x][k] = nullptr;
    }
  for (int k = 0; k < NBUCKET; ++k) {
    if (b->exec_flush[k]) (void)hipGraphExecDestroy(b->exec_flush[k]);
    if (b->graph_flush[k]) (void)hipGraphDestroy(b->graph_flush[k]);
    b->exec_flush[k] = nullptr;
    b->graph_flush[k] = nullptr;
  }
}

// Widest bucket any stream can be in at the next push: a stream's basis
// grows by at most one column per push, so after p pushes since the reset no
// basis is wider than min(p, largest capacity - 1).  (Views cannot push and
// nothing else changes a basis size.)  Buckets above it are certainly empty
// and their launches are left out of that push's graph.
int widest_bucket(const foa_batch_s *b) {
  const int j = std::min(b->pushes, std::max(b->B.max_nmax - 1, 0));
  if (j == 0) return 0;
  const int cols = batch_cols_per_qw(b->prec == FOA_PREC_F64);
  int k = 1;
  for (int qw = 1; qw < 16 && qw * cols < j; qw *= 2) ++k;
  return k;
}

foa_status ensure_graph(foa_batch_s *b, bool x_f64, int kmax, bool flush = false) {
  hipGraphExec_t &slot = flush ? b->exec_flush[kmax] : b->exec[x_f64 ? 1 : 0][kmax];
  hipGraph_t &gslot = flush ? b->graph_flush[kmax] : b->graph[x_f64 ? 1 : 0][kmax];
  if (slot) return FOA_OK;
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return FOA_E_DEVICE;
  if (flush) b->args.ls_mode = 2;  // captured by value into the step's kernels
  hipError_t e = enqueue_step(b, x_f64, b->cap, kmax);
  if (flush) b->args.ls_mode = 1;
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return FOA_E_DEVICE;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return FOA_E_DEVICE;
  }
  gslot = g;
  slot = x;
  return FOA_OK;
}

// One-reduction form: finish the pending columns of every stream (two flush
// steps cover the deepest pipeline; a stream with nothing pending is left
// alone).
foa_status ls_flush(foa_batch_s *b) {
  if (b->form != 1 || !b->ls_pending) return FOA_OK;
  const int kmax = widest_bucket(b);
  foa_status r = ensure_graph(b, false, kmax, true);
  if (r != FOA_OK) return r;
  for (int i = 0; i < 2; ++i)
    if (hipGraphLaunch(b->exec_flush[kmax], b->stream) != hipSuccess) return FOA_E_DEVICE;
  b->ls_pending = false;
  for (foa_ctx_s *v : b->views) {
    v->mirror_valid = false;
    v->dmd.valid = false;
  }
  return FOA_OK;
}

foa_status reset_states(foa_batch_s *b) {
  if (launch_batch_init_states(b->args, b->tol, b->stream) != hipSuccess) return FOA_E_DEVICE;
  b->pushes = 0;
  if (hipMemsetAsync(b->ws + b->B.qctl, 0, kCtlInts * sizeof(int), b->stream) != hipSuccess) return FOA_E_DEVICE;
  for (foa_ctx_s *v : b->views) {
    v->q_host = 0;
    v->dev_status = ST_ACTIVE;
    v->mirror_valid = false;
    v->dmd.valid = false;
    v->trunc_r = 0;
    v->trunc_m = 0;
    v->Ur.clear();
  }
  return FOA_OK;
}

// ---- autotuner table: {"entries": [{"key": K, "unit_panels": U, "grid": G, "ms_per_step": T}, ...]}
struct TuneEntry {
  std::string key;
  int unit = 0, grid = 0, persist = 0;
  double ms = 0;
};

std::vector<TuneEntry> read_table(const std::string &path) {
  std::vector<TuneEntry> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t pos = 0;
  while ((pos = t.find("\"key\"", pos)) != std::string::npos) {
    TuneEntry e;
    const size_t q1 = t.find('"', t.find(':', pos) + 1);
    const size_t q2 = t.find('"', q1 + 1);
    if (q1 == std::string::npos || q2 == std::string::npos) break;
    e.key = t.substr(q1 + 1, q2 - q1 - 1);
    const size_t end = t.find('}', q2);
    auto num = [&](const char *name) -> double {
      const size_t k = t.find(name, q2);
      if (k == std::string::npos || k > end) return 0.0;
      return std::atof(t.c_str() + t.find(':', k) + 1);
    };
    e.unit = (int)num("\"unit_panels\"");
    e.grid = (int)num("\"grid\"");
    e.persist = (int)num("\"persist\"");
    e.ms = num("\"ms_per_step\"");
    if (e.unit > 0 && e.grid > 0) out.push_back(e);
    pos = q2;
  }
  return out;
}

void write_table(const std::string &path, const std::vector<TuneEntry> &ents) {
  std::ofstream f(path);
  f << "{\"entries\": [\n";
  for (size_t i = 0; i < ents.size(); ++i)
    f << "  {\"key\": \"" << ents[i].key << "\", \"unit_panels\": " << ents[i].unit << ", \"grid\": " << ents[i].grid << ", \"persist\": " << ents[i].persist
      << ", \"ms_per_step\": " << ents[i].ms << "}" << (i + 1 < ents.size() ? "," : "") << "\n";
  f << "]}\n";
}

// Estimated run time of one configuration: every stream from q = 0 to its
// capacity, one snapshot per step.  The run's steps are cut into kTuneSamples
// equal intervals; for each, the states are set to the interval's midpoint
// basis size (streams already full are idle) and one step is timed after one
// untimed step.  Inputs are a hash sequence; the basis contents are whatever
// the workspace holds (timing only: every state is reset afterwards).
foa_status time_config(foa_batch_s *b, int unit, int grid, bool persist, double *ms_out) {
  b->grid = std::min(grid, kMaxBatchGrid);
  b->persist = persist;
  foa_status r = upload_config(b, unit);
  if (r != FOA_OK) return r;
  if ((r = reset_states(b)) != FOA_OK) return r;
  float *tx = reinterpret_cast<float *>(b->ws + b->B.tune_x);
  std::vector<const void *> ptrs(b->S);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FOA_E_DEVICE;
  hipError_t e = hipSuccess;
  const int T = b->B.max_nmax;
  double est = 0.0;
  for (int k = 0; k < kTuneSamples && e == hipSuccess; ++k) {
    const int t = (int)(((2 * k + 1) * (int64_t)T) / (2 * kTuneSamples));
    for (int s = 0; s < b->S; ++s) ptrs[s] = t < b->nmax[s] ? (const void *)tx : nullptr;
    e = hipMemcpyAsync(b->ws + b->B.xptrs, ptrs.data(), ptrs.size() * sizeof(void *), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess) e = launch_fill_random(tx, b->B.max_n, (uint32_t)k, b->stream);
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = launch_tune_states(b->args, t, b->stream);
      if (e == hipSuccess && rep == 1) e = hipEventRecord(e0, b->stream);
      if (e == hipSuccess) e = enqueue_step(b, false, b->stream, NBUCKET - 1);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);  // the host pointer array is reused
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    est += (double)ms * T / kTuneSamples;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return FOA_E_DEVICE;
  int err = 0;
  if (hipMemcpy(&err, b->ws + b->B.qctl + kCtlErr * sizeof(int), sizeof(int), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return FOA_E_DEVICE;
  if (err != 0) {
    if (!persist) return FOA_E_DEVICE;
    *ms_out = 1e300;  // the persistent step did not complete here: never chosen
    return reset_states(b);
  }
  *ms_out = est;
  return FOA_OK;
}

// The XCD ids that workgroups of this device run on: the persistent step
// keeps one work queue per XCD so that every exchange between its workgroups
// stays inside one L2.  More ids than queues, or none: no persistent mode.
foa_status probe_xcds(foa_batch_s *b) {
  b->args.p_groups = 0;
  b->args.p_xmap = ~0ull;
  unsigned *mask = reinterpret_cast<unsigned *>(b->ws + b->B.qctl + kCtlProbe * sizeof(int));
  unsigned m = 0;
  if (hipMemsetAsync(mask, 0, sizeof(unsigned), b->stream) != hipSuccess ||
      launch_xcc_probe(mask, 16 * b->cus, b->stream) != hipSuccess ||
      hipMemcpyAsync(&m, mask, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return FOA_E_DEVICE;
  int g = 0;
  uint64_t map = ~0ull;
  for (int id = 0; id < 16; ++id)
    if (m & (1u << id)) {
      if (g == kMaxGroups) return FOA_OK;
      map = (map & ~(0xFull << (4 * id))) | ((uint64_t)g << (4 * id));
      ++g;
    }
  // workgroups per XCD: the resident complement of the launch, split evenly
  const int ranks = std::min(b->pgrid / g, kMaxRanks);
  if (ranks < 1) return FOA_OK;
  b->args.p_groups = g;
  b->args.p_xmap = map;
  b->args.p_ranks = ranks;
  b->pgrid = ranks * g;
  return FOA_OK;
}

foa_status apply_config(foa_batch_s *b, int unit, int grid, bool persist) {
  b->grid = std::min(grid, kMaxBatchGrid);
  b->persist = persist && b->prec == FOA_PREC_F32 && b->args.p_groups > 0;
  return upload_config(b, unit);
}

foa_status tune(foa_batch_s *b) {
  std::vector<TuneEntry> table;
  if (!b->tune_path.empty()) {
    table = read_table(b->tune_path);
    for (const TuneEntry &t : table)
      if (t.key == b->tune_key) {
        b->tuned_ms = t.ms;
        return apply_config(b, t.unit, t.grid, t.persist != 0);
      }
  }
  double best = 1e300;
  int bu = 16, bg = 2 * b->cus, bp = 0;
  auto consider = [&](int unit, int grid, bool persist) -> foa_status {
    double ms = 0;
    foa_status r = time_config(b, unit, grid, persist, &ms);
    if (r != FOA_OK) return r;
    if (ms < best) {
      best = ms;
      bu = unit;
      bg = grid;
      bp = persist ? 1 : 0;
    }
    return FOA_OK;
  };
  foa_status r;
  for (int unit : kUnitCandidates)
    for (int gm : {1, 2, 4})
      if ((r = consider(unit, gm * b->cus, false)) != FOA_OK) return r;
  if (b->prec == FOA_PREC_F32 && b->args.p_groups > 0 && b->form == 0)
    for (int unit : kUnitCandidates)
      if ((r = consider(unit, 2 * b->cus, true)) != FOA_OK) return r;
  b->tuned_ms = best;
  if ((r = apply_config(b, bu, bg, bp != 0)) != FOA_OK) return r;
  if (!b->tune_path.empty()) {
    table.push_back(TuneEntry{b->tune_key, bu, bg, bp, best});
    write_table(b->tune_path, table);
  }
  return FOA_OK;
}

}  // namespace

extern "C" {

foa_status foa_batch_workspace_bytes(int32_t S, const int64_t *n, const int32_t *n_max, foa_prec prec, size_t *bytes) {
  if (S < 1 || !n || !n_max || !bytes || (prec != FOA_PREC_F32 && prec != FOA_PREC_F64)) return FOA_E_ARG;
  for (int s = 0; s < S; ++s)
    if (n[s] < 1 || n_max[s] < 1 || n_max[s] > FOA_MAX_CAPACITY) return FOA_E_ARG;
  *bytes = batch_layout(S, n, n_max, prec).total;
  return FOA_OK;
}

foa_status foa_batch_init(foa_batch *out, int32_t S, const int64_t *n, const int32_t *n_max, foa_prec prec,
                          void *d_workspace, size_t ws_bytes, void *hip_stream, double breakdown_tol,
                          const char *tune_table_json) {
  if (!out) return FOA_E_ARG;
  *out = nullptr;
  size_t need = 0;
  if (foa_batch_workspace_bytes(S, n, n_max, prec, &need) != FOA_OK) return FOA_E_ARG;
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % kAlign || std::isnan(breakdown_tol))
    return FOA_E_ARG;
  if (ws_bytes < need) return FOA_E_NOMEM;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FOA_E_DEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return FOA_E_DEVICE;
  foa_batch_s *b = new (std::nothrow) foa_batch_s();
  if (!b) return FOA_E_NOMEM;
  b->S = S;
  b->prec = prec;
  b->ws = static_cast<char *>(d_workspace);
  b->ws_bytes = ws_bytes;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->device = dev;
  b->cus = cus;
  b->grid = std::min(2 * cus, kMaxBatchGrid);
  b->B = batch_layout(S, n, n_max, prec);
  b->n.assign(n, n + S);
  b->nmax.assign(n_max, n_max + S);
  int max_nmax = 0;
  for (int s = 0; s < S; ++s) max_nmax = std::max<int>(max_nmax, n_max[s]);
  b->tol = breakdown_tol < 0 ? (double)max_nmax * std::ldexp(1.0, -52) : breakdown_tol;
  DevState *states = reinterpret_cast<DevState *>(b->ws + b->B.states);
  for (int s = 0; s < S; ++s) {
    foa_ctx_s *v = new (std::nothrow) foa_ctx_s();
    if (!v) {
      foa_batch_destroy(b);
      return FOA_E_NOMEM;
    }
    v->n = n[s];
    v->n_max = n_max[s];
    v->prec = prec;
    v->ws = b->ws + b->B.off[s];
    v->ws_bytes = b->B.L[s].total;
    v->stream = b->stream;
    v->L = b->B.L[s];
    v->device = dev;
    v->cus = cus;
    v->tol = b->tol;
    v->is_view = true;
    bind_pointers(v);
    v->sa.st = states + s;  // all scalar states are contiguous for one-copy syncs
    b->views.push_back(v);
  }
  b->args.streams = reinterpret_cast<const BatchStream *>(b->ws + b->B.streams);
  b->args.list = reinterpret_cast<int *>(b->ws + b->B.plist);
  b->args.pre = reinterpret_cast<int64_t *>(b->ws + b->B.ppre);
  b->args.first = reinterpret_cast<int *>(b->ws + b->B.pfirst);
  b->args.meta = reinterpret_cast<int *>(b->ws + b->B.pmeta);
  b->args.spos = reinterpret_cast<int *>(b->ws + b->B.pspos);
  b->args.p_list = reinterpret_cast<int *>(b->ws + b->B.qlist);
  b->args.p_pre = reinterpret_cast<int64_t *>(b->ws + b->B.qpre);
  b->args.p_sgrp = reinterpret_cast<int *>(b->ws + b->B.qsgrp);
  b->args.p_first = reinterpret_cast<int *>(b->ws + b->B.qfirst);
  b->args.p_ctl = reinterpret_cast<int *>(b->ws + b->B.qctl);
  b->args.cols_per_qw = batch_cols_per_qw(prec == FOA_PREC_F64);
  // Test hook: FOA_PERSIST_SPIN bounds the persistent step's barrier waits
  // (0 makes every wait give up at once, so the error path can be exercised
  // with every kernel still ending normally).
  b->args.p_spin = kPersistSpin;
  if (const char *e = std::getenv("FOA_PERSIST_SPIN")) b->args.p_spin = std::max(0, std::atoi(e));
  b->args.xptrs = reinterpret_cast<const void *const *>(b->ws + b->B.xptrs);
  b->args.rblk_stream = reinterpret_cast<const int *>(b->ws + b->B.rblk_s);
  b->args.rblk_c0 = reinterpret_cast<const int *>(b->ws + b->B.rblk_c);
  b->args.S = S;
  b->args.max_nmax = b->B.max_nmax;
  std::vector<int> rs, rc;
  for (int s = 0; s < S; ++s)
    for (int c0 = 0; c0 < n_max[s] + 1; c0 += 4) {
      rs.push_back(s);
      rc.push_back(c0);
    }
  b->args.n_rblocks = (int)rs.size();
  if (hipMemcpy(b->ws + b->B.rblk_s, rs.data(), rs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->ws + b->B.rblk_c, rc.data(), rc.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    foa_batch_destroy(b);
    return FOA_E_DEVICE;
  }
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  int64_t sum_n = 0;
  for (int s = 0; s < S; ++s) sum_n += n[s];
  char key[256];
  std::snprintf(key, sizeof key, "%s/%s/S%d/n%lld/m%d/cu%d", arch.c_str(), prec == FOA_PREC_F64 ? "f64" : "f32", S,
                (long long)sum_n, max_nmax, cus);
  b->tune_key = key;
  if (tune_table_json) b->tune_path = tune_table_json;
  b->pgrid = prec == FOA_PREC_F32 ? step_persist_occupancy() * cus : 0;
  foa_status r = prec == FOA_PREC_F32 ? probe_xcds(b) : FOA_OK;
  if (r == FOA_OK) r = tune(b);
  if (r == FOA_OK) r = reset_states(b);
  if (r == FOA_OK && hipStreamSynchronize(b->stream) != hipSuccess) r = FOA_E_DEVICE;
  if (r != FOA_OK) {
    foa_batch_destroy(b);
    return r;
  }
  *out = b;
  return FOA_OK;
}

foa_status foa_batch_push(foa_batch b, const void *const *d_x_ptrs, foa_dtype x_dtype) {
  if (!b) return FOA_E_ARG;
  if (!d_x_ptrs || (x_dtype != FOA_F32 && x_dtype != FOA_F64)) return FOA_E_ARG;
  const int kmax = widest_bucket(b);
  foa_status r = ensure_graph(b, x_dtype == FOA_F64, kmax);
  if (r != FOA_OK) return r;
  if (hipMemcpyAsync(b->ws + b->B.xptrs, d_x_ptrs, (size_t)b->S * sizeof(void *), hipMemcpyDeviceToDevice,
                     b->stream) != hipSuccess)
    return FOA_E_DEVICE;
  if (hipGraphLaunch(b->exec[x_dtype == FOA_F64 ? 1 : 0][kmax], b->stream) != hipSuccess) return FOA_E_DEVICE;
  ++b->pushes;
  if (b->form == 1) b->ls_pending = true;
  for (foa_ctx_s *v : b->views) {
    v->mirror_valid = false;
    v->dmd.valid = false;
  }
  return FOA_OK;
}

foa_status foa_batch_sync(foa_batch b, int32_t *h_q, int32_t *h_status) {
  if (!b) return FOA_E_ARG;
  foa_status r = ls_flush(b);
  if (r != FOA_OK) return r;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return FOA_E_DEVICE;
  b->hstates.resize(b->S);
  if (hipMemcpy(b->hstates.data(), b->ws + b->B.states, (size_t)b->S * sizeof(DevState), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return FOA_E_DEVICE;
  for (int s = 0; s < b->S; ++s) {
    const DevState &d = b->hstates[s];
    foa_ctx_s *v = b->views[s];
    v->q_host = d.q;
    v->dev_status = d.status;
    v->pushes = d.pushes;
    if (h_q) h_q[s] = d.q;
    if (h_status) h_status[s] = (d.status == ST_ACTIVE && d.full) ? FOA_E_CAPACITY : map_status(d.status);
  }
  int err = 0;  // the persistent step did not complete (a bounded wait ran out)
  if (hipMemcpy(&err, b->ws + b->B.qctl + kCtlErr * sizeof(int), sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      err != 0)
    return FOA_E_DEVICE;
  return FOA_OK;
}

foa_status foa_batch_view(foa_batch b, int32_t s, foa_ctx *view) {
  if (!b || !view || s < 0 || s >= b->S) return FOA_E_ARG;
  *view = b->views[s];
  return FOA_OK;
}

foa_status foa_batch_reset(foa_batch b) {
  if (!b) return FOA_E_ARG;
  b->ls_pending = false;
  return reset_states(b);
}

foa_status foa_batch_flush(foa_batch b) {
  if (!b) return FOA_E_ARG;
  return ls_flush(b);
}

foa_status foa_batch_set_form(foa_batch b, foa_form form) {
  if (!b) return FOA_E_ARG;
  if (form != FOA_FORM_CGS2 && form != FOA_FORM_ONE_REDUCTION) return FOA_E_ARG;
  if (b->pushes != 0) return FOA_E_STATE;  // before the first push (after init or reset)
  const int f = form == FOA_FORM_ONE_REDUCTION ? 1 : 0;
  if (f == 1 && b->prec == FOA_PREC_F64 && b->B.max_nmax > 257) return FOA_E_ARG;
  if (f == b->form) return FOA_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return FOA_E_DEVICE;
  drop_graphs(b);
  b->form = f;
  b->args.ls_mode = f;
  b->persist = false;
  for (int k = 0; k < NBUCKET; ++k) b->occ[k] = 0;
  const size_t cut = b->tune_key.find("/form");
  if (cut != std::string::npos) b->tune_key.resize(cut);
  if (f == 1) b->tune_key += "/form1";
  foa_status r = tune(b);
  if (r == FOA_OK) r = reset_states(b);
  if (r == FOA_OK && hipStreamSynchronize(b->stream) != hipSuccess) r = FOA_E_DEVICE;
  return r;
}

foa_status foa_batch_destroy(foa_batch b) {
  if (!b) return FOA_E_ARG;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (foa_ctx_s *v : b->views) {
    release_events(v);
    delete v;
  }
  delete b;
  return FOA_OK;
}

}  // extern "C"
