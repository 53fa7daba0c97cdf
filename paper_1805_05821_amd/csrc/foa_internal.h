// Internal declarations shared by the HIP kernels (foa_kernels.hip) and the
// host side of the C ABI (foa_api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace foa {

// Rows per storage panel.  V lives in the workspace in "panel" layout: rows are
// grouped in panels of PANEL rows; inside a panel the storage is column-major
// with all n_max columns, so the first j columns of a panel are one contiguous
// PANEL*j*sizeof(T) range and every wavefront load below reads 1 KiB contiguous.
constexpr int PANEL = 64;

// Device status codes (mirrors foa_status for the device-detected cases).
constexpr int ST_ACTIVE = 0;
constexpr int ST_INVARIANT = 1;
constexpr int ST_NONFINITE = -4;
constexpr int ST_ZERO = -8;

// Device-resident scalar state of one stream.
struct DevState {
  int q;          // basis vectors committed
  int status;     // ST_*
  int pushes;     // snapshots offered (including ignored ones)
  int jstep;      // batched form: q at the start of the current step
  int act;        // batched form: 1 if the stream takes a snapshot this step
  int full;       // batched form: a snapshot arrived after the capacity was reached
  double xfro2;   // ||X_1^q||_F^2 of the committed snapshots
  double xn2;     // ||x||^2 of the snapshot being pushed
  double scaleA;  // 1 / beta_{q,q}: scale of w for the next push (eq. avpsijp1beta)
  double tol;     // breakdown tolerance (relative to ||X||_F)
  double hlast;   // last h_{j+1,j}
  int nseg;       // batched form: partial-sum slots written by this step's passes
  int seg0;       // batched form: first workgroup of this step's passes on the stream
  int pers;       // batched form: this step is run by the persistent step kernel
  int pad1;
  // one-reduction form (foa_lowsync.hip): pending columns after the final q
  int ls_u;       // column q is under its second projection (w in h, coefW in coefA)
  int ls_x;       // column q + ls_u holds a snapshot copy (z in s, coefZ in coefB)
  int ls_nx;      // snapshots accepted (final + pending)
  int ls_pad;
  double ls_alpha;  // ||u||^2 of the pending column
  double ls_gamma;  // u^T x of the pending column and snapshot
  double ls_rhohat; // estimated norm sqrt(alpha - ||w||^2) of the pending column
  double ls_rt;     // first-pass coefficient of the snapshot on the pending column
  double ls_cq;     // ls_rt / ls_rhohat (0 if the estimate is 0)
};

// Pass modes of the fused row kernel.
enum PassMode : int {
  PM_INIT = 0,  // q = 0: V(:,0) <- x, partial ||x||^2            (first snapshot)
  PM_A = 1,     // w_A = (x - V c0) * scale, partial V^T w_A, ||x||^2  (w and its projection)
  PM_B = 2,     // w_B = w_A - V c1, partial V^T w_B                  (orthogonalisation, reprojection)
  PM_C = 3,     // w_C = w_B - V c2, V(:,j) <- w_C, partial ||w_C||^2 (reorthogonalisation, norm)
};

struct PassArgs {
  const void *W;        // V storage (panel layout), element type TV
  const void *x;        // snapshot, element type TX
  double *w;            // FP64 work vector, n_pad entries (shapes that store w)
  const double *coef[3];  // sigma o b, sigma o h, sigma o s (j entries each)
  const DevState *st;   // status (read) and scaleA
  double *part;         // column partials, layout part[c * ldg + block]
  double *partn;        // norm partials, one per block
  int64_t n;            // valid rows
  int64_t P;            // panels
  int j;                // active columns (basis size q)
  int n_max;            // capacity (columns per panel)
  int ldg;              // leading dimension of part (>= gridDim.x)
};

// Small-matrix pointers of one stream (FP64, column-major).
struct SmallArgs {
  DevState *st;
  double *H;       // H_bar, ldH rows
  double *beta;    // beta, ldB rows
  double *sigma;   // per-column scale: v_c = sigma_c * stored column c
  double *bvec;    // partial beta column of the current push (eq. betacolumnupdate)
  double *h;       // h_{1:j,j}
  double *s;       // s_{1:j}
  double *coefA;   // sigma o b
  double *coefB;   // sigma o h
  double *coefC;   // sigma o s
  const double *part;
  const double *partn;
  int ldH, ldB;
  int n_max;
  int G;           // partial blocks of the preceding pass
  int ldg;
  int j;           // basis size before this push (host's expectation)
};

// ---- batched form ----------------------------------------------------------
// Per-stream descriptor (device memory).
struct BatchStream {
  void *W;
  double *w, *part, *partn;
  DevState *st;
  double *H, *beta, *sigma, *bvec, *h, *s, *coefA, *coefB, *coefC;
  double *part1, *red, *xpre;  // one-reduction form
  double *part2, *E, *what;    // one-reduction form, FP32 basis: the Gram correction
  int64_t n, P;
  int n_max, ldg, ldH, ldB;
};
// Buckets of the per-step plan: 0 = first push of a stream (basis empty);
// 1 + log2(QW) = basis size in the column-tile range of tile width QW.
constexpr int NBUCKET = 6;
constexpr int kMaxBatchGrid = 4096;
// Partial-sum slots of a single stream (leading dimension of its pass
// partials): the most workgroups a single-stream row pass may use.
constexpr int kStreamSlots = 1024;
// Per-step plan (device memory, rebuilt by the plan kernels every step): for
// bucket k, the active streams in stream order with their panel prefix sums,
// the number of workgroups that share the bucket's panels, and for each of
// them the list position of its first stream.
struct BatchArgs {
  const BatchStream *streams;
  const void *const *xptrs;  // device array of S snapshot pointers (NULL: idle)
  const int *rblk_stream;    // reduce blocks: stream of block b
  const int *rblk_c0;        // reduce blocks: first column of block b
  int *list;                 // NBUCKET x S
  int64_t *pre;              // NBUCKET x (S + 1)
  int *first;                // NBUCKET x kMaxBatchGrid
  int *meta;                 // NBUCKET x 2: streams in the bucket, workgroups in use
  int *spos;                 // S: bucket (high 8 bits) and list position of each active stream
  int S, n_rblocks, max_nmax;
  int ls_mode;               // 0: three-sweep form; one-reduction form: 1 push step, 2 flush step
  int cols_per_qw;           // basis columns per unit of tile width
  int gridb[NBUCKET];        // workgroups of the row-pass launches of bucket k
  int min_seg;               // fewest panels per workgroup
  // persistent step (streams with 1..kPersistCols basis columns, FP32 basis):
  int *p_list;               // S: its streams, in stream order
  int64_t *p_pre;            // S + 1: their panel prefix sums
  int *p_sgrp;               // S: group of each listed stream
  int *p_first;              // kMaxGroups x kMaxRanks: first list position of each rank's range
  int *p_ctl;                // kCtlInts control words (layout below)
  int p_unit;                // fewest panels per rank
  int p_ranks;               // workgroups per XCD in the launch (at most kMaxRanks)
  int p_groups;              // groups, one per XCD the device showed (1..kMaxGroups)
  int p_spin;                // polls of a barrier wait before it gives up (kPersistSpin)
  uint64_t p_xmap;           // group of each XCD id, 4 bits per id (15: none)
};
// Persistent step: widest basis it takes (FP32 tiles of up to 8 groups of
// 8 wavefronts x 4 columns) and its workgroup shape.
constexpr int kPersistCols = 256;
constexpr int kPersistNW = 8;
// Persistent-step control words: [2] listed streams, [3] error flag (a
// wait ran out, or a group left ranks unfinished), [4] workgroups done, [5]
// XCD-id mask of the probe; from kCtlGroup0, per group (kGc* offsets): its
// list range, ranks, column blocks of the reductions, arrival counter,
// phase barrier counters and finished ranks.
constexpr int kMaxGroups = 8;
constexpr int kMaxRanks = 256;
constexpr int kPersistSpin = 1 << 22;  // default polls of a persistent-step barrier wait
constexpr int kCtlStreams = 2, kCtlErr = 3, kCtlExit = 4, kCtlProbe = 5;
constexpr int kCtlGroup0 = 8, kCtlGroupStride = 16;
constexpr int kGcLo = 0, kGcCnt = 1, kGcRanks = 2, kGcBlocks = 3, kGcArrive = 4, kGcBar = 5, kGcPhases = 5,
              kGcDone = 10;
constexpr int kCtlInts = kCtlGroup0 + kCtlGroupStride * kMaxGroups;

// ---- blocked form ------------------------------------------------------------
constexpr int BPK = 4;  // snapshots per block
// small-area offsets (doubles): R = R1 + R2 (+ R3) (n_max x BPK,
// [c * BPK + k]), ||y_k||^2, S_total and T_0 .. T_2 (BPK x BPK, row-major),
// R2 alone (the test for a third projection)
constexpr int SM_R = 0;
constexpr int SM_YN2 = SM_R + 512 * BPK;
constexpr int SM_S = SM_YN2 + BPK;
constexpr int SM_T = SM_S + BPK * BPK;       // T_0, T_1, T_2: the Cholesky steps' inverses
constexpr int SM_R2 = SM_T + 3 * BPK * BPK;
constexpr int SM_TOTAL = SM_R2 + 512 * BPK;
struct BlockArgs {
  void *W;          // stored basis (panel layout)
  const void *x;    // first snapshot of the block; snapshot k at x + k * ldx (elements)
  int64_t ldx;
  double *Z;        // n_pad x BPK block, panel layout [panel][k][64]
  double *coef;     // pass coefficients, [c * BPK + k]
  double *partb;    // block-pass partials, [(c * BPK + k) * ldg + slot]
  double *partg;    // block Gram partials, [slot * BPK * BPK + k * BPK + l]
  double *sm;       // small area (SM_* offsets)
  int *flag;        // nonzero: the block (or an earlier one) was rejected
  const int *gate;  // non-null: the kernel runs only while *gate is nonzero (third projection)
  int tlev;         // block passes: triangular factors T_0 .. T_{tlev-1} applied to each row of Z
  int c0;           // block row passes: first basis column of the window (j columns from it)
  const void *xn;   // BP_ZR: first snapshot of the next block (same ldx and type as x)
  double *dnext;    // raw column sums V^T Y of the next block over this block's j columns, [c * BPK + k]
  double *partq;    // ZG_YNQ partials of (previous block's new columns)^T Y, [slot * BPK * BPK + c * BPK + k]
  int qy;           // this block's V^T Y comes from dnext (old columns) and partq (the 4 newest)
  DevState *st;
  double *H, *beta, *sigma;
  int64_t n, P;
  int j, n_max, ldg, ldH, ldB;
  int G;            // workgroups of the block passes (partial slots)
  int Gz;           // workgroups of the block Gram passes
};

// ---- one-reduction form (foa_lowsync.hip) -----------------------------------
// One sweep over the rows per push: second projection of the pending column
// (index q when ls_u), first projection of the pending snapshot copy (index
// q + ls_u when ls_x), copy of the new snapshot, and the column sums of the
// one reduction.  Partial sums per workgroup slot: part0[c * ldg + slot]
// (stored column c against the formed column), part1[c * ldg + slot] (against
// the new snapshot), and part1[(n_max + k) * ldg + slot] for the six scalar
// sums LS_S*.
enum { LS_UU = 0, LS_UF = 1, LS_UX = 2, LS_FF = 3, LS_FX = 4, LS_XX = 5, LS_NSC = 6 };
struct LsArgs {
  void *W;               // basis storage (panel layout), element type TV
  const void *x;         // new snapshot (type TX), NULL for a flush sweep
  const double *coefW;   // sigma o w (second projection of the pending column)
  const double *coefZ;   // sigma o z (first projection of the pending snapshot)
  const DevState *st;
  double *part0, *part1;
  double *part2;         // FP32 basis: the finished column's rounding error against each column
  int64_t n, P;
  int n_max, ldg;
  int flush;             // 1: no new snapshot
};
struct LsSmall {
  DevState *st;
  double *H, *beta, *sigma;
  double *w, *z;         // pending coefficient vectors (FP64, unscaled)
  double *coefW, *coefZ; // sigma-scaled copies for the next sweep
  double *red;           // reduced sums: [0, n_max) part0 columns, [n_max, 2 n_max) part1, then LS_NSC
                         // scalars, then (FP32 basis) [2 n_max + LS_NSC, 3 n_max + LS_NSC) part2 columns
  double *bvec;          // H_bar product of the column the finalize finishes
  double *xpre;          // prefix sums of ||x_i||^2 of the accepted snapshots
  double *E;             // FP32 basis: Q^T Q - I of the final columns (n_max x n_max, column-major)
  double *what;          // E w for the new pending column (from k_ls_hprod), then (I - E) w
  const double *part0, *part1, *part2;
  int ldH, ldB, n_max, ldg;
  int G;                 // partial slots written by the sweep
  int nt;                // host's expectation of q (upper bound of the device's)
  int flush;
  int gram;              // 1: FP32 basis, the second projection uses (I - E) w
};

// ---- launchers (defined in foa_kernels.hip) --------------------------------
// tv_f64: V stored in FP64; tx_f64: snapshot in FP64.
// nw: wavefronts per workgroup for an FP32 basis (8 or 16; FP64 uses 16).
hipError_t launch_pass(int mode, bool tv_f64, bool tx_f64, bool prefetch, int nw, int grid,
                       const PassArgs &a, hipStream_t s);
// blocked form (foa_block.hip)
bool block_supported(bool tv_f64, int qw);
hipError_t launch_bpass(int mode, bool tv_f64, bool tx_f64, int nw, int qw, int grid, const BlockArgs &a,
                        hipStream_t s);
hipError_t launch_zgram(int mode, bool tv_f64, bool tx_f64, int grid, const BlockArgs &a, hipStream_t s);
hipError_t launch_breduce(int mode, const BlockArgs &a, hipStream_t s);
hipError_t launch_bchol(int round, const BlockArgs &a, hipStream_t s);
hipError_t launch_bcommit(const BlockArgs &a, hipStream_t s);
hipError_t launch_bflag_clear(int *flag, hipStream_t s);
hipError_t launch_bthird(const BlockArgs &a, int *gate, double unit, hipStream_t s);
// Device address of this device's static block workspace (looked up once per
// device with that device current; the result, or the lookup's error, is kept).
hipError_t block_static_scratch(int device, char **ptr);
// wavefronts per row-pass workgroup at basis size j (nw_opt 0: automatic)
int pass_nw(bool tv_f64, int nw_opt, int j);
// resident workgroups per CU of the row-pass kernel used at tile width qw
int pass_occupancy(bool tv_f64, bool tx_f64, bool prefetch, int nw, int qw);
hipError_t launch_reduce(int mode, const SmallArgs &a, hipStream_t s);
hipError_t launch_finalize(const SmallArgs &a, hipStream_t s);
hipError_t launch_finalize_init(const SmallArgs &a, hipStream_t s);
hipError_t launch_nextb(const SmallArgs &a, hipStream_t s);
hipError_t launch_copy_basis(bool tv_f64, const void *W, const double *sigma, int64_t r0,
                             int64_t nrows, int n_max, int ncols, void *out, int64_t ld,
                             bool out_f64, hipStream_t s);
hipError_t launch_init_state(const SmallArgs &a, double tol, hipStream_t s);
// Phi = W * B for the panel-layout basis W (n x k used columns) and a k x r
// coefficient matrix (sigma already folded in); Phi is column-major with
// leading dimension ld.  Two coefficient layouts, chosen by modes_use_mfma:
//  * FP32 MFMA path (FP32 basis and FP32 output): B is FP32, row-major
//    modes_kpad(k) x modes_rpad(r) (mode index contiguous), zero-padded;
//  * otherwise: B is FP64, column-major k x r (leading dimension k).
bool modes_use_mfma(bool tv_f64, bool out_f64);
int modes_kpad(int k);
int modes_rpad(int r);
hipError_t launch_modes_gemm(bool tv_f64, const void *W, int64_t n, int n_max, int k,
                             const void *B, int r, void *out, int64_t ld, bool out_f64,
                             hipStream_t s);

int pick_qw(int j, int cols_per_qw);
// groups per wavefront of the row pass at basis size j with nw wavefronts
int pass_qw(bool tv_f64, int nw, int j);
// index of a tile width (groups per wavefront: 1, 2, 4, 8, 16, 6, 12) in
// per-width caches, 0..6
int tile_slot(int qw);

// one-reduction form
// wavefronts per sweep workgroup (nw_opt 16: sixteen above 128 columns, FP32 basis)
int ls_nw(bool tv_f64, int q, int nw_opt);
int ls_qw(bool tv_f64, int q, int nw_opt);
bool ls_supported(bool tv_f64, int q);
int ls_occupancy(bool tv_f64, bool tx_f64, int q, int nw_opt);
hipError_t launch_ls_pass(bool tv_f64, bool tx_f64, int q, int nw_opt, int grid, const LsArgs &a, hipStream_t s);
hipError_t launch_ls_reduce(const LsSmall &a, hipStream_t s);
hipError_t launch_ls_finalize(const LsSmall &a, hipStream_t s);
// batched one-reduction form: the sweep of bucket k (0 = empty basis, 1..5 as
// the three-sweep buckets), then the per-stream reduce, H_bar product and finalize
bool ls_batch_supported(bool tv_f64, int k);
int ls_batch_occupancy(bool tv_f64, int k);
hipError_t launch_ls_batch_pass(bool tv_f64, bool tx_f64, int k, int grid, const BatchArgs &b, hipStream_t s);
hipError_t launch_ls_batch_small(const BatchArgs &b, hipStream_t s);

// batched form (one call per kernel of a step; all captured in one graph)
hipError_t launch_batch_plan(const BatchArgs &b, hipStream_t s);
hipError_t launch_persist_plan(const BatchArgs &b, hipStream_t s);
hipError_t launch_tune_states(const BatchArgs &b, int t, hipStream_t s);
hipError_t launch_step_persist(bool tx_f64, int grid, const BatchArgs &b, hipStream_t s);
int step_persist_occupancy();
// ORs 1 << (XCD id) into *mask from `blocks` one-wavefront workgroups
hipError_t launch_xcc_probe(unsigned *mask, int blocks, hipStream_t s);
// row pass of bucket k (0: the first push of a stream, PM_INIT)
hipError_t launch_batch_pass(int mode, bool tv_f64, bool tx_f64, int k, int grid, const BatchArgs &b,
                             hipStream_t s);
hipError_t launch_batch_reduce(int mode, const BatchArgs &b, hipStream_t s);
hipError_t launch_batch_finalize(const BatchArgs &b, hipStream_t s);
hipError_t launch_batch_nextb(const BatchArgs &b, hipStream_t s);
hipError_t launch_batch_init_states(const BatchArgs &b, double tol, hipStream_t s);
// fills out[0..n) with a deterministic pseudo-random sequence of tuning input k
hipError_t launch_fill_random(float *out, int64_t n, uint32_t k, hipStream_t s);
int batch_cols_per_qw(bool tv_f64);
// resident workgroups per CU of the batched row-pass kernel of bucket k
int batch_pass_occupancy(bool tv_f64, int k);

}  // namespace foa
