// Batched form of the FOA push (one iteration of Algorithm 1 for many independent
// streams per step): the per-step plan, the row passes over the planned
// segments, and the per-stream reductions and small kernels.
#include "foa_device.h"

namespace foa {

// ---------------------------------------------------------------------------
// Batched form: many independent streams advanced by one snapshot per step.
// Every kernel reads the per-stream step state (jstep, act, seg0, nseg)
// frozen by the plan kernels, so a captured graph of the step replays
// unchanged while the streams grow.
//
// Plan: the active streams are grouped into buckets by basis size (one row-pass
// instantiation per column-tile width), and within a bucket the concatenation
// of the streams' panels is cut into G equal contiguous ranges, one per
// workgroup (G = min(grid, panels / min_seg)).  A workgroup walks the (one or
// few) streams its range overlaps; its partial sums for a stream go to slot
// (workgroup - first workgroup on that stream), so each stream's slots are
// dense and the reductions sum them in a fixed order.  An empty bucket's
// launch exits at once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ SmallArgs small_of(const BatchStream &d) {
  SmallArgs a{};
  a.st = d.st;
  a.H = d.H;
  a.beta = d.beta;
  a.sigma = d.sigma;
  a.bvec = d.bvec;
  a.h = d.h;
  a.s = d.s;
  a.coefA = d.coefA;
  a.coefB = d.coefB;
  a.coefC = d.coefC;
  a.part = d.part;
  a.partn = d.partn;
  a.ldH = d.ldH;
  a.ldB = d.ldB;
  a.n_max = d.n_max;
  a.G = d.st->nseg;
  a.ldg = d.ldg;
  a.j = d.st->jstep;
  return a;
}

// bucket of an active stream with basis size j: 0 for the first push, else
// 1 + log2 of the tile width (in units of cols_per_qw columns, at most 16)
__device__ __forceinline__ int bucket_of(int j, int cols_per_qw) {
  if (j == 0) return 0;
  int k = 1, qw = 1;
  while (qw < 16 && qw * cols_per_qw < j) {
    qw *= 2;
    ++k;
  }
  return k;
}

// Step state, bucket lists and workgroup ranges, one workgroup of 1024
// threads.  Streams are taken 1024 at a time; per bucket a wavefront prefix
// sum (count and panels) plus the per-wavefront totals give each active
// stream its list position and panel offset; a last sweep cuts each
// bucket's panels into its workgroups' ranges.
__global__ __launch_bounds__(1024) void k_batch_plan(BatchArgs b) {
  __shared__ int s_wcnt[16][NBUCKET];
  __shared__ int64_t s_wpan[16][NBUCKET];
  __shared__ int s_cnt[NBUCKET];
  __shared__ int64_t s_tot[NBUCKET];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < NBUCKET) {
    s_cnt[tid] = 0;
    s_tot[tid] = 0;
  }
  __syncthreads();
  for (int c0 = 0; c0 < b.S; c0 += 1024) {
    const int s = c0 + tid;
    int bk = -1;
    int64_t P = 0;
    if (s < b.S) {
      const BatchStream &d = b.streams[s];
      DevState *st = d.st;
      const bool offered = b.ls_mode != 2 && b.xptrs[s] != nullptr;
      const int j = st->q;
      // one-reduction form: the pending columns also hold snapshots; a flush
      // step runs every stream that has pending columns (also after a
      // non-finite snapshot stopped it)
      const bool room = (b.ls_mode ? j + st->ls_u + st->ls_x : j) < d.n_max;
      const int act = b.ls_mode == 2
                          ? ((st->status == ST_ACTIVE || st->status == ST_NONFINITE) && (st->ls_u || st->ls_x))
                          : ((st->status == ST_ACTIVE && offered && room) ? 1 : 0);
      st->jstep = j;
      st->act = act;
      st->nseg = 0;
      st->pers = 0;
      if (offered && !room && st->status == ST_ACTIVE) st->full = 1;
      if (act) {
        bk = bucket_of(j, b.cols_per_qw);
        P = d.P;
      }
    }
    int myf = 0;
    int64_t myp = 0;
#pragma unroll
    for (int k = 0; k < NBUCKET; ++k) {
      int f = bk == k ? 1 : 0;
      int64_t pp = bk == k ? P : 0;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int tf = __shfl_up(f, o, 64);
        const int64_t tp = __shfl_up(pp, o, 64);
        if (lane >= o) {
          f += tf;
          pp += tp;
        }
      }
      if (bk == k) {
        myf = f;
        myp = pp;
      }
      if (lane == 63) {
        s_wcnt[wave][k] = f;
        s_wpan[wave][k] = pp;
      }
    }
    __syncthreads();
    if (bk >= 0) {
      int wb = 0;
      int64_t wp = 0;
      for (int w = 0; w < wave; ++w) {
        wb += s_wcnt[w][bk];
        wp += s_wpan[w][bk];
      }
      const int pos = s_cnt[bk] + wb + myf - 1;
      b.list[(size_t)bk * b.S + pos] = s;
      b.pre[(size_t)bk * (b.S + 1) + pos] = s_tot[bk] + wp + myp - P;
      b.spos[s] = (bk << 24) | pos;
    }
    __syncthreads();
    if (tid < NBUCKET) {
      int c = 0;
      int64_t t = 0;
      for (int w = 0; w < 16; ++w) {
        c += s_wcnt[w][tid];
        t += s_wpan[w][tid];
      }
      s_cnt[tid] += c;
      s_tot[tid] += t;
    }
    __syncthreads();
  }
  __shared__ int s_G[NBUCKET];
  if (tid < NBUCKET) {
    const int c = s_cnt[tid];
    const int64_t T = s_tot[tid];
    b.pre[(size_t)tid * (b.S + 1) + c] = T;
    int G = 0;
    if (T > 0) {
      const int64_t g = T / b.min_seg;
      G = (int)(g < 1 ? 1 : (g > b.gridb[tid] ? b.gridb[tid] : g));
    }
    b.meta[2 * tid] = c;
    b.meta[2 * tid + 1] = G;
    s_G[tid] = G;
  }
  __syncthreads();
  // Ranges: workgroup g of bucket k covers panels [g T / G, (g + 1) T / G)
  // of the bucket's concatenation, so the workgroup holding panel p is
  // ((p + 1) G - 1) / T.  Per active stream (panels [p0, p1) of its bucket):
  // its first workgroup and workgroup count, and it is the first stream of
  // workgroups ceil(p0 G / T) .. ceil(p1 G / T) - 1 (those whose range
  // starts inside it).
  for (int s = tid; s < b.S; s += 1024) {
    DevState *st = b.streams[s].st;
    if (!st->act) continue;
    const int code = b.spos[s];
    const int k = code >> 24, pos = code & 0xFFFFFF;
    const int G = s_G[k];
    const int64_t T = s_tot[k];
    const int64_t *pre = b.pre + (size_t)k * (b.S + 1);
    const int64_t p0 = pre[pos], p1 = pre[pos + 1];
    const int g0 = (int)(((p0 + 1) * G - 1) / T);
    const int g1 = (int)((p1 * G - 1) / T);
    st->seg0 = g0;
    st->nseg = g1 - g0 + 1;
    const int f0 = (int)((p0 * G + T - 1) / T), f1 = (int)((p1 * G + T - 1) / T);
    for (int g = f0; g < f1 && g < G; ++g) b.first[k * kMaxBatchGrid + g] = pos;
  }
}

// Bucket BK's row pass.  The bucket fixes the basis-size range (tile width
// BK's multiple of cols_per_qw); NW and QW are the kernel shape that covers it.
// Every plan and stream value is read through uniform(): the kernel's stores
// may alias the plan as far as the compiler can tell, so plain loads would
// stay in vector registers, together with everything derived from them.
template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF, int BK>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(pass_waves<TV, QW>())))
void k_pass_batch(BatchArgs b) {
  constexpr int k = MODE == PM_INIT ? 0 : BK;
  __shared__ double lds[pass_lds_doubles<TV, NW, QW, MODE>()];
  const int G = uniform(b.meta[2 * k + 1]);
  if ((int)blockIdx.x >= G) return;
  const int cnt = uniform(b.meta[2 * k]);
  const int64_t *pre = b.pre + (size_t)k * (b.S + 1);
  const int *list = b.list + (size_t)k * b.S;
  const int64_t T = pre[cnt];
  int64_t lo = uniform((int64_t)blockIdx.x * T / G);
  const int64_t hi = uniform((int64_t)(blockIdx.x + 1) * T / G);
  int i = uniform(b.first[k * kMaxBatchGrid + blockIdx.x]);
  while (lo < hi) {
    const int s = uniform(list[i]);
    const int64_t ps = uniform(pre[i]), pe = uniform(pre[i + 1]);
    const int64_t e = pe < hi ? pe : hi;
    const BatchStream &d = b.streams[s];
    const DevState *st = uniform(d.st);
    PassArgs a{};
    a.W = uniform(d.W);
    a.x = uniform(b.xptrs[s]);
    a.w = uniform(d.w);
    a.coef[0] = uniform(d.coefA);
    a.coef[1] = uniform(d.coefB);
    a.coef[2] = uniform(d.coefC);
    a.st = st;
    a.part = uniform(d.part);
    a.partn = uniform(d.partn);
    a.n = uniform(d.n);
    a.P = uniform(d.P);
    a.j = uniform(st->jstep);
    a.n_max = uniform(d.n_max);
    a.ldg = uniform(d.ldg);
    row_pass_body<TV, TX, NW, QW, MODE, PREF>(a, lo - ps, e - ps, 1, (int)blockIdx.x - uniform(st->seg0), lds);
    lo = e;
    ++i;
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_reduce_batch(BatchArgs b) {
  const int s = b.rblk_stream[blockIdx.x];
  const BatchStream &d = b.streams[s];
  if (!d.st->act || d.st->jstep == 0 || d.st->pers) return;
  reduce_body<MODE>(small_of(d), b.rblk_c0[blockIdx.x]);
}

__global__ __launch_bounds__(256) void k_finalize_batch(BatchArgs b) {
  const int s = blockIdx.x;
  const BatchStream &d = b.streams[s];
  DevState *st = d.st;
  if (b.xptrs[s] == nullptr) return;  // idle this step
  if (!st->act) {                      // offered to a stream that no longer takes snapshots
    if (threadIdx.x == 0) st->pushes += 1;
    return;
  }
  if (st->pers) return;                // finalized by the persistent step kernel
  const SmallArgs a = small_of(d);
  if (st->jstep == 0)
    finalize_init_body(a);
  else
    finalize_body(a);
}

__global__ __launch_bounds__(256) void k_nextb_batch(BatchArgs b) {
  const BatchStream &d = b.streams[blockIdx.y];
  if (!d.st->act || d.st->pers) return;
  if ((int)blockIdx.x * 64 > d.st->q) return;
  nextb_body(small_of(d), blockIdx.x);
}

__global__ __launch_bounds__(256) void k_batch_init_states(BatchArgs b, double tol) {
  init_state_body(small_of(b.streams[blockIdx.y]), tol);
}

// Tuning: every stream that can still take a snapshot at step t is put at
// basis size t (active); its other state is left as it is.
__global__ __launch_bounds__(256) void k_tune_states(BatchArgs b, int t) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= b.S) return;
  const BatchStream &d = b.streams[s];
  DevState *st = d.st;
  if (t < d.n_max) {
    st->q = t;
    st->status = ST_ACTIVE;
    st->full = 0;
    // one-reduction form: the steady state (a column and a snapshot pending)
    st->ls_u = st->ls_x = (b.ls_mode && t + 2 < d.n_max) ? 1 : 0;
  }
}

// Tuning inputs: a fixed integer hash (splitmix64 finaliser) of (k, i) mapped
// to [-1, 1).  Not part of the method.
__global__ __launch_bounds__(256) void k_fill_random(float *out, int64_t n, uint32_t k) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t z = ((uint64_t)k << 40) ^ (uint64_t)i;
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[i] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
  }
}

int batch_cols_per_qw(bool tv_f64) { return tv_f64 ? 16 * 2 : 8 * 4; }

// Kernel shape of bucket k (1..5: basis sizes up to 32, 64, 128, 256, 512
// columns).  FP32 basis: 1 and 2 wavefronts with 8 groups for k = 1, 2, 4
// wavefronts with 8 groups for k = 3, then 8 wavefronts with 8 and 16 groups
// (16 wavefronts of 8 groups, the single push's choice above 320 columns,
// measured 0.5-1.5% slower here over the whole run);
// FP64 basis: 16 wavefronts with 1 .. 16 groups, 16 groups without prefetch.
// Up to 32 columns a panel carries too little data to pay for the
// cross-wavefront reduction and barriers of a wider workgroup: one-wavefront
// workgroups (16 per CU) keep many more panels in flight (single-stream
// passes at 4, 8, 16 and 32 columns: 1.85, 1.49, 1.24 and 1.08 times the
// rate of 4-wavefront workgroups); at 33-64 columns 2-wavefront workgroups of
// 8 groups took the batched run's steps there from 55.4 to 51.6 ms.
template <typename TV, typename TX, int MODE, int BK>
static hipError_t launch_bucket(int grid, const BatchArgs &b, hipStream_t s) {
  if constexpr (sizeof(TV) == 8) {
    constexpr int QW = 1 << (BK - 1);
    constexpr bool PREF = QW < 16;
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 16, QW, MODE, PREF, BK>), dim3(grid), dim3(16 * 64), 0, s, b);
  } else if constexpr (BK == 1) {
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 1, 8, MODE, true, BK>), dim3(grid), dim3(64), 0, s, b);
  } else if constexpr (BK == 2) {
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 2, 8, MODE, true, BK>), dim3(grid), dim3(128), 0, s, b);
  } else if constexpr (BK <= 3) {
    constexpr int QW = 2 << (BK - 1);
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 4, QW, MODE, true, BK>), dim3(grid), dim3(4 * 64), 0, s, b);
  } else {
    constexpr int QW = BK == 4 ? 8 : 16;
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 8, QW, MODE, true, BK>), dim3(grid), dim3(8 * 64), 0, s, b);
  }
  return hipGetLastError();
}

template <typename TV, typename TX, int MODE>
static hipError_t launch_bucket_k(int k, int grid, const BatchArgs &b, hipStream_t s) {
  switch (k) {
    case 1: return launch_bucket<TV, TX, MODE, 1>(grid, b, s);
    case 2: return launch_bucket<TV, TX, MODE, 2>(grid, b, s);
    case 3: return launch_bucket<TV, TX, MODE, 3>(grid, b, s);
    case 4: return launch_bucket<TV, TX, MODE, 4>(grid, b, s);
    case 5: return launch_bucket<TV, TX, MODE, 5>(grid, b, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TV, typename TX>
static hipError_t launch_batch_t(int mode, int k, int grid, const BatchArgs &b, hipStream_t s) {
  constexpr int NWI = sizeof(TV) == 8 ? 16 : 8;
  switch (mode) {
    case PM_INIT:
      hipLaunchKernelGGL((k_pass_batch<TV, TX, NWI, 1, PM_INIT, false, 0>), dim3(grid), dim3(NWI * 64), 0, s, b);
      return hipGetLastError();
    case PM_A: return launch_bucket_k<TV, TX, PM_A>(k, grid, b, s);
    case PM_B: return launch_bucket_k<TV, TX, PM_B>(k, grid, b, s);
    default: return launch_bucket_k<TV, TX, PM_C>(k, grid, b, s);
  }
}

hipError_t launch_batch_pass(int mode, bool tv_f64, bool tx_f64, int k, int grid, const BatchArgs &b,
                             hipStream_t s) {
  if (tv_f64)
    return tx_f64 ? launch_batch_t<double, double>(mode, k, grid, b, s)
                  : launch_batch_t<double, float>(mode, k, grid, b, s);
  return tx_f64 ? launch_batch_t<float, double>(mode, k, grid, b, s)
                : launch_batch_t<float, float>(mode, k, grid, b, s);
}

// ---------------------------------------------------------------------------
// Persistent step: one launch runs passes A, B and C, their reductions, the
// finalize and the next partial beta column of every stream whose basis has
// 1..kPersistCols columns.
//
// Groups: the streams are split into one contiguous group per XCD, balanced
// by bytes (panels x (j + 1)), and a workgroup works only on the group of
// the XCD it runs on (hardware XCC id), so each barrier involves the
// workgroups of one XCD.  Partial sums, reduced coefficients and the other
// values handed between workgroups inside the launch are stored and loaded
// at device scope (they bypass the non-coherent caches; a plain store is
// not seen by a workgroup on the same XCD that holds the line in its L2),
// so a barrier needs no cache write-back or invalidation.
//
// Phases, as in the bucket launches but separated by group barriers instead
// of kernel boundaries: pass A | reduce A | pass B | reduce B | pass C |
// finalize + next b.  In a pass, the group's concatenated panels are cut
// into G equal contiguous ranges (G = min(workgroups per XCD, panels /
// p_unit)); the workgroup of arrival rank r on its XCD takes range r and
// writes its partial sums for a stream to slot r - seg0 of that stream.
// Reductions take (stream, 8-column block) tasks r, r + G, ...; finalize and
// next b take streams r, r + G, ...  A barrier waits until all G ranks have
// finished the phase.  Ranks need G workgroups on the XCD, resident at once
// (the launch is sized to the resident complement); waits are bounded, and
// the last workgroup to finish checks that all G ranks of every group ran
// to the end: either failure sets the error flag, which the host reports.
// ---------------------------------------------------------------------------

__device__ inline int xcc_id() {
  // hardware register XCC_ID (20), bits 3:0: the XCD the wavefront runs on
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15);
}

__global__ void k_xcc_probe(unsigned *mask) {
  if (threadIdx.x == 0) atomicOr(mask, 1u << xcc_id());
}

__device__ inline bool persist_eligible(const DevState *st) {
  return st->act && st->jstep >= 1 && st->jstep <= kPersistCols;
}

// Plan of the persistent step, one workgroup, three sweeps over the streams:
// totals; the eligible list (stream order) with its panel prefix and the
// group of each stream (by the middle of its byte range); per stream its
// ranks (seg0, nseg), per group and rank its first list position.
__global__ __launch_bounds__(1024) void k_persist_plan(BatchArgs b) {
  __shared__ int s_wc[16];
  __shared__ int64_t s_wp[16], s_ww[16];
  __shared__ int s_cbase;
  __shared__ int64_t s_pbase, s_wbase, s_wtot;
  __shared__ int s_glo[kMaxGroups], s_ghi[kMaxGroups], s_gj[kMaxGroups];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NG = b.p_groups;
  int *ctl = b.p_ctl;
  if (tid < kMaxGroups) {
    s_glo[tid] = INT_MAX;
    s_ghi[tid] = 0;
    s_gj[tid] = 0;
  }
  if (tid == 0) s_wtot = 0;
  for (int sweep = 0; sweep < 2; ++sweep) {
    if (tid == 0) {
      s_cbase = 0;
      s_pbase = 0;
      s_wbase = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < b.S; c0 += 1024) {
      const int s = c0 + tid;
      int f = 0, j = 0;
      int64_t P = 0, w = 0;
      if (s < b.S) {
        const BatchStream &d = b.streams[s];
        if (persist_eligible(d.st)) {
          f = 1;
          j = d.st->jstep;
          P = d.P;
          w = P * (j + 1);
        }
      }
      int fi = f;
      int64_t pi = P, wi = w;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int tf = __shfl_up(fi, o, 64);
        const int64_t tp = __shfl_up(pi, o, 64), tw = __shfl_up(wi, o, 64);
        if (lane >= o) {
          fi += tf;
          pi += tp;
          wi += tw;
        }
      }
      if (lane == 63) {
        s_wc[wave] = fi;
        s_wp[wave] = pi;
        s_ww[wave] = wi;
      }
      __syncthreads();
      if (sweep == 1 && f) {
        int wc = 0;
        int64_t wp = 0, ww = 0;
        for (int q = 0; q < wave; ++q) {
          wc += s_wc[q];
          wp += s_wp[q];
          ww += s_ww[q];
        }
        const int pos = s_cbase + wc + fi - 1;
        const int64_t pfirst = s_pbase + wp + pi - P;
        const int64_t wfirst = s_wbase + ww + wi - w;
        int g = (int)(((2 * wfirst + w) * NG) / (2 * s_wtot));  // group of the stream's middle byte
        g = g < NG - 1 ? g : NG - 1;
        b.p_list[pos] = s;
        b.p_pre[pos] = pfirst;
        b.p_sgrp[pos] = g;
        b.streams[s].st->pers = 1;
        atomicMin(&s_glo[g], pos);
        atomicMax(&s_ghi[g], pos + 1);
        atomicMax(&s_gj[g], j);
      }
      __syncthreads();
      if (tid == 0) {
        int tc = 0;
        int64_t tp = 0, tw = 0;
        for (int q = 0; q < 16; ++q) {
          tc += s_wc[q];
          tp += s_wp[q];
          tw += s_ww[q];
        }
        s_cbase += tc;
        s_pbase += tp;
        s_wbase += tw;
      }
      __syncthreads();
    }
    if (tid == 0) {
      s_wtot = s_wbase;
      if (sweep == 1) b.p_pre[s_cbase] = s_pbase;
    }
    __syncthreads();
  }
  // per group: list range, panels, ranks, column blocks; counters reset
  const int W = b.p_ranks;
  if (tid < kMaxGroups) {
    int *gc = ctl + kCtlGroup0 + kCtlGroupStride * tid;
    const int lo = s_glo[tid] < s_ghi[tid] ? s_glo[tid] : 0;
    const int hi = s_glo[tid] < s_ghi[tid] ? s_ghi[tid] : 0;
    const int64_t T = b.p_pre[hi] - b.p_pre[lo];
    int G = 0;
    if (hi > lo && tid < NG) {
      const int64_t gg = T / b.p_unit;
      G = (int)(gg < 1 ? 1 : (gg > W ? W : gg));
    }
    gc[kGcLo] = lo;
    gc[kGcCnt] = hi - lo;
    gc[kGcRanks] = G;
    gc[kGcBlocks] = (s_gj[tid] + 1 + kPersistNW - 1) / kPersistNW;
    gc[kGcArrive] = 0;
    for (int q = 0; q < kGcPhases; ++q) gc[kGcBar + q] = 0;
    gc[kGcDone] = 0;
  }
  if (tid == 0) {
    ctl[kCtlExit] = 0;
    ctl[kCtlStreams] = s_cbase;
  }
  __syncthreads();
  // per eligible stream: its ranks; per (group, rank): first list position
  const int E = s_cbase;
  for (int pos = tid; pos < E; pos += 1024) {
    const int g = b.p_sgrp[pos];
    const int *gc = ctl + kCtlGroup0 + kCtlGroupStride * g;
    const int lo = gc[kGcLo], G = gc[kGcRanks];
    const int64_t base = b.p_pre[lo], T = b.p_pre[lo + gc[kGcCnt]] - base;
    const int64_t p0 = b.p_pre[pos] - base, p1 = b.p_pre[pos + 1] - base;
    DevState *st = b.streams[b.p_list[pos]].st;
    const int g0 = (int)(((p0 + 1) * G - 1) / T);
    const int g1 = (int)((p1 * G - 1) / T);
    st->seg0 = g0;
    st->nseg = g1 - g0 + 1;
  }
  for (int q = tid; q < NG * kMaxRanks; q += 1024) {
    const int g = q / kMaxRanks, r = q - g * kMaxRanks;
    const int *gc = ctl + kCtlGroup0 + kCtlGroupStride * g;
    const int G = gc[kGcRanks];
    if (r >= G) continue;
    const int lo = gc[kGcLo], cnt = gc[kGcCnt];
    const int64_t base = b.p_pre[lo], T = b.p_pre[lo + cnt] - base;
    const int64_t start = base + (int64_t)r * T / G;
    int a = lo, c = lo + cnt - 1;  // largest list position i with pre[i] <= start
    while (a < c) {
      const int m = (a + c + 1) / 2;
      if (b.p_pre[m] <= start)
        a = m;
      else
        c = m - 1;
    }
    b.p_first[q] = a;
  }
}

constexpr int kPersistThreads = kPersistNW * 64;

// Everything one workgroup hands to another inside the launch goes through
// device-scope stores and loads (xst / xld), so a barrier needs no cache
// maintenance: release = every wavefront waits until its stores are
// complete (the asm statement also keeps the compiler from moving stores
// past it), then the workgroup syncs.
__device__ inline void wg_release() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// Group barrier: this workgroup's phase is done (release, count), then wait
// (one lane polls, relaxed, with sleeps) until all G ranks have counted.
// False, with the error flag set, at the bound or when an earlier wait
// already failed.
__device__ inline bool group_barrier(int *cnt, int G, int *err, int spin, int *s_ok) {
  wg_release();
  if (threadIdx.x == 0) {
    atomicAdd(cnt, 1);
    int ok = 0;
    for (int it = 0; it < spin; ++it) {
      if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= G) {
        ok = 1;
        break;
      }
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok) atomicOr(err, 1);
    *s_ok = ok;
  }
  __syncthreads();
  const int ok = *s_ok;
  __syncthreads();
  return ok != 0;
}

template <typename TX, int MODE>
__device__ inline void persist_pass(int qw, const PassArgs &a, int64_t lo, int64_t hi, int slot, double *lds) {
  static_assert(pass_lds_doubles<float, kPersistNW, 8, MODE>() <= pass_lds_doubles<float, kPersistNW, 8, PM_C>() &&
                    pass_lds_doubles<float, kPersistNW, 1, MODE>() <= pass_lds_doubles<float, kPersistNW, 8, PM_C>(),
                "persistent step LDS");
  switch (qw) {
    case 1: row_pass_body<float, TX, kPersistNW, 1, MODE, true, true>(a, lo, hi, 1, slot, lds); break;
    case 2: row_pass_body<float, TX, kPersistNW, 2, MODE, true, true>(a, lo, hi, 1, slot, lds); break;
    case 4: row_pass_body<float, TX, kPersistNW, 4, MODE, true, true>(a, lo, hi, 1, slot, lds); break;
    default: row_pass_body<float, TX, kPersistNW, 8, MODE, true, true>(a, lo, hi, 1, slot, lds); break;
  }
}

// Range `rank` of the group's concatenated panels, pass MODE.
template <typename TX, int MODE>
__device__ inline void persist_range(const BatchArgs &b, const int *gc, int rank, int g, double *lds) {
  const int lo_pos = uniform(gc[kGcLo]), cnt = uniform(gc[kGcCnt]), G = uniform(gc[kGcRanks]);
  const int64_t base = uniform(b.p_pre[lo_pos]);
  const int64_t T = uniform(b.p_pre[lo_pos + cnt]) - base;
  int64_t lo = base + (int64_t)rank * T / G;
  const int64_t hi = base + (int64_t)(rank + 1) * T / G;
  int i = uniform(b.p_first[g * kMaxRanks + rank]);
  while (lo < hi) {
    const int s = uniform(b.p_list[i]);
    const int64_t ps = uniform(b.p_pre[i]), pe = uniform(b.p_pre[i + 1]);
    const int64_t e = pe < hi ? pe : hi;
    const BatchStream &d = b.streams[s];
    const DevState *st = uniform(d.st);
    PassArgs a{};
    a.W = uniform(d.W);
    a.x = uniform(b.xptrs[s]);
    a.w = uniform(d.w);
    a.coef[0] = uniform(d.coefA);
    a.coef[1] = uniform(d.coefB);
    a.coef[2] = uniform(d.coefC);
    a.st = st;
    a.part = uniform(d.part);
    a.partn = uniform(d.partn);
    a.n = uniform(d.n);
    a.P = uniform(d.P);
    a.j = uniform(st->jstep);
    a.n_max = uniform(d.n_max);
    a.ldg = uniform(d.ldg);
    const int j = a.j;
    const int qw = j <= 32 ? 1 : (j <= 64 ? 2 : (j <= 128 ? 4 : 8));
    persist_pass<TX, MODE>(qw, a, lo - ps, e - ps, rank - uniform(st->seg0), lds);
    lo = e;
    ++i;
  }
}

template <typename TX>
__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_step_persist(BatchArgs b) {
  __shared__ double lds[pass_lds_doubles<float, kPersistNW, 8, PM_C>()];
  __shared__ int s_rank, s_ok;
  int *ctl = b.p_ctl;
  int *err = ctl + kCtlErr;
  const int spin = b.p_spin;
  const int g = (int)((b.p_xmap >> (4 * xcc_id())) & 15);
  if (g < b.p_groups) {
    int *gc = ctl + kCtlGroup0 + kCtlGroupStride * g;
    const int G = uniform(gc[kGcRanks]);
    if (threadIdx.x == 0) s_rank = atomicAdd(gc + kGcArrive, 1);
    __syncthreads();
    const int rank = uniform(s_rank);
    if (rank < G) {
      const int lo_pos = uniform(gc[kGcLo]), cnt = uniform(gc[kGcCnt]), CB = uniform(gc[kGcBlocks]);
      bool ok = true;
      for (int ph = 0; ph < 3 && ok; ++ph) {
        if (ph == 0)
          persist_range<TX, PM_A>(b, gc, rank, g, lds);
        else if (ph == 1)
          persist_range<TX, PM_B>(b, gc, rank, g, lds);
        else
          persist_range<TX, PM_C>(b, gc, rank, g, lds);
        ok = group_barrier(gc + kGcBar + 2 * ph, G, err, spin, &s_ok);
        if (!ok || ph == 2) break;
        // reduce of pass ph: (stream, 8-column block) tasks rank, rank + G, ...
        for (int t = rank; t < cnt * CB; t += G) {
          const int i = t / CB, cb = t - i * CB;
          const BatchStream &d = b.streams[uniform(b.p_list[lo_pos + i])];
          const SmallArgs sa = small_of(d);
          if (ph == 0)
            reduce_body<1, true>(sa, cb * kPersistNW);
          else
            reduce_body<2, true>(sa, cb * kPersistNW);
        }
        ok = group_barrier(gc + kGcBar + 2 * ph + 1, G, err, spin, &s_ok);
      }
      if (ok) {
        // finalize and next b: streams rank, rank + G, ...
        for (int i = rank; i < cnt; i += G) {
          const BatchStream &d = b.streams[uniform(b.p_list[lo_pos + i])];
          const SmallArgs sa = small_of(d);
          finalize_body_t<kPersistThreads, true>(sa);
          __syncthreads();
          const int J = uniform(d.st->q);
          for (int c = 0; c * 64 < J; c += kPersistThreads / 256) {
            nextb_body_t<kPersistThreads>(sa, c);
            __syncthreads();
          }
        }
        if (threadIdx.x == 0) atomicAdd(gc + kGcDone, 1);
      }
    }
  }
  // the last workgroup to finish checks that every group completed its ranks
  // (the finished-rank count is complete before the exit count is taken:
  // two relaxed atomics to different addresses may otherwise land in either
  // order)
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_s_waitcnt(0);
  if (threadIdx.x == 0 && atomicAdd(ctl + kCtlExit, 1) == (int)gridDim.x - 1) {
    for (int q = 0; q < b.p_groups; ++q) {
      int *gq = ctl + kCtlGroup0 + kCtlGroupStride * q;
      if (__hip_atomic_load(gq + kGcDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gq[kGcRanks])
        atomicOr(err, 2);
    }
  }
}

template <typename F>
static int occ_of(F f, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(f), threads, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <typename TV, int BK>
static int occ_bucket() {
  if constexpr (sizeof(TV) == 8) {
    constexpr int QW = 1 << (BK - 1);
    return occ_of(&k_pass_batch<TV, float, 16, QW, PM_A, (QW < 16), BK>, 16 * 64);
  } else if constexpr (BK == 1) {
    return occ_of(&k_pass_batch<TV, float, 1, 8, PM_A, true, BK>, 64);
  } else if constexpr (BK == 2) {
    return occ_of(&k_pass_batch<TV, float, 2, 8, PM_A, true, BK>, 128);
  } else if constexpr (BK <= 3) {
    return occ_of(&k_pass_batch<TV, float, 4, (2 << (BK - 1)), PM_A, true, BK>, 4 * 64);
  } else {
    return occ_of(&k_pass_batch<TV, float, 8, (BK == 4 ? 8 : 16), PM_A, true, BK>, 8 * 64);
  }
}

template <typename TV>
static int occ_batch_k(int k) {
  constexpr int NWI = sizeof(TV) == 8 ? 16 : 8;
  switch (k) {
    case 0: return occ_of(&k_pass_batch<TV, float, NWI, 1, PM_INIT, false, 0>, NWI * 64);
    case 1: return occ_bucket<TV, 1>();
    case 2: return occ_bucket<TV, 2>();
    case 3: return occ_bucket<TV, 3>();
    case 4: return occ_bucket<TV, 4>();
    default: return occ_bucket<TV, 5>();
  }
}

int batch_pass_occupancy(bool tv_f64, int k) { return tv_f64 ? occ_batch_k<double>(k) : occ_batch_k<float>(k); }

int step_persist_occupancy() { return occ_of(&k_step_persist<float>, kPersistThreads); }

hipError_t launch_xcc_probe(unsigned *mask, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(blocks), dim3(64), 0, s, mask);
  return hipGetLastError();
}

hipError_t launch_persist_plan(const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_persist_plan, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_step_persist(bool tx_f64, int grid, const BatchArgs &b, hipStream_t s) {
  if (tx_f64)
    hipLaunchKernelGGL(k_step_persist<double>, dim3(grid), dim3(kPersistThreads), 0, s, b);
  else
    hipLaunchKernelGGL(k_step_persist<float>, dim3(grid), dim3(kPersistThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_plan(const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(int mode, const BatchArgs &b, hipStream_t s) {
  if (mode == 1)
    hipLaunchKernelGGL(k_reduce_batch<1>, dim3(b.n_rblocks), dim3(256), 0, s, b);
  else
    hipLaunchKernelGGL(k_reduce_batch<2>, dim3(b.n_rblocks), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_batch, dim3(b.S), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_nextb(const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_nextb_batch, dim3((b.max_nmax + 64) / 64, b.S), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_init_states(const BatchArgs &b, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init_states, dim3(4, b.S), dim3(256), 0, s, b, tol);
  return hipGetLastError();
}

hipError_t launch_tune_states(const BatchArgs &b, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_tune_states, dim3((b.S + 255) / 256), dim3(256), 0, s, b, t);
  return hipGetLastError();
}

hipError_t launch_fill_random(float *out, int64_t n, uint32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_random, dim3(256), dim3(256), 0, s, out, n, k);
  return hipGetLastError();
}

}  // namespace foa
