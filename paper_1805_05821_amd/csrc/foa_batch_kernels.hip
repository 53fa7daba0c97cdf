// Batched form of the FOA push (Algorithm 1 steps 5-18 for many independent
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

// Step state and bucket lists, one workgroup of 1024 threads.  Streams are
// taken 1024 at a time; per bucket a wavefront prefix sum (count and panels)
// plus the per-wavefront totals give each active stream its list position
// and panel offset.
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
      const bool offered = b.xptrs[s] != nullptr;
      const int j = st->q;
      const bool room = j < d.n_max;
      const int act = (st->status == ST_ACTIVE && offered && room) ? 1 : 0;
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
  }
}

// Workgroup g of bucket k covers panels [g T / G, (g + 1) T / G) of the
// bucket's concatenation; the workgroup holding panel p is
// ((p + 1) G - 1) / T.  Blocks 0..NBUCKET-1: first stream of every
// workgroup (binary search in the prefix); the rest: per stream, its first
// workgroup and the number of workgroups (partial slots) on it.
__global__ __launch_bounds__(256) void k_batch_plan_ranges(BatchArgs b) {
  if (blockIdx.x < NBUCKET) {
    const int k = blockIdx.x;
    const int cnt = b.meta[2 * k], G = b.meta[2 * k + 1];
    const int64_t *pre = b.pre + (size_t)k * (b.S + 1);
    const int64_t T = uniform(pre[cnt]);
    for (int g = threadIdx.x; g < G; g += 256) {
      const int64_t lo = (int64_t)g * T / G;
      int a = 0, c = cnt - 1;  // largest i with pre[i] <= lo
      while (a < c) {
        const int m = (a + c + 1) / 2;
        if (pre[m] <= lo)
          a = m;
        else
          c = m - 1;
      }
      b.first[k * kMaxBatchGrid + g] = a;
    }
    return;
  }
  const int s = (blockIdx.x - NBUCKET) * 256 + threadIdx.x;
  if (s >= b.S) return;
  DevState *st = b.streams[s].st;
  if (!st->act) return;
  const int code = b.spos[s];
  const int k = code >> 24, pos = code & 0xFFFFFF;
  const int cnt = b.meta[2 * k], G = b.meta[2 * k + 1];
  const int64_t *pre = b.pre + (size_t)k * (b.S + 1);
  const int64_t T = pre[cnt];
  const int64_t p0 = pre[pos], p1 = pre[pos + 1];
  const int g0 = (int)(((p0 + 1) * G - 1) / T);
  const int g1 = (int)((p1 * G - 1) / T);
  st->seg0 = g0;
  st->nseg = g1 - g0 + 1;
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
// columns).  FP32 basis: 4 wavefronts with 2, 4, 8 groups for k <= 3, then 8
// wavefronts with 8 and 16 groups (the single push's automatic choice); FP64
// basis: 16 wavefronts with 1 .. 16 groups, 16 groups without prefetch.
template <typename TV, typename TX, int MODE, int BK>
static hipError_t launch_bucket(int grid, const BatchArgs &b, hipStream_t s) {
  if constexpr (sizeof(TV) == 8) {
    constexpr int QW = 1 << (BK - 1);
    constexpr bool PREF = QW < 16;
    hipLaunchKernelGGL((k_pass_batch<TV, TX, 16, QW, MODE, PREF, BK>), dim3(grid), dim3(16 * 64), 0, s, b);
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
// 1..kPersistCols columns.  Work items are (pass, stream, chunk of panels).
//
// Queues: the streams are split into one contiguous group per XCD (by chunk
// count, so by bytes: chunks hold about the same bytes at every basis width,
// panels scale with 64/(j+1)), and a workgroup takes items only from the
// queue of the XCD it runs on (hardware XCC id).  Every exchange between
// workgroups of one stream -- chunk partials, reduced coefficients, the
// work vectors -- therefore stays inside one L2, where a release is the
// completion of the stores (the vector L1 writes through) and an acquire is
// an invalidation of the L1; no L2 write-back or invalidation is needed
// until the kernel ends.
//
// Within a queue, items are numbered pass-major and taken from an atomic
// counter; each workgroup fetches its next item while it runs the current
// one.  A pass B or C item waits until its stream's previous pass is
// reduced; the items of that pass have smaller numbers, so they were taken
// earlier by running workgroups of the same XCD, and a workgroup only ever
// holds items in increasing order: the smallest unfinished item always has
// every dependency done, so every wait ends.  The workgroup that finishes a
// stream's last chunk of a pass reduces the pass (after C: finalize and the
// next b).  Partial sums go to slot = chunk, reduced in slot order, so the
// results do not depend on which workgroup ran what.  Waits are bounded,
// and the last workgroup to finish checks that every queue completed all of
// its streams (a queue whose XCD received no workgroup would not): either
// failure sets the error flag, which the host reports as a device error.
// ---------------------------------------------------------------------------

__device__ inline int xcc_id() {
  // hardware register XCC_ID (20), bits 3:0: the XCD the wavefront runs on
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15);
}

__global__ void k_xcc_probe(unsigned *mask) {
  if (threadIdx.x == 0) atomicOr(mask, 1u << xcc_id());
}

// Plan of the persistent step, one workgroup, two sweeps over the streams:
// the total chunk count, then the chunk descriptors in stream order, the
// queue of each stream and each queue's range; sync words reset.
__global__ __launch_bounds__(1024) void k_persist_plan(BatchArgs b) {
  __shared__ int s_wsum[16];
  __shared__ int s_base, s_total;
  __shared__ int s_glo[kMaxGroups], s_ghi[kMaxGroups], s_gcnt[kMaxGroups];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = b.p_groups;
  if (tid < kMaxGroups) {
    s_glo[tid] = INT_MAX;
    s_ghi[tid] = 0;
    s_gcnt[tid] = 0;
  }
  if (tid == 0) s_total = 0;
  for (int sweep = 0; sweep < 2; ++sweep) {
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < b.S; c0 += 1024) {
      const int s = c0 + tid;
      int m = 0, chunk = kMinChunk, j = 0;
      if (s < b.S) {
        const BatchStream &d = b.streams[s];
        const DevState *st = d.st;
        j = st->jstep;
        if (st->act && j >= 1 && j <= kPersistCols) {
          const int c = (int)((64LL * b.p_unit) / (j + 1));
          chunk = c > kMinChunk ? c : kMinChunk;
          m = (int)((d.P + chunk - 1) / chunk);
        }
      }
      int mi = m;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int tm = __shfl_up(mi, o, 64);
        if (lane >= o) mi += tm;
      }
      if (lane == 63) s_wsum[wave] = mi;
      __syncthreads();
      if (sweep == 1 && s < b.S) {
        int *sy = b.p_sync + 4 * (size_t)s;
        sy[0] = 0;
        sy[1] = 0;
        sy[2] = 0;
        sy[3] = 0;
        if (m > 0) {
          int wm = 0;
          for (int w = 0; w < wave; ++w) wm += s_wsum[w];
          const int first = s_base + wm + mi - m;
          int g = (int)(((2LL * first + m) * G) / (2LL * s_total));  // queue of the stream's middle chunk
          g = g < G - 1 ? g : G - 1;
          b.streams[s].st->pers = 1;
          for (int c = 0; c < m; ++c) {
            PersistTask tk{};
            tk.s = s;
            tk.chunk = c;
            tk.m = m;
            tk.cp = chunk;
            tk.j = j;
            b.p_task[first + c] = tk;
          }
          atomicMin(&s_glo[g], first);
          atomicMax(&s_ghi[g], first + m);
          atomicAdd(&s_gcnt[g], 1);
        }
      }
      __syncthreads();
      if (tid == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += s_wsum[w];
        s_base += t;
      }
      __syncthreads();
    }
    if (tid == 0) s_total = s_base;
    __syncthreads();
  }
  if (tid < kMaxGroups) {
    int *gc = b.p_ctl + kCtlGroup0 + kCtlGroupStride * tid;
    const int lo = s_glo[tid], hi = s_ghi[tid];
    gc[0] = 0;                       // next item
    gc[1] = lo < hi ? hi - lo : 0;   // chunks per pass
    gc[2] = lo < hi ? lo : 0;        // first chunk
    gc[3] = s_gcnt[tid];             // streams
    gc[4] = 0;                       // streams completed
  }
  if (tid == 0) {
    b.p_ctl[1] = s_total;
    b.p_ctl[kCtlExit] = 0;
  }
}

constexpr int kPersistNW = 8;
constexpr int kPersistThreads = kPersistNW * 64;
constexpr int kPersistSpin = 1 << 22;  // polls of a wait before it gives up

// Release / acquire between workgroups on one XCD.  Release: every wavefront
// waits until its stores are complete in L2, then the workgroup syncs.
// Acquire: one lane invalidates the CU's vector L1 (shared by the whole
// workgroup), then the workgroup syncs; later loads read L2.
__device__ inline void wg_release_xcd() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}
__device__ inline void wg_acquire_xcd() {
  if (threadIdx.x == 0) {
    asm volatile("buffer_inv sc0" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
}

// Wait (one lane polls, relaxed, with sleeps) until *flag >= want; false,
// with the error flag set, at the bound or when an earlier wait already
// failed.  Acquire on success.
__device__ inline bool persist_wait(int *flag, int want, int *err, int *s_ok) {
  if (threadIdx.x == 0) {
    int ok = 0;
    for (int it = 0; it < kPersistSpin; ++it) {
      if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) {
        ok = 1;
        break;
      }
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      __builtin_amdgcn_s_sleep(8);
    }
    if (!ok) atomicOr(err, 1);
    *s_ok = ok;
  }
  __syncthreads();
  const int ok = *s_ok;
  if (ok) wg_acquire_xcd();  // the reduced coefficients are read after this
  __syncthreads();
  return ok != 0;
}

template <typename TX, int MODE>
__device__ inline void persist_pass(int qw, const PassArgs &a, int64_t lo, int64_t hi, int slot, double *lds) {
  static_assert(pass_lds_doubles<float, kPersistNW, 8, MODE>() <= pass_lds_doubles<float, kPersistNW, 8, PM_C>() &&
                    pass_lds_doubles<float, kPersistNW, 1, MODE>() <= pass_lds_doubles<float, kPersistNW, 8, PM_C>(),
                "persistent step LDS");
  switch (qw) {
    case 1: row_pass_body<float, TX, kPersistNW, 1, MODE, true>(a, lo, hi, 1, slot, lds); break;
    case 2: row_pass_body<float, TX, kPersistNW, 2, MODE, true>(a, lo, hi, 1, slot, lds); break;
    case 4: row_pass_body<float, TX, kPersistNW, 4, MODE, true>(a, lo, hi, 1, slot, lds); break;
    default: row_pass_body<float, TX, kPersistNW, 8, MODE, true>(a, lo, hi, 1, slot, lds); break;
  }
}

template <typename TX>
__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_step_persist(BatchArgs b) {
  __shared__ double lds[pass_lds_doubles<float, kPersistNW, 8, PM_C>()];
  __shared__ int s_t, s_last, s_ok;
  int *ctl = b.p_ctl;
  const int g = (int)((b.p_xmap >> (4 * xcc_id())) & 15);
  if (g < b.p_groups) {
    int *gc = ctl + kCtlGroup0 + kCtlGroupStride * g;
    const int M = uniform(gc[1]);
    const int base = uniform(gc[2]);
    if (threadIdx.x == 0) s_t = atomicAdd(gc, 1);
    __syncthreads();
    int t = uniform(s_t);
    while (t < 3 * M) {
      __syncthreads();  // every wavefront has read s_t
      int nxt = 0;      // the next work item, fetched while this one runs
      if (threadIdx.x == 0) nxt = atomicAdd(gc, 1);
      const int ph = t / M;
      const PersistTask *tp = b.p_task + base + (t - ph * M);
      const int s = uniform(tp->s);
      const int chunk = uniform(tp->chunk);
      const int m = uniform(tp->m);
      const int cp = uniform(tp->cp);
      const int j = uniform(tp->j);
      int *sy = b.p_sync + 4 * (size_t)s;
      if (ph == 0 || persist_wait(sy + 3, ph, ctl + kCtlErr, &s_ok)) {
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
        a.j = j;
        a.n_max = uniform(d.n_max);
        a.ldg = uniform(d.ldg);
        const int qw = j <= 32 ? 1 : (j <= 64 ? 2 : (j <= 128 ? 4 : 8));
        const int64_t plo = (int64_t)chunk * cp;
        const int64_t phi = plo + cp < a.P ? plo + cp : a.P;
        if (ph == 0)
          persist_pass<TX, PM_A>(qw, a, plo, phi, chunk, lds);
        else if (ph == 1)
          persist_pass<TX, PM_B>(qw, a, plo, phi, chunk, lds);
        else
          persist_pass<TX, PM_C>(qw, a, plo, phi, chunk, lds);
        wg_release_xcd();  // this chunk's partial sums (and work vectors) before the count
        if (threadIdx.x == 0) s_last = (atomicAdd(sy + ph, 1) == m - 1) ? 1 : 0;
        __syncthreads();
        if (s_last) {
          wg_acquire_xcd();  // every chunk's partial sums are visible after this
          SmallArgs sa = small_of(d);
          sa.G = m;
          sa.j = j;
          if (ph == 0) {
            for (int c = 0; c <= j; c += kPersistNW) reduce_body<1>(sa, c);
          } else if (ph == 1) {
            for (int c = 0; c < j; c += kPersistNW) reduce_body<2>(sa, c);
          } else {
            finalize_body_t<kPersistThreads>(sa);
            __syncthreads();
            const int J = uniform(d.st->q);
            for (int c = 0; c * 64 < J; c += kPersistThreads / 256) {
              nextb_body_t<kPersistThreads>(sa, c);
              __syncthreads();
            }
          }
          wg_release_xcd();
          if (threadIdx.x == 0) {
            __hip_atomic_store(sy + 3, ph + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ph == 2) atomicAdd(gc + 4, 1);
          }
        }
      }
      if (threadIdx.x == 0) s_t = nxt;
      __syncthreads();
      t = uniform(s_t);
    }
  }
  // the last workgroup to finish checks that every queue completed its streams
  __syncthreads();
  if (threadIdx.x == 0 && atomicAdd(ctl + kCtlExit, 1) == (int)gridDim.x - 1) {
    for (int q = 0; q < b.p_groups; ++q) {
      int *gq = ctl + kCtlGroup0 + kCtlGroupStride * q;
      if (__hip_atomic_load(gq + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
          __hip_atomic_load(gq + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicOr(ctl + kCtlErr, 2);
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
  hipLaunchKernelGGL(k_batch_plan_ranges, dim3(NBUCKET + (b.S + 255) / 256), dim3(256), 0, s, b);
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
