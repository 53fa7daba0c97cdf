// HIP kernels (gfx950) of one FOA push: Algorithm 1 steps 5-18 of
// Anantharamu & Mahesh, restructured as three fused row passes over the basis.
//
// The paper's literal schedule sweeps V five times per snapshot (steps 9, 10,
// 11, 12 and 14).  Each of steps (9,10), (11,12) and (14,15) is "apply a
// row-local update with coefficients known before the pass, then reduce over
// the rows", so one pass over V serves both halves; the two projections must
// finish globally before the next update, so three sweeps is the minimum for
// classical Gram-Schmidt with one reorthogonalisation.
//
//   pass A : w = (psi - V b) / beta_jj ; partial V^T w ; partial ||psi||^2
//   reduce : h = V^T w                           (step 10)
//   pass B : w = w - V h ; partial V^T w         (steps 11-12)
//   reduce : s = V^T w ; h = h + s               (step 13)
//   pass C : w = w - V s ; v_{j+1} <- w ; partial ||w||^2   (steps 14-15)
//   finalize: h_{j+1,j} = ||w||, breakdown test, H_bar column, beta column
//             (steps 15-18), then the next push's partial beta column
//             (steps 5-8, eq. betacolumnupdate) in a small multi-block kernel.
//
// The basis is stored unnormalised: column c holds fl(w_c) and
// v_c = sigma_c * column_c with sigma_c = 1 / h_{c,c-1} (sigma_1 = 1/beta_11).
// Every coefficient vector handed to a pass is pre-multiplied by sigma and every
// projection is post-multiplied by sigma, so step 15's division never needs its
// own sweep over n.  All dot products, norms and small-matrix arithmetic are FP64.
//
// Reductions are deterministic: every partial sum has a fixed association
// (per-lane register sums in panel order, butterfly within a wavefront, fixed
// per-block order); no floating-point atomics are used.

#include <math.h>

#include "foa_buffer.h"
#include "foa_internal.h"

namespace foa {

template <typename TV>
struct Vec {
  static constexpr int EPL = 16 / sizeof(TV);  // rows per lane per 16-byte load
};


__device__ __forceinline__ double xor_shfl(double v, int m) { return __shfl_xor(v, m, 64); }

template <typename T>
__device__ __forceinline__ double buf_load_scalar(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buf_load_scalar<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load_scalar<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store_scalar(T v, __amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ void buf_store_scalar<float>(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void buf_store_scalar<double>(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// Whole-vector bit casts only: casting a single element lvalue of an
// ext_vector (e.g. __builtin_bit_cast(float, v.y)) reads element 0.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename TV>
__device__ __forceinline__ void unpack16(const u32x4 &v, TV (&o)[16 / sizeof(TV)]);
template <>
__device__ __forceinline__ void unpack16<float>(const u32x4 &v, float (&o)[4]) {
  const f32x4 f = __builtin_bit_cast(f32x4, v);
  o[0] = f.x;
  o[1] = f.y;
  o[2] = f.z;
  o[3] = f.w;
}
template <>
__device__ __forceinline__ void unpack16<double>(const u32x4 &v, double (&o)[2]) {
  const f64x2 d = __builtin_bit_cast(f64x2, v);
  o[0] = d.x;
  o[1] = d.y;
}

// ---------------------------------------------------------------------------
// Fused row pass.
//
// Work decomposition: one workgroup walks panels blockIdx.x, +gridDim.x, ...
// Within a panel (64 rows x j columns), wavefront `wave` owns column groups
// g*NW + wave (g < QW); a group is the 1 KiB contiguous block of CPW columns
// read by one 16-byte load per lane.  Lane l holds rows EPL*(l % LPC) .. +EPL-1
// of column (group start) + l / LPC.
//   phase 1 (row sums  u_r = sum_c V_rc coef_c): per-lane FMA over its groups,
//            butterfly over the lanes sharing rows, then across wavefronts
//            through LDS in wavefront order;
//   update  (every wavefront, 64/NW rows each): w_r = (y_r - u_r) * scale;
//   phase 2 (column sums V^T w): per-lane FP64 accumulators that persist
//            across panels; one butterfly per column at the end.
// With PREF the next panel's tile is loaded while the current one is reduced.
// ---------------------------------------------------------------------------
// One workgroup processes panels pstart, pstart + pstep, ... < pend of one
// stream and writes its partial sums to slot `slot`.  Called uniformly by
// the whole workgroup (it synchronises).
template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF>
__device__ __forceinline__ void row_pass_body(const PassArgs &a, int64_t pstart, int64_t pend, int64_t pstep,
                                              int slot) {
  constexpr int EPL = Vec<TV>::EPL;
  constexpr int LPC = 64 / EPL;  // lanes per 64-row column segment
  constexpr int CPW = EPL;       // columns per wavefront load
  constexpr int JCAP = QW * NW * CPW;
  constexpr int RPW = PANEL / NW;  // rows updated by each wavefront
  constexpr bool HAS_P1 = (MODE != PM_INIT);
  constexpr bool HAS_P2 = (MODE == PM_A || MODE == PM_B);
  constexpr bool SRC_X = (MODE == PM_INIT || MODE == PM_A);
  constexpr int GSTRIDE = NW * CPW;  // columns between a wavefront's groups

  __shared__ double s_coef[JCAP];
  __shared__ double s_red[2][NW][PANEL];
  __shared__ double s_w[PANEL];
  __shared__ double s_nrm[NW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wavefront index made provably uniform so per-wave offsets stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cs = lane / LPC;
  const int rg = lane % LPC;
  const int j = a.j;

  __syncthreads();  // the previous call of this workgroup may still read LDS
  for (int c = tid; c < JCAP; c += NW * 64) s_coef[c] = (c < j) ? a.coef[c] : 0.0;
  const double scale = (MODE == PM_A) ? a.st->scaleA : 1.0;
  __syncthreads();

  const int cbase = wave * CPW + cs;  // column of this lane in group 0
  // byte offset of this lane's 16-byte fragment of group g: goff0 + g * GBYTES
  const unsigned goff0 = (unsigned)((wave * CPW * PANEL + lane * EPL) * sizeof(TV));
  constexpr unsigned GBYTES = (unsigned)(GSTRIDE * PANEL * sizeof(TV));
  const unsigned tile_bytes = (unsigned)(j * PANEL * sizeof(TV));
  // update rows: lane < RPW owns panel row urow; the others only carry values
  const bool uact = lane < RPW;
  const int urow = wave * RPW + (lane % RPW);

  double acc[QW];
#pragma unroll
  for (int g = 0; g < QW; ++g) acc[g] = 0.0;
  double nrm = 0.0;

  const char *Wb = static_cast<const char *>(a.W);
  const size_t pbytes = (size_t)a.n_max * PANEL * sizeof(TV);

  TV t[QW][EPL];
  TV tn[QW][EPL];

  // bytes = 0 turns every load into an out-of-range load returning 0 without
  // memory traffic (used past the last panel, so the loop has no branch
  // around its loads).
  auto load_tile = [&](int64_t p, TV (&dst)[QW][EPL], unsigned bytes) {
    if (!HAS_P1) return;
    const __amdgpu_buffer_rsrc_t rt = make_rsrc(Wb + (size_t)p * pbytes, bytes);
#pragma unroll
    for (int g = 0; g < QW; ++g) {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rt, (int)(goff0 + g * GBYTES), 0, 0);
      unpack16<TV>(v, dst[g]);
    }
  };

  int64_t p = pstart;
  if (PREF && p < pend) {
    load_tile(p, t, tile_bytes);
    // Complete the first tile before the loop: otherwise its pending loads
    // merge with the loop back edge and every iteration waits for the
    // prefetched tile before phase 1.
#pragma unroll
    for (int g = 0; g < QW; ++g) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
    }
  }
  int par = 0;
  for (; p < pend; p += pstep) {
    // y for the update rows of this wavefront (snapshot or work vector)
    double y;
    if (SRC_X) {
      const int64_t rem = a.n - p * PANEL;
      const unsigned xb = (unsigned)((rem >= PANEL ? PANEL : (rem > 0 ? rem : 0)) * sizeof(TX));
      const __amdgpu_buffer_rsrc_t rx = make_rsrc(static_cast<const TX *>(a.x) + p * PANEL, xb);
      y = buf_load_scalar<TX>(rx, uact ? (unsigned)(urow * sizeof(TX)) : kOOR);
    } else {
      const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.w + p * PANEL, PANEL * 8);
      y = buf_load_scalar<double>(rw, uact ? (unsigned)(urow * 8) : kOOR);
    }
    if (PREF) {
      const bool more = p + pstep < pend;
      load_tile(more ? p + pstep : p, tn, more ? tile_bytes : 0u);
    } else {
      load_tile(p, t, tile_bytes);
    }

    if (HAS_P1) {
      double u[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) u[e] = 0.0;
#pragma unroll
      for (int g = 0; g < QW; ++g) {
        const double cf = s_coef[cbase + g * GSTRIDE];
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[e] = fma((double)t[g][e], cf, u[e]);
      }
#pragma unroll
      for (int m = LPC; m < 64; m <<= 1) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[e] += xor_shfl(u[e], m);
      }
      if (cs == 0) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) s_red[par][wave][rg * EPL + e] = u[e];
      }
      __syncthreads();
    }
    double us = 0.0;
    if (HAS_P1) {
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) us += s_red[par][w2][urow];
    }
    const double wv = (MODE == PM_A) ? (y - us) * scale : (y - us);
    if (MODE == PM_A || MODE == PM_B) {
      const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.w + p * PANEL, PANEL * 8);
      buf_store_scalar<double>(wv, rw, uact ? (unsigned)(urow * 8) : kOOR);
    }
    if (MODE == PM_C || MODE == PM_INIT) {
      const __amdgpu_buffer_rsrc_t rv =
          make_rsrc(Wb + (size_t)p * pbytes + (size_t)j * PANEL * sizeof(TV), PANEL * sizeof(TV));
      buf_store_scalar<TV>((TV)wv, rv, uact ? (unsigned)(urow * sizeof(TV)) : kOOR);
    }
    if (uact) {
      if (SRC_X) nrm = fma(y, y, nrm);
      if (MODE == PM_C) nrm = fma(wv, wv, nrm);
      if (HAS_P2) s_w[urow] = wv;
    }
    if (HAS_P2) {
      __syncthreads();
      double wr[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) wr[e] = s_w[rg * EPL + e];
      if constexpr (sizeof(TV) == 4) {
        // Keep only the FP32 tile live across the two phases: convert again
        // here instead of holding the FP64 copies made in phase 1.
#pragma unroll
        for (int g = 0; g < QW; ++g) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
        }
      }
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[g] = fma((double)t[g][e], wr[e], acc[g]);
      }
    }
    if (PREF) {
      // The prefetched tile is first needed here: keep the register moves
      // (and with them the wait for its loads) at the end of the iteration.
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(tn[g][e]));
      }
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) t[g][e] = tn[g][e];
      }
    }
    par ^= 1;
  }

  if (HAS_P2) {
#pragma unroll
    for (int g = 0; g < QW; ++g) {
      double v = acc[g];
#pragma unroll
      for (int m = 1; m < LPC; m <<= 1) v += xor_shfl(v, m);
      const int c = cbase + g * GSTRIDE;
      if (rg == 0 && c < j) a.part[(size_t)c * a.ldg + slot] = v;
    }
  }
  if (MODE != PM_B) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) nrm += xor_shfl(nrm, m);
    if (lane == 0) s_nrm[wave] = nrm;
    __syncthreads();
    if (tid == 0) {
      double t2 = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) t2 += s_nrm[w2];
      a.partn[slot] = t2;
    }
  }
}

template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF>
__global__ __launch_bounds__(NW * 64) void k_pass(PassArgs a) {
  if (a.st->status != ST_ACTIVE) return;
  row_pass_body<TV, TX, NW, QW, MODE, PREF>(a, blockIdx.x, a.P, gridDim.x, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Column reduction of the pass partials, one wavefront per column (fixed order:
// lane-strided sums, then a butterfly).  MODE 1 (after pass A): h = sigma o t,
// coefB = sigma o h, and the extra wavefront c == j reduces ||psi||^2.
// MODE 2 (after pass B): s = sigma o t, h += s (step 13), coefC = sigma o s.
// ---------------------------------------------------------------------------
template <int MODE>
__device__ void reduce_body(const SmallArgs &a, int c0) {
  const int lane = threadIdx.x & 63;
  const int c = c0 + (threadIdx.x >> 6);
  if (c < a.j) {
    const double *pc = a.part + (size_t)c * a.ldg;
    double t = 0.0;
    for (int g = lane; g < a.G; g += 64) t += pc[g];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    if (lane == 0) {
      const double sg = a.sigma[c];
      const double v = sg * t;
      if (MODE == 1) {
        a.h[c] = v;
        a.coefB[c] = sg * v;
      } else {
        a.s[c] = v;
        a.h[c] = a.h[c] + v;
        a.coefC[c] = sg * v;
      }
    }
  } else if (MODE == 1 && c == a.j) {
    double t = 0.0;
    for (int g = lane; g < a.G; g += 64) t += a.partn[g];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    if (lane == 0) a.st->xn2 = t;
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(SmallArgs a) {
  if (a.st->status != ST_ACTIVE) return;
  reduce_body<MODE>(a, blockIdx.x * 4);
}

__device__ double block_sum_256(double t, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = t;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = sh[tid] + sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Steps 15-18 plus the breakdown rule; single workgroup.
__device__ void finalize_body(const SmallArgs &a) {
  __shared__ double sh[256];
  __shared__ int s_status;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  if (st->status != ST_ACTIVE) {
    if (tid == 0) st->pushes += 1;
    return;
  }
  const int j = a.j;
  double t = 0.0;
  for (int g = tid; g < a.G; g += 256) t += a.partn[g];
  const double wn2 = block_sum_256(t, sh);
  int bad = 0;
  for (int i = tid; i < j; i += 256) bad |= !isfinite(a.h[i]);
  bad = __syncthreads_or(bad);
  const double bjj = a.beta[(size_t)(j - 1) * a.ldB + (j - 1)];
  if (tid == 0) {
    const double hn = sqrt(wn2);
    const double xn2 = st->xn2;
    int status = ST_ACTIVE;
    if (bad || !isfinite(hn) || !isfinite(xn2)) {
      status = ST_NONFINITE;
    } else {
      const double xf = st->xfro2 + xn2;
      st->xfro2 = xf;
      st->hlast = hn;
      if (hn * bjj <= st->tol * sqrt(xf)) status = ST_INVARIANT;
    }
    s_status = status;
  }
  __syncthreads();
  const int status = s_status;
  if (status == ST_NONFINITE) {
    if (tid == 0) {
      st->status = ST_NONFINITE;
      st->pushes += 1;
    }
    return;
  }
  for (int i = tid; i < j; i += 256) {
    const double hi = a.h[i];
    a.H[(size_t)(j - 1) * a.ldH + i] = hi;
    a.beta[(size_t)j * a.ldB + i] = a.bvec[i] + hi * bjj;  // steps 16-18
  }
  if (tid == 0) {
    if (status == ST_INVARIANT) {
      a.H[(size_t)(j - 1) * a.ldH + j] = 0.0;
      a.beta[(size_t)j * a.ldB + j] = 0.0;
      st->status = ST_INVARIANT;
    } else {
      const double hn = st->hlast;
      a.H[(size_t)(j - 1) * a.ldH + j] = hn;
      a.beta[(size_t)j * a.ldB + j] = hn * bjj;
      a.sigma[j] = 1.0 / hn;
      st->q = j + 1;
    }
    st->pushes += 1;
  }
}

// Steps 2-3 for the first snapshot.
__device__ void finalize_init_body(const SmallArgs &a) {
  __shared__ double sh[256];
  DevState *st = a.st;
  const int tid = threadIdx.x;
  if (st->status != ST_ACTIVE) {
    if (tid == 0) st->pushes += 1;
    return;
  }
  double t = 0.0;
  for (int g = tid; g < a.G; g += 256) t += a.partn[g];
  const double xn2 = block_sum_256(t, sh);
  if (tid == 0) {
    const double b11 = sqrt(xn2);
    if (!isfinite(b11)) {
      st->status = ST_NONFINITE;
    } else if (b11 == 0.0) {
      st->status = ST_ZERO;
    } else {
      a.beta[0] = b11;
      a.sigma[0] = 1.0 / b11;
      st->xfro2 = xn2;
      st->q = 1;
    }
    st->pushes += 1;
  }
}

// Steps 5-8 for the next push (J = q basis vectors):
//   b_i = sum_{l = max(1, i-1)}^{J-1} h_{i,l} beta_{l,J}  (1-based), i = 1..J,
// computed as 64 rows x 4 contiguous l-slices per block, slices combined in
// order.  Also coefA = sigma o b and scaleA = 1 / beta_{J,J}.
__device__ void nextb_body(const SmallArgs &a, int chunk) {
  __shared__ double sh[4][64];
  DevState *st = a.st;
  if (st->status != ST_ACTIVE) return;
  const int J = st->q;
  const int r = threadIdx.x & 63;
  const int sl = threadIdx.x >> 6;
  const int i = chunk * 64 + r;  // 0-based row
  double t = 0.0;
  if (i < J) {
    const int lo = i > 0 ? i - 1 : 0;
    const int hi = J - 1;  // exclusive upper bound (columns 0..J-2)
    const int len = hi > lo ? hi - lo : 0;
    const int a0 = lo + (len * sl) / 4;
    const int a1 = lo + (len * (sl + 1)) / 4;
    const double *bc = a.beta + (size_t)(J - 1) * a.ldB;
    for (int l = a0; l < a1; ++l) t = fma(a.H[(size_t)l * a.ldH + i], bc[l], t);
  }
  sh[sl][r] = t;
  __syncthreads();
  if (sl == 0 && i < J) {
    const double b = ((sh[0][r] + sh[1][r]) + sh[2][r]) + sh[3][r];
    a.bvec[i] = b;
    a.coefA[i] = a.sigma[i] * b;
  }
  if (chunk == 0 && threadIdx.x == 0) st->scaleA = 1.0 / a.beta[(size_t)(J - 1) * a.ldB + (J - 1)];
}

__global__ __launch_bounds__(256) void k_finalize(SmallArgs a) { finalize_body(a); }
__global__ __launch_bounds__(256) void k_finalize_init(SmallArgs a) { finalize_init_body(a); }
__global__ __launch_bounds__(256) void k_nextb(SmallArgs a) { nextb_body(a, blockIdx.x); }

// Reset of one stream: scalar state, and zeros in every small array (the
// entries of H_bar below the subdiagonal and of beta below the diagonal are
// never written by the push kernels and must read as zero).
__device__ void init_state_body(const SmallArgs &a, double tol) {
  const size_t nH = (size_t)a.ldH * (a.n_max + 1), nB = (size_t)a.ldB * (a.n_max + 1);
  const size_t nv = (size_t)a.n_max + 1;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nH; i += stride) a.H[i] = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nB; i += stride) a.beta[i] = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    a.sigma[i] = 0.0;
    a.bvec[i] = 0.0;
    a.h[i] = 0.0;
    a.s[i] = 0.0;
    a.coefA[i] = 0.0;
    a.coefB[i] = 0.0;
    a.coefC[i] = 0.0;
  }
  DevState *st = a.st;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->q = 0;
    st->status = ST_ACTIVE;
    st->pushes = 0;
    st->jstep = 0;
    st->act = 0;
    st->full = 0;
    st->xfro2 = 0.0;
    st->xn2 = 0.0;
    st->scaleA = 0.0;
    st->tol = tol;
    st->hlast = 0.0;
  }
}

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

template <typename TV, typename TX, int NW, int MODE, bool PREF>
static hipError_t launch_pass_q(int qw, int grid, const PassArgs &a, hipStream_t s) {
  constexpr int NT = NW * 64;
  switch (qw) {
    case 1: hipLaunchKernelGGL((k_pass<TV, TX, NW, 1, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pass<TV, TX, NW, 2, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pass<TV, TX, NW, 4, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_pass<TV, TX, NW, 8, MODE, PREF>), dim3(grid), dim3(NT), 0, s, a); break;
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
  const int qw = pick_qw(a.j, NW * Vec<TV>::EPL);
  pref = pref && prefetch_fits<TV, NW>(qw);
  switch (mode) {
    case PM_INIT: return launch_pass_q<TV, TX, NW, PM_INIT, false>(1, grid, a, s);
    case PM_A:
      return pref ? launch_pass_q<TV, TX, NW, PM_A, true>(qw, grid, a, s)
                  : launch_pass_q<TV, TX, NW, PM_A, false>(qw, grid, a, s);
    case PM_B:
      return pref ? launch_pass_q<TV, double, NW, PM_B, true>(qw, grid, a, s)
                  : launch_pass_q<TV, double, NW, PM_B, false>(qw, grid, a, s);
    default:
      return pref ? launch_pass_q<TV, double, NW, PM_C, true>(qw, grid, a, s)
                  : launch_pass_q<TV, double, NW, PM_C, false>(qw, grid, a, s);
  }
}

hipError_t launch_pass(int mode, bool tv_f64, bool tx_f64, bool prefetch, int nw, int grid,
                       const PassArgs &a, hipStream_t s) {
  if (tv_f64) {
    return tx_f64 ? launch_pass_m<double, double, 16>(mode, prefetch, grid, a, s)
                  : launch_pass_m<double, float, 16>(mode, prefetch, grid, a, s);
  }
  if (nw == 8)
    return tx_f64 ? launch_pass_m<float, double, 8>(mode, prefetch, grid, a, s)
                  : launch_pass_m<float, float, 8>(mode, prefetch, grid, a, s);
  return tx_f64 ? launch_pass_m<float, double, 16>(mode, prefetch, grid, a, s)
                : launch_pass_m<float, float, 16>(mode, prefetch, grid, a, s);
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


// ---------------------------------------------------------------------------
// Batched form: many independent streams advanced by one snapshot per step.
// Every kernel reads the per-stream step state (jstep, act) frozen by
// k_batch_begin, so a captured graph of the step replays unchanged while the
// streams grow.  Row passes walk (stream, panel range) work units; one pass
// kernel per column-tile bucket processes the units of the streams whose
// basis size falls in its bucket.
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
  a.G = d.nslot;
  a.ldg = d.ldg;
  a.j = d.st->jstep;
  return a;
}

__global__ __launch_bounds__(256) void k_batch_begin(BatchArgs b) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= b.S) return;
  const BatchStream &d = b.streams[s];
  DevState *st = d.st;
  const bool offered = b.xptrs[s] != nullptr;
  const bool room = st->q < d.n_max;
  st->jstep = st->q;
  st->act = (st->status == ST_ACTIVE && offered && room) ? 1 : 0;
  if (offered && !room && st->status == ST_ACTIVE) st->full = 1;
}

template <int NW, int EPL>
__device__ __forceinline__ int qw_of(int j) {
  int qw = 1;
  while (qw < 16 && qw * NW * EPL < j) qw *= 2;
  return qw;
}

template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF>
__global__ __launch_bounds__(NW * 64) void k_pass_batch(BatchArgs b) {
  for (int u = blockIdx.x; u < b.n_units; u += gridDim.x) {
    const BatchUnit un = b.units[u];
    const BatchStream &d = b.streams[un.s];
    const DevState *st = d.st;
    if (!st->act) continue;
    const int j = st->jstep;
    if (MODE == PM_INIT) {
      if (j != 0) continue;
    } else {
      if (j == 0 || qw_of<NW, Vec<TV>::EPL>(j) != QW) continue;
    }
    PassArgs a{};
    a.W = d.W;
    a.x = b.xptrs[un.s];
    a.w = d.w;
    a.coef = MODE == PM_A ? d.coefA : (MODE == PM_B ? d.coefB : d.coefC);
    a.st = st;
    a.part = d.part;
    a.partn = d.partn;
    a.n = d.n;
    a.P = d.P;
    a.j = j;
    a.n_max = d.n_max;
    a.ldg = d.ldg;
    row_pass_body<TV, TX, NW, QW, MODE, PREF>(a, un.p0, un.p1, 1, un.slot);
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_reduce_batch(BatchArgs b) {
  const int s = b.rblk_stream[blockIdx.x];
  const BatchStream &d = b.streams[s];
  if (!d.st->act || d.st->jstep == 0) return;
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
  const SmallArgs a = small_of(d);
  if (st->jstep == 0)
    finalize_init_body(a);
  else
    finalize_body(a);
}

__global__ __launch_bounds__(256) void k_nextb_batch(BatchArgs b) {
  const BatchStream &d = b.streams[blockIdx.y];
  if (!d.st->act) return;
  if ((int)blockIdx.x * 64 > d.st->q) return;
  nextb_body(small_of(d), blockIdx.x);
}

__global__ __launch_bounds__(256) void k_batch_init_states(BatchArgs b, double tol) {
  init_state_body(small_of(b.streams[blockIdx.y]), tol);
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

template <typename TV, typename TX, int NW, int MODE, bool PREF>
static hipError_t launch_batch_q(int qw, int grid, const BatchArgs &b, hipStream_t s) {
  constexpr int NT = NW * 64;
  switch (qw) {
    case 1: hipLaunchKernelGGL((k_pass_batch<TV, TX, NW, 1, MODE, PREF>), dim3(grid), dim3(NT), 0, s, b); break;
    case 2: hipLaunchKernelGGL((k_pass_batch<TV, TX, NW, 2, MODE, PREF>), dim3(grid), dim3(NT), 0, s, b); break;
    case 4: hipLaunchKernelGGL((k_pass_batch<TV, TX, NW, 4, MODE, PREF>), dim3(grid), dim3(NT), 0, s, b); break;
    case 8: hipLaunchKernelGGL((k_pass_batch<TV, TX, NW, 8, MODE, PREF>), dim3(grid), dim3(NT), 0, s, b); break;
    default:
      if constexpr (sizeof(TV) == 4 || !PREF)
        hipLaunchKernelGGL((k_pass_batch<TV, TX, NW, 16, MODE, PREF>), dim3(grid), dim3(NT), 0, s, b);
      else
        return hipErrorInvalidValue;
      break;
  }
  return hipGetLastError();
}

template <typename TV, typename TX, int NW>
static hipError_t launch_batch_m(int mode, int qw, int grid, const BatchArgs &b, hipStream_t s) {
  // FP64 tiles of 16 groups are not double buffered (register budget)
  const bool pref = !(sizeof(TV) == 8 && qw >= 16);
  switch (mode) {
    case PM_INIT: return launch_batch_q<TV, TX, NW, PM_INIT, false>(1, grid, b, s);
    case PM_A:
      return pref ? launch_batch_q<TV, TX, NW, PM_A, true>(qw, grid, b, s)
                  : launch_batch_q<TV, TX, NW, PM_A, false>(qw, grid, b, s);
    case PM_B:
      return pref ? launch_batch_q<TV, double, NW, PM_B, true>(qw, grid, b, s)
                  : launch_batch_q<TV, double, NW, PM_B, false>(qw, grid, b, s);
    default:
      return pref ? launch_batch_q<TV, double, NW, PM_C, true>(qw, grid, b, s)
                  : launch_batch_q<TV, double, NW, PM_C, false>(qw, grid, b, s);
  }
}

hipError_t launch_batch_pass(int mode, bool tv_f64, bool tx_f64, int qw, int grid, const BatchArgs &b,
                             hipStream_t s) {
  if (tv_f64)
    return tx_f64 ? launch_batch_m<double, double, 16>(mode, qw, grid, b, s)
                  : launch_batch_m<double, float, 16>(mode, qw, grid, b, s);
  return tx_f64 ? launch_batch_m<float, double, 8>(mode, qw, grid, b, s)
                : launch_batch_m<float, float, 8>(mode, qw, grid, b, s);
}

hipError_t launch_batch_begin(const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_begin, dim3((b.S + 255) / 256), dim3(256), 0, s, b);
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

hipError_t launch_fill_random(float *out, int64_t n, uint32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_random, dim3(256), dim3(256), 0, s, out, n, k);
  return hipGetLastError();
}

}  // namespace foa
