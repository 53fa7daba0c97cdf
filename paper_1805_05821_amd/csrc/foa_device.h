// Device bodies of the FOA push kernels (one iteration of Algorithm 1), shared
// by the single-stream kernels and the batched kernels.
#pragma once

#include <math.h>

#include "foa_buffer.h"
#include "foa_internal.h"

namespace foa {


template <typename TV>
struct Vec {
  static constexpr int EPL = 16 / sizeof(TV);  // rows per lane per 16-byte load
};


__device__ __forceinline__ double xor_shfl(double v, int m) { return __shfl_xor(v, m, 64); }

// v(lane) + v(lane ^ M) for M = 16 or 32 with the lane-swap VALU instructions
// (no LDS traffic).  With both operands equal, the 32-swap returns the lower
// half of the wave in both halves of one result and the upper half in both
// halves of the other (16-swap: rows 0,0,2,2 and 1,1,3,3), so the sum of the
// two results is the butterfly sum in every lane, identical in both partners.
template <int M>
__device__ __forceinline__ double xor_sum(double v) {
  static_assert(M == 16 || M == 32, "lane-swap butterfly distance");
  const u32x2 b = __builtin_bit_cast(u32x2, v);
  u32x2 p, q;
  if constexpr (M == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(b.x, b.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(b.y, b.y, false, false);
    p = u32x2{lo[0], hi[0]};
    q = u32x2{lo[1], hi[1]};
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(b.x, b.x, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(b.y, b.y, false, false);
    p = u32x2{lo[0], hi[0]};
    q = u32x2{lo[1], hi[1]};
  }
  return __builtin_bit_cast(double, p) + __builtin_bit_cast(double, q);
}

// A value that is the same in every lane, moved to scalar registers.
template <typename T>
__device__ __forceinline__ T uniform(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  } else {
    const u32x2 w = __builtin_bit_cast(u32x2, v);
    const u32x2 r = u32x2{(unsigned)__builtin_amdgcn_readfirstlane((int)w.x),
                          (unsigned)__builtin_amdgcn_readfirstlane((int)w.y)};
    return __builtin_bit_cast(T, r);
  }
}

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

// Register budget of the row-pass kernels, as waves per SIMD (amdgpu
// attribute): FP32 tiles of 8 groups are held to 128 VGPRs and of 4 groups
// to 96, the budgets at which passes A, B and C of one shape reach the same
// occupancy.  The few values that do not fit are spilled outside the panel
// loop (a reload inside it would wait for the prefetched tile).
template <typename TV, int QW>
constexpr int pass_waves() {
  return sizeof(TV) == 4 ? ((QW == 8 || QW == 6) ? 4 : (QW == 4 ? 5 : 1)) : 1;
}

// Work-vector schemes of the row passes (see the fused row pass below).
enum WScheme : int {
  W_REBUILD = 0,   // nothing stored: B and C rebuild w_A (and w_B) from the snapshot
  W_STORE_AB = 1,  // A stores w_A, B reads it and stores w_B, C reads w_B
};
template <typename TV, int QW>
constexpr int w_scheme() {
  return (sizeof(TV) == 4 && QW >= 2 && QW <= 8) ? W_REBUILD : W_STORE_AB;
}

// Coefficient vectors a pass of this shape uses: K0 .. K1-1 of PassArgs::coef
// (b, h, s); REBUILD: w is rebuilt from the snapshot instead of stored.
template <typename TV, int QW, int MODE>
struct PassCoefs {
  static constexpr bool REBUILD = w_scheme<TV, QW>() == W_REBUILD;
  static constexpr int K1 = MODE == PM_A ? 1 : (MODE == PM_B ? 2 : (MODE == PM_C ? 3 : 0));
  static constexpr int K0 = (REBUILD || K1 <= 1) ? 0 : K1 - 1;
  static constexpr int NC = K1 - K0;
  static constexpr int NCS = NC > 0 ? NC : 1;
};

// LDS of one row-pass call, in doubles: the norm slots, the update rows, the
// coefficient vectors and two parity buffers of per-wavefront row sums (the
// first push uses the norm slots only).
template <typename TV, int NW, int QW, int MODE>
constexpr int pass_lds_doubles() {
  constexpr int NCS = PassCoefs<TV, QW, MODE>::NCS;
  constexpr int JCAP = QW * NW * Vec<TV>::EPL;
  return MODE == PM_INIT ? NW : NW + PANEL + NCS * JCAP + 2 * NCS * NW * PANEL;
}

// ---------------------------------------------------------------------------
// Fused row pass.
//
// Work decomposition: one workgroup walks panels blockIdx.x, +gridDim.x, ...
// Within a panel (64 rows x j columns), wavefront `wave` owns column groups
// g*NW + wave (g < QW); a group is the 1 KiB contiguous block of CPW columns
// read by one 16-byte load per lane.  Lane l holds rows EPL*(l % LPC) .. +EPL-1
// of column (group start) + l / LPC.
//   phase 1 (row sums  u_r = sum_c V_rc coef_c, for NC coefficient vectors at
//            once): per-lane FMA over its groups, butterfly over the lanes
//            sharing rows, then across wavefronts through LDS in wavefront
//            order;
//   update  (every wavefront, 64/NW rows each): w_r = (x_r - u0_r) * scale,
//            then w_r -= u1_r (pass B) and w_r -= u2_r (pass C);
//   phase 2 (column sums V^T w): per-lane FP64 accumulators that persist
//            across panels; one butterfly per column at the end.
// Work vector: for FP32 tiles of 2 to 8 groups (up to 256 columns) w never
// goes to memory: passes B and C rebuild w_A (and w_B) row by row from the
// snapshot and the earlier passes' coefficients, with the same operations in
// the same order, so every pass sees bitwise the values the previous one
// computed and the only store is the new basis column (pass C).  A stream of
// small writes between the basis reads costs far more HBM bandwidth than its
// size (about 15% at 64 columns).  For the other shapes (one group, sixteen
// groups, FP64 tiles) the extra phase-1 work outweighs that, and passes A and
// B store w (FP64) for the next pass to read.
// With PREF the next panel's tile is loaded while the current one is reduced.
// ---------------------------------------------------------------------------
// One workgroup processes panels pstart, pstart + pstep, ... < pend of one
// stream and writes its partial sums to slot `slot`.  Called uniformly by
// the whole workgroup (it synchronises).  lds: pass_lds_doubles() doubles of
// the caller's shared memory.
// Values exchanged between workgroups inside one launch (partial sums,
// reduced coefficients): with COH they are stored and loaded at device
// scope, which writes through and reads past the non-coherent caches, so a
// barrier needs only store completion and no cache write-back or
// invalidation.  Without COH (exchange across kernel boundaries) plain.
template <bool COH>
__device__ __forceinline__ double xld(const double *p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool COH>
__device__ __forceinline__ void xst(double *p, double v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

template <typename TV, typename TX, int NW, int QW, int MODE, bool PREF, bool COH = false>
__device__ __forceinline__ void row_pass_body(const PassArgs &a, int64_t pstart, int64_t pend, int64_t pstep,
                                              int slot, double *lds) {
  // w_A, w_B and w_C are each rounded to FP64 before the next subtraction,
  // as they were when stored between passes: no implicit FMA contraction
  // (the explicit fma() calls of the dot products are unaffected).
#pragma clang fp contract(off)
  constexpr int EPL = Vec<TV>::EPL;
  constexpr int LPC = 64 / EPL;  // lanes per 64-row column segment
  static_assert(LPC == 16 || LPC == 32, "16-byte fragments of FP32 or FP64");
  constexpr int CPW = EPL;       // columns per wavefront load
  constexpr int JCAP = QW * NW * CPW;
  constexpr int RPW = PANEL / NW;  // rows updated by each wavefront
  // where w comes from: rebuilt from the snapshot in every pass, or stored
  // by passes A and B for the next pass; coefficient vectors K0 .. K1-1 of
  // a.coef (b, h, s) enter phase 1
  using PC = PassCoefs<TV, QW, MODE>;
  constexpr bool REBUILD = PC::REBUILD;
  constexpr int K0 = PC::K0;
  constexpr bool STORE_W = !REBUILD && (MODE == PM_A || MODE == PM_B);
  constexpr int NC = PC::NC;
  constexpr bool SRC_X = K0 == 0;  // y is the snapshot, else the stored w
  constexpr bool HAS_P1 = NC > 0;
  constexpr bool HAS_P2 = (MODE == PM_A || MODE == PM_B);
  constexpr int GSTRIDE = NW * CPW;  // columns between a wavefront's groups
  constexpr int NCS = PC::NCS;

  double *s_nrm = lds;
  double *s_w = lds + NW;
  double (*s_coef)[JCAP] = reinterpret_cast<double (*)[JCAP]>(lds + NW + PANEL);
  double (*s_red)[NCS][NW][PANEL] = reinterpret_cast<double (*)[NCS][NW][PANEL]>(lds + NW + PANEL + NCS * JCAP);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wavefront index made provably uniform so per-wave offsets stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cs = lane / LPC;
  const int rg = lane % LPC;
  const int j = a.j;

  __syncthreads();  // the previous call of this workgroup may still read LDS
#pragma unroll
  for (int k = 0; k < NC; ++k)
    for (int c = tid; c < JCAP; c += NW * 64) s_coef[k][c] = (c < j) ? xld<COH>(a.coef[K0 + k] + c) : 0.0;
  const double scale = (MODE == PM_INIT) ? 1.0 : uniform(a.st->scaleA);
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
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rt, (int)(goff0 + g * GBYTES), 0, kTileLoad);
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
    // y for the update rows of this wavefront (snapshot or stored w)
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
      double u[NCS][EPL];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[k][e] = 0.0;
      }
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const double cf = s_coef[k][cbase + g * GSTRIDE];
#pragma unroll
          for (int e = 0; e < EPL; ++e) u[k][e] = fma((double)t[g][e], cf, u[k][e]);
        }
      }
      // butterfly over the lanes sharing rows (distances LPC .. 32)
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        if constexpr (LPC <= 16) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) u[k][e] = xor_sum<16>(u[k][e]);
        }
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[k][e] = xor_sum<32>(u[k][e]);
      }
      if (cs == 0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) s_red[par][k][wave][rg * EPL + e] = u[k][e];
        }
      }
      __syncthreads();
    }
    // w_A = (x - V coef0) * scale; w_B = w_A - V coef1; w_C = w_B - V coef2
    double wv = y;
    if (HAS_P1) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        double us = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) us += s_red[par][k][w2][urow];
        wv = K0 + k == 0 ? (wv - us) * scale : wv - us;
      }
    }
    if (STORE_W) {
      const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.w + p * PANEL, PANEL * 8);
      buf_store_scalar<double>(wv, rw, uact ? (unsigned)(urow * 8) : kOOR);
    }
    if (MODE == PM_C || MODE == PM_INIT) {
      const __amdgpu_buffer_rsrc_t rv =
          make_rsrc(Wb + (size_t)p * pbytes + (size_t)j * PANEL * sizeof(TV), PANEL * sizeof(TV));
      buf_store_scalar<TV>((TV)wv, rv, uact ? (unsigned)(urow * sizeof(TV)) : kOOR);
    }
    if (uact) {
      if (MODE == PM_INIT || MODE == PM_A) nrm = fma(y, y, nrm);
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
      if (rg == 0 && c < j) xst<COH>(a.part + (size_t)c * a.ldg + slot, v);
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
      xst<COH>(a.partn + slot, t2);
    }
  }
}

// ---------------------------------------------------------------------------
// Column reduction of the pass partials, one wavefront per column (fixed order:
// lane-strided sums, then a butterfly).  MODE 1 (after pass A): h = sigma o t,
// coefB = sigma o h, and the extra wavefront c == j reduces ||psi||^2.
// MODE 2 (after pass B): s = sigma o t, h += s, coefC = sigma o s.
// ---------------------------------------------------------------------------
template <int MODE, bool COH = false>
__device__ inline void reduce_body(const SmallArgs &a, int c0) {
  const int lane = threadIdx.x & 63;
  const int c = c0 + (threadIdx.x >> 6);
  if (c < a.j) {
    const double *pc = a.part + (size_t)c * a.ldg;
    double t = 0.0;
    for (int g = lane; g < a.G; g += 64) t += xld<COH>(pc + g);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    if (lane == 0) {
      const double sg = a.sigma[c];
      const double v = sg * t;
      if (MODE == 1) {
        xst<COH>(a.h + c, v);
        xst<COH>(a.coefB + c, sg * v);
      } else {
        xst<COH>(a.s + c, v);
        xst<COH>(a.h + c, xld<COH>(a.h + c) + v);
        xst<COH>(a.coefC + c, sg * v);
      }
    }
  } else if (MODE == 1 && c == a.j) {
    double t = 0.0;
    for (int g = lane; g < a.G; g += 64) t += xld<COH>(a.partn + g);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    if (lane == 0) xst<COH>(&a.st->xn2, t);
  }
}

// Sum over a workgroup of NT threads (fixed tree order).
template <int NT>
__device__ inline double block_sum_t(double t, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = t;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = sh[tid] + sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline double block_sum_256(double t, double *sh) { return block_sum_t<256>(t, sh); }

// Normalisation, beta completion and the breakdown rule; one workgroup of NT threads.
template <int NT, bool COH = false>
__device__ inline void finalize_body_t(const SmallArgs &a) {
  __shared__ double sh[NT];
  __shared__ int s_status;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  if (st->status != ST_ACTIVE) {
    if (tid == 0) st->pushes += 1;
    return;
  }
  const int j = a.j;
  double t = 0.0;
  for (int g = tid; g < a.G; g += NT) t += xld<COH>(a.partn + g);
  const double wn2 = block_sum_t<NT>(t, sh);
  int bad = 0;
  for (int i = tid; i < j; i += NT) bad |= !isfinite(xld<COH>(a.h + i));
  bad = __syncthreads_or(bad);
  const double bjj = a.beta[(size_t)(j - 1) * a.ldB + (j - 1)];
  if (tid == 0) {
    const double hn = sqrt(wn2);
    const double xn2 = xld<COH>(&st->xn2);
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
  for (int i = tid; i < j; i += NT) {
    const double hi = xld<COH>(a.h + i);
    a.H[(size_t)(j - 1) * a.ldH + i] = hi;
    a.beta[(size_t)j * a.ldB + i] = a.bvec[i] + hi * bjj;  // beta completion
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

__device__ inline void finalize_body(const SmallArgs &a) { finalize_body_t<256>(a); }

// Normalisation of the first snapshot.
__device__ inline void finalize_init_body(const SmallArgs &a) {
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

// Partial beta column for the next push (eq. betacolumnupdate, J = q basis vectors):
//   b_i = sum_{l = max(1, i-1)}^{J-1} h_{i,l} beta_{l,J}  (1-based), i = 1..J,
// computed as 64 rows x 4 contiguous l-slices per 256 threads, slices
// combined in order; a workgroup of NT threads takes NT / 256 consecutive
// 64-row chunks from chunk0.  Also coefA = sigma o b and scaleA = 1 / beta_{J,J}.
template <int NT>
__device__ inline void nextb_body_t(const SmallArgs &a, int chunk0) {
  __shared__ double sh[NT / 64][64];
  DevState *st = a.st;
  if (st->status != ST_ACTIVE) return;
  const int J = st->q;
  const int r = threadIdx.x & 63;
  const int sl = (threadIdx.x >> 6) & 3;
  const int sub = threadIdx.x >> 8;
  const int chunk = chunk0 + sub;
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
  sh[4 * sub + sl][r] = t;
  __syncthreads();
  if (sl == 0 && i < J) {
    const double b = ((sh[4 * sub][r] + sh[4 * sub + 1][r]) + sh[4 * sub + 2][r]) + sh[4 * sub + 3][r];
    a.bvec[i] = b;
    a.coefA[i] = a.sigma[i] * b;
  }
  if (chunk == 0 && threadIdx.x == 0) st->scaleA = 1.0 / a.beta[(size_t)(J - 1) * a.ldB + (J - 1)];
}

__device__ inline void nextb_body(const SmallArgs &a, int chunk) { nextb_body_t<256>(a, chunk); }

// Reset of one stream: scalar state, and zeros in every small array (the
// entries of H_bar below the subdiagonal and of beta below the diagonal are
// never written by the push kernels and must read as zero).
__device__ inline void init_state_body(const SmallArgs &a, double tol) {
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
    st->pers = 0;
    st->ls_u = 0;
    st->ls_x = 0;
    st->ls_nx = 0;
    st->ls_alpha = 0.0;
    st->ls_gamma = 0.0;
    st->ls_rhohat = 0.0;
    st->ls_rt = 0.0;
    st->ls_cq = 0.0;
  }
}

}  // namespace foa
