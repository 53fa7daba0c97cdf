// One-reduction form of the FOA step (gfx950).
//
// The modified FOA factorises the snapshots as X = V beta (the QR view of
// Section 3.1) with H_bar following from beta through eq. betacolumnupdate.
// Algorithm 1 orthogonalises with classical Gram-Schmidt applied twice, so a
// push needs three sweeps over the basis and three global reductions.  Here
// the snapshots themselves are orthogonalised and the two projections of
// consecutive snapshots share a sweep (delayed reorthogonalisation, Bielich et
// al., Parallel Computing 2022): the sweep of a push
//   * finishes the pending column: u - Q w, with w = Q^T u from the previous
//     reduction (the second projection);
//   * gives the pending snapshot copy its first projection: x - Q z - q_hat
//     R_tilde, with z = Q^T x and the coefficient on the column just finished,
//     R_tilde = (u^T x - w^T z) / rho_hat, from the previous reduction
//     (rho_hat = sqrt(||u||^2 - ||w||^2), the estimated norm);
//   * copies the new snapshot into the next basis column;
// and forms every column sum the next step needs in the same pass.  One
// fixed-order reduction then gives the exact norm of the finished column, w
// of the new pending column, and z of the new snapshot.  Per push: one sweep
// reading the final columns once, two pending columns read and written, the
// new snapshot read and stored -- about a third of the three-sweep form's
// traffic.  Columns become final two pushes after their snapshot; a flush
// (sweeps without a snapshot) finishes the pending ones.
//
// Storage: column c holds the unnormalised vector, v_c = sigma_c column_c
// with sigma_c = 1 / ||column_c|| (the exact norm of the stored values), as in
// the three-sweep form.  Every dot product, norm and small-matrix operation is
// FP64; stored columns are rounded to the basis precision, and every sum uses
// the rounded values the next sweep will read.
//
// Kernels (all on the context stream):
//   k_ls_pass     : the sweep (panel walk, tile layout and prefetch of the
//                   three-sweep row pass; two coefficient vectors in phase 1,
//                   two right-hand sides in phase 2, six scalar sums);
//   k_ls_reduce   : fixed-order reduction of the workgroup partials;
//   k_ls_finalize : one workgroup: the finished column's norm, scale and
//                   breakdown test, H_bar's column from beta, beta's column of
//                   the new pending column, the next sweep's coefficients.
#include "foa_device.h"
#include "foa_tile.h"

namespace foa {

// ---------------------------------------------------------------------------
// Sweep body.  One workgroup walks panels blockIdx.x, + gridDim.x, ...
// Tile: the q final columns of a panel (lane layout of row_pass_body).  The
// pending columns and the snapshot are read per update row.
// ---------------------------------------------------------------------------
#ifndef LS_PF16
#define LS_PF16 8
#endif
#ifndef LS_PF8
#define LS_PF8 4
#endif

template <typename TV, int NW, int QW>
constexpr int ls_lds_doubles() {
  constexpr int JCAP = QW * NW * Vec<TV>::EPL;
  return 2 * JCAP + 2 * 2 * NW * PANEL + 3 * PANEL + NW * LS_NSC;
}

// Groups of the next panel's tile loaded ahead (the prefetch): all of them,
// except for the FP32 16-group tile, where the Gram sums leave room for 8 (a
// full prefetch spills).  The other groups load at the start of their panel.
template <typename TV, int NW, int QW>
constexpr int ls_pf() {
  return sizeof(TV) == 4 && QW == 16 ? LS_PF16 : (sizeof(TV) == 4 && QW == 8 && NW < 8 ? LS_PF8 : QW);
}

// One workgroup processes panels pstart, pstart + pstep, ... < pend of one
// stream and writes its partial sums to slot `slot`.  Called uniformly by the
// whole workgroup (it synchronises).
template <typename TV, typename TX, int NW, int QW, int PF>
__device__ __forceinline__ void ls_pass_body(const LsArgs &a, int64_t pstart, int64_t pend, int64_t pstep,
                                             int slot, double *lds) {
#pragma clang fp contract(off)
  constexpr int EPL = Vec<TV>::EPL;
  constexpr int LPC = 64 / EPL;
  constexpr int CPW = EPL;
  constexpr int JCAP = QW * NW * CPW;
  constexpr int RPW = PANEL / NW;
  constexpr int GSTRIDE = NW * CPW;

  double (*s_coef)[JCAP] = reinterpret_cast<double (*)[JCAP]>(lds);
  double (*s_red)[2][NW][PANEL] = reinterpret_cast<double (*)[2][NW][PANEL]>(lds + 2 * JCAP);
  double *s_u = lds + 2 * JCAP + 4 * NW * PANEL;
  double *s_x = s_u + PANEL;
  float *s_d = reinterpret_cast<float *>(s_x + PANEL);  // rounding error of the finished column
  double (*s_sc)[LS_NSC] = reinterpret_cast<double (*)[LS_NSC]>(s_x + 2 * PANEL);
  // FP32 basis: the finished column's inner products with the final columns
  // (the Gram correction of the second projection) need the sums of its
  // rounding error against the tile; FP32 accumulation of those tiny values
  // suffices for a correction.  An FP64 basis needs none.
  constexpr bool GRAM = sizeof(TV) == 4;

  const DevState *st = a.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cs = lane / LPC;
  const int rg = lane % LPC;

  // step state (uniform)
  const int q = uniform(st->q);
  const int hu = uniform(st->ls_u);
  const int hf = uniform(st->ls_x);
  const int hn = a.flush ? 0 : 1;
  const int cc = q;            // column under its second projection
  const int cf = q + hu;       // snapshot copy that gets its first projection
  const int cn = cf + hf;      // column the new snapshot is copied to
  const double cq = hu && hf ? uniform(st->ls_cq) : 0.0;

  __syncthreads();  // the previous call of this workgroup may still read LDS
  for (int k = 0; k < 2; ++k)
    for (int c = tid; c < JCAP; c += NW * 64) s_coef[k][c] = (c < q) ? (k ? a.coefZ[c] : a.coefW[c]) : 0.0;
  __syncthreads();

  const int cbase = wave * CPW + cs;
  const unsigned goff0 = (unsigned)((wave * CPW * PANEL + lane * EPL) * sizeof(TV));
  constexpr unsigned GBYTES = (unsigned)(GSTRIDE * PANEL * sizeof(TV));
  const unsigned tile_bytes = (unsigned)(q * PANEL * sizeof(TV));
  const bool uact = lane < RPW;
  const int urow = wave * RPW + (lane % RPW);
  const unsigned pan_bytes = (unsigned)((size_t)a.n_max * PANEL * sizeof(TV));
  // per-row offsets of the pending columns inside a panel (kOOR: absent)
  const unsigned ocu = (uact && hu) ? (unsigned)((cc * PANEL + urow) * sizeof(TV)) : kOOR;
  const unsigned ocf = (uact && hf) ? (unsigned)((cf * PANEL + urow) * sizeof(TV)) : kOOR;
  const unsigned ocn = (uact && hn) ? (unsigned)((cn * PANEL + urow) * sizeof(TV)) : kOOR;

  double acc0[QW], acc1[QW];
  float acc2[GRAM ? QW : 1];
#pragma unroll
  for (int g = 0; g < QW; ++g) acc0[g] = acc1[g] = 0.0;
#pragma unroll
  for (int g = 0; g < (GRAM ? QW : 1); ++g) acc2[g] = 0.f;
  double sc[LS_NSC];
#pragma unroll
  for (int k = 0; k < LS_NSC; ++k) sc[k] = 0.0;

  char *Wb = static_cast<char *>(a.W);
  const size_t pbytes = (size_t)a.n_max * PANEL * sizeof(TV);
  TV t[QW][EPL];
  TV tn[PF > 0 ? PF : 1][EPL];

  int64_t p = pstart;
  if (PF > 0 && p < pend) {
    load_tile_groups<TV, 0, PF, 0>(make_rsrc(Wb + (size_t)p * pbytes, tile_bytes), goff0, GBYTES, t);
#pragma unroll
    for (int g = 0; g < PF; ++g) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
    }
  }
  int par = 0;
  for (; p < pend; p += pstep) {
    // per-row inputs: pending column, snapshot copy, new snapshot (loaded at
    // the start of their own panel: prefetching them with the tile was slower)
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(Wb + (size_t)p * pbytes, pan_bytes);
    const double yu = buf_load_scalar<TV>(rp, ocu);
    const double yf = buf_load_scalar<TV>(rp, ocf);
    double xv;
    {
      const int64_t rem = a.n - p * PANEL;
      const unsigned xb = hn ? (unsigned)((rem >= PANEL ? PANEL : (rem > 0 ? rem : 0)) * sizeof(TX)) : 0u;
      const __amdgpu_buffer_rsrc_t rx = make_rsrc(static_cast<const TX *>(a.x) + (hn ? p * PANEL : 0), xb);
      xv = buf_load_scalar<TX>(rx, uact ? (unsigned)(urow * sizeof(TX)) : kOOR);
    }
    if constexpr (PF < QW) {
      // the groups not prefetched, straight into their place
      load_tile_groups<TV, PF, QW, PF>(make_rsrc(Wb + (size_t)p * pbytes, tile_bytes), goff0, GBYTES, t);
    }
    if constexpr (PF > 0) {
      const bool more = p + pstep < pend;
      load_tile_groups<TV, 0, PF, 0>(make_rsrc(Wb + (size_t)(more ? p + pstep : p) * pbytes, more ? tile_bytes : 0u),
                                   goff0, GBYTES, tn);
    }

    // phase 1: row sums of the tile against sigma o w and sigma o z
    double u[2][EPL];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) u[k][e] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < QW; ++g) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double cf_ = s_coef[k][cbase + g * GSTRIDE];
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[k][e] = fma((double)t[g][e], cf_, u[k][e]);
      }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if constexpr (LPC <= 16) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) u[k][e] = xor_sum<16>(u[k][e]);
      }
#pragma unroll
      for (int e = 0; e < EPL; ++e) u[k][e] = xor_sum<32>(u[k][e]);
    }
    if (cs == 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) s_red[par][k][wave][rg * EPL + e] = u[k][e];
      }
    }
    __syncthreads();
    double sw = 0.0, sz = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) {
      sw += s_red[par][0][w2][urow];
      sz += s_red[par][1][w2][urow];
    }
    // row update: finished column, formed column, snapshot copy (each rounded
    // to the storage type; the sums below use the rounded values)
    const TV ut_s = (TV)(yu - sw);
    const double ut = (double)ut_s;
    const TV uf_s = (TV)((yf - sz) - ut * cq);
    const double uf = (double)uf_s;
    const TV xs_s = (TV)xv;
    const double xs = (double)xs_s;
    buf_store_scalar<TV>(ut_s, rp, ocu);
    buf_store_scalar<TV>(uf_s, rp, ocf);
    buf_store_scalar<TV>(xs_s, rp, ocn);
    if (uact) {
      sc[LS_UU] = fma(ut, ut, sc[LS_UU]);
      sc[LS_UF] = fma(ut, uf, sc[LS_UF]);
      sc[LS_UX] = fma(ut, xs, sc[LS_UX]);
      sc[LS_FF] = fma(uf, uf, sc[LS_FF]);
      sc[LS_FX] = fma(uf, xs, sc[LS_FX]);
      sc[LS_XX] = fma(xv, xv, sc[LS_XX]);
      s_u[urow] = uf;
      s_x[urow] = xs;
      if constexpr (GRAM) s_d[urow] = (float)(ut - (yu - sw));
    }
    __syncthreads();
    // phase 2: column sums of the tile against the formed column and the snapshot
    double wu[EPL], wx[EPL];
    float wd[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      wu[e] = s_u[rg * EPL + e];
      wx[e] = s_x[rg * EPL + e];
      wd[e] = GRAM ? s_d[rg * EPL + e] : 0.f;
    }
    if constexpr (sizeof(TV) == 4) {
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
      }
    }
#pragma unroll
    for (int g = 0; g < QW; ++g) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const double tv = (double)t[g][e];
        acc0[g] = fma(tv, wu[e], acc0[g]);
        acc1[g] = fma(tv, wx[e], acc1[g]);
      }
    }
    if constexpr (GRAM) {
#pragma unroll
      for (int g = 0; g < QW; ++g)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc2[g] = fmaf((float)t[g][e], wd[e], acc2[g]);
    }
    if constexpr (PF > 0) {
#pragma unroll
      for (int g = 0; g < PF; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(tn[g][e]));
      }
#pragma unroll
      for (int g = 0; g < PF; ++g) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) t[g][e] = tn[g][e];
      }
    }
    par ^= 1;
  }

#pragma unroll
  for (int g = 0; g < QW; ++g) {
    double v0 = acc0[g], v1 = acc1[g];
#pragma unroll
    for (int m = 1; m < LPC; m <<= 1) {
      v0 += xor_shfl(v0, m);
      v1 += xor_shfl(v1, m);
    }
    const int c = cbase + g * GSTRIDE;
    if (rg == 0 && c < q) {
      a.part0[(size_t)c * a.ldg + slot] = v0;
      a.part1[(size_t)c * a.ldg + slot] = v1;
    }
    if constexpr (GRAM) {
      float v2 = acc2[g];
#pragma unroll
      for (int m = 1; m < LPC; m <<= 1) v2 += __shfl_xor(v2, m);
      if (rg == 0 && c < q) a.part2[(size_t)c * a.ldg + slot] = (double)v2;
    }
  }
#pragma unroll
  for (int k = 0; k < LS_NSC; ++k) {
    double v = sc[k];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += xor_shfl(v, m);
    if (lane == 0) s_sc[wave][k] = v;
  }
  __syncthreads();
  if (tid < LS_NSC) {
    double v = 0.0;
    for (int w2 = 0; w2 < NW; ++w2) v += s_sc[w2][tid];
    a.part1[(size_t)(a.n_max + tid) * a.ldg + slot] = v;
  }
}

// Sweeps run while the stream is active; flush sweeps also after a
// non-finite snapshot stopped it (the snapshots before it are completed).
__device__ __forceinline__ bool ls_runs(const DevState *st, int flush) {
  const int s = st->status;
  return s == ST_ACTIVE || (flush && s == ST_NONFINITE);
}

// Register budget as waves per SIMD: tiles of up to 4 groups fit 128 VGPRs,
// 6 and 8 groups 168, 12 and 16 groups 256 (two right-hand sides of FP64
// accumulators, the FP32 basis's Gram sums, the current and the prefetched
// tile; the FP32 16-group tile prefetches half of its groups).
template <typename TV, int NW, int QW>
constexpr int ls_waves() {
  // an 8-wavefront workgroup keeps one workgroup per CU at 2 or 3 waves per
  // SIMD, so 8-wavefront tiles of 8 groups take the larger budget (no spill of
  // the FP32 basis's Gram sums)
  return (NW == 16 || QW <= 4) ? 4 : ((QW <= 8 && NW < 8) || QW == 6 ? 3 : 2);
}

template <typename TV, typename TX, int NW, int QW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(ls_waves<TV, NW, QW>()))) void k_ls_pass(
    LsArgs a) {
  if (!ls_runs(a.st, a.flush)) return;
  if (a.flush && !a.st->ls_u && !a.st->ls_x) return;
  __shared__ double lds[ls_lds_doubles<TV, NW, QW>()];
  ls_pass_body<TV, TX, NW, QW, ls_pf<TV, NW, QW>()>(a, blockIdx.x, a.P, gridDim.x, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Reduction: one wavefront per value (part0 columns, part1 columns, scalars),
// lane-strided sums over the slots, then a butterfly: a fixed association.
// ---------------------------------------------------------------------------
// one wavefront per value; vblock selects four consecutive values
__device__ inline void ls_reduce_body(const LsSmall &a, int vblock) {
  const int lane = threadIdx.x & 63;
  const int v = vblock * 4 + (threadIdx.x >> 6);
  const int q = a.st->q;
  const double *src;
  int out;
  if (v < a.nt) {
    if (v >= q) return;
    src = a.part0 + (size_t)v * a.ldg;
    out = v;
  } else if (v < 2 * a.nt) {
    if (v - a.nt >= q) return;
    src = a.part1 + (size_t)(v - a.nt) * a.ldg;
    out = a.n_max + (v - a.nt);
  } else if (v < 2 * a.nt + LS_NSC) {
    src = a.part1 + (size_t)(a.n_max + v - 2 * a.nt) * a.ldg;
    out = 2 * a.n_max + (v - 2 * a.nt);
  } else if (a.gram && v < 3 * a.nt + LS_NSC) {
    const int c = v - 2 * a.nt - LS_NSC;
    if (c >= q || !a.st->ls_u) return;
    src = a.part2 + (size_t)c * a.ldg;
    out = 2 * a.n_max + LS_NSC + c;
  } else {
    return;
  }
  double t = 0.0;
  for (int g = lane; g < a.G; g += 64) t += src[g];
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
  if (lane == 0) a.red[out] = t;
}

__global__ __launch_bounds__(256) void k_ls_reduce(LsSmall a) {
  if (!ls_runs(a.st, a.flush)) return;
  if (a.flush && !a.st->ls_u && !a.st->ls_x) return;
  ls_reduce_body(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Finalize (one workgroup of 512 threads, q <= 511 after the push).
// ---------------------------------------------------------------------------
template <int NT>
__device__ inline double ls_block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// The part of H_bar's column c-1 that the earlier columns give, for the
// column c = q that the coming finalize finishes (eq. betacolumnupdate):
// b_i = sum_{l = max(0, i-1)}^{c-2} H_bar[i, l] beta[l, c-1], i < c.  64 rows
// x 4 contiguous l-slices per 256 threads, slices summed in order.
__device__ inline void ls_hprod_body(const LsSmall &a, int rblock) {
  __shared__ double sh[4][64];
  const DevState *st = a.st;
  const int c = st->q;
  const int r = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int i = rblock * 64 + r;
  double t = 0.0;
  if (i < c) {
    const int lo = i > 0 ? i - 1 : 0, len = c - 1 > lo ? c - 1 - lo : 0;
    const int a0 = lo + (len * sl) / 4, a1 = lo + (len * (sl + 1)) / 4;
    const double *bprev = a.beta + (size_t)(c - 1) * a.ldB;
    // four independent chains, so the loads of several columns are in flight
    double t4[4] = {0.0, 0.0, 0.0, 0.0};
    int l = a0;
    for (; l + 4 <= a1; l += 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) t4[k] = fma(a.H[(size_t)(l + k) * a.ldH + i], bprev[l + k], t4[k]);
    }
    for (; l < a1; ++l) t4[0] = fma(a.H[(size_t)l * a.ldH + i], bprev[l], t4[0]);
    t = (t4[0] + t4[1]) + (t4[2] + t4[3]);
  }
  sh[sl][r] = t;
  __syncthreads();
  if (sl == 0 && i < c) a.bvec[i] = ((sh[0][r] + sh[1][r]) + sh[2][r]) + sh[3][r];
}

// FP32 basis: E w over the earlier final columns for the column that the
// coming finalize makes pending (w_l = sigma_l * its reduced sum l, l < q):
// the same 64 rows x 4 slices, E symmetric with a zero diagonal.  The terms of
// the column finished in the same sweep are added by the finalize.
__device__ inline void ls_ew_body(const LsSmall &a, int rblock) {
  __shared__ double sh[4][64];
  const DevState *st = a.st;
  const int c = st->q;
  const int r = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int i = rblock * 64 + r;
  double t = 0.0;
  if (i < c) {
    const int a0 = (c * sl) / 4, a1 = (c * (sl + 1)) / 4;
    const double *Ei = a.E + i;  // row i (= column i)
    double t4[4] = {0.0, 0.0, 0.0, 0.0};
    int l = a0;
    for (; l + 4 <= a1; l += 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) t4[k] = fma(Ei[(size_t)(l + k) * a.n_max], a.red[l + k] * a.sigma[l + k], t4[k]);
    }
    for (; l < a1; ++l) t4[0] = fma(Ei[(size_t)l * a.n_max], a.red[l] * a.sigma[l], t4[0]);
    t = (t4[0] + t4[1]) + (t4[2] + t4[3]);
  }
  sh[sl][r] = t;
  __syncthreads();
  if (sl == 0 && i < c) a.what[i] = ((sh[0][r] + sh[1][r]) + sh[2][r]) + sh[3][r];
}

__global__ __launch_bounds__(256) void k_ls_hprod(LsSmall a) {
  if (!ls_runs(a.st, a.flush)) return;
  if (a.st->ls_u) ls_hprod_body(a, blockIdx.x);
  if (a.gram && a.st->ls_x) {
    __syncthreads();
    ls_ew_body(a, blockIdx.x);
  }
}

// H_bar's column c-1 once beta's column c is final: h = (beta_{0:c,c} -
// [b; 0]) / beta_{c-1,c-1} with b from k_ls_hprod.
template <int NT>
__device__ inline void ls_hbar_column(const LsSmall &a, int c) {
  const double *bcol = a.beta + (size_t)c * a.ldB;
  const double d = a.beta[(size_t)(c - 1) * a.ldB + (c - 1)];
  for (int i = threadIdx.x; i <= c; i += NT)
    a.H[(size_t)(c - 1) * a.ldH + i] = (bcol[i] - (i < c ? a.bvec[i] : 0.0)) / d;
}

template <int NT>
__device__ inline void ls_finalize_body(const LsSmall &a) {
  __shared__ double sh[NT];
  __shared__ int s_flag;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const bool push = !a.flush;
  if (!ls_runs(st, a.flush) || (a.flush && !st->ls_u && !st->ls_x)) {
    __syncthreads();
    if (tid == 0 && push) st->pushes += 1;
    return;
  }
  const int q0 = st->q;
  const int hu = st->ls_u, hf = st->ls_x;
  int hn = push ? 1 : 0;
  const double *red0 = a.red, *red1 = a.red + a.n_max, *sc = a.red + 2 * a.n_max;
  const double rhohat0 = st->ls_rhohat, rt0 = st->ls_rt;
  // the new snapshot: non-finite -> dropped, the stream stops; zero first -> q = 0
  if (hn) {
    const double xn2 = sc[LS_XX];
    if (!isfinite(xn2)) {
      hn = 0;
      __syncthreads();
      if (tid == 0) st->status = ST_NONFINITE;
    } else if (q0 == 0 && !hu && !hf && xn2 == 0.0) {
      __syncthreads();
      if (tid == 0) {
        st->status = ST_ZERO;
        st->pushes += 1;
      }
      return;
    }
  }
  // 1. the pending column is finished: exact norm, breakdown test, H_bar
  int q = q0;
  double rho = 0.0;
  if (hu) {
    rho = sqrt(sc[LS_UU]);
    const double xf = a.xpre[q0];
    if (tid == 0) s_flag = !(rho > st->tol * sqrt(xf)) ? (isfinite(rho) ? 1 : 2) : 0;
    __syncthreads();
    const int flag = s_flag;
    if (flag) {
      // dependent (or non-finite) column: the stream keeps the q0 columns before it
      if (flag == 1) {
        if (tid == 0) a.beta[(size_t)q0 * a.ldB + q0] = 0.0;
        __syncthreads();
        if (q0 > 0) ls_hbar_column<NT>(a, q0);
      }
      __syncthreads();
      if (tid == 0) {
        st->status = flag == 1 ? ST_INVARIANT : ST_NONFINITE;
        st->ls_u = 0;
        st->ls_x = 0;
        if (push) st->pushes += 1;
      }
      return;
    }
    if (tid == 0) {
      a.beta[(size_t)q0 * a.ldB + q0] = rho;
      a.sigma[q0] = 1.0 / rho;
    }
    if (a.gram) {
      // E's new column: q_i^T q_q0 = sigma_i (stored_i^T delta) / rho, delta the
      // rounding error of the stored column (the rest is O(||E||^2))
      const double *red2 = a.red + 2 * a.n_max + LS_NSC;
      for (int i = tid; i < q0; i += NT) {
        const double g = a.sigma[i] * red2[i] / rho;
        a.E[(size_t)q0 * a.n_max + i] = g;
        a.E[(size_t)i * a.n_max + q0] = g;
      }
      if (tid == 0) a.E[(size_t)q0 * a.n_max + q0] = 0.0;
    }
    __syncthreads();
    if (q0 > 0) ls_hbar_column<NT>(a, q0);
    q = q0 + 1;
  }
  __syncthreads();
  // 2. the snapshot copy became the pending column: its beta column is the
  // first projection plus the second (w), both on the final columns
  double alpha = 0.0, wn2 = 0.0;
  if (hf) {
    const int c = q;  // 0-based index of the new pending column
    const double sk = hu ? a.sigma[q0] : 0.0;
    // FP32 basis: E w.  k_ls_hprod left the part over the earlier final
    // columns in what[0, q0); the finished column q0 adds w_q0 E[i, q0] to
    // rows i < q0 and the whole row q0, sum_l E[q0, l] w_l.
    double eq0 = 0.0;
    if (a.gram && hu) {
      double t = 0.0;
      for (int l = tid; l < q0; l += NT) t = fma(a.E[(size_t)q0 * a.n_max + l], red0[l] * a.sigma[l], t);
      eq0 = ls_block_sum<NT>(t, sh);
    }
    for (int i = tid; i < c; i += NT) {
      double wi, pi, ewi = 0.0;
      if (i < q0) {
        wi = red0[i] * a.sigma[i];
        pi = a.z[i];
        if (a.gram) ewi = a.what[i] + (hu ? a.E[(size_t)q0 * a.n_max + i] * (sc[LS_UF] * sk) : 0.0);
      } else {  // i == q0: the column finished in this sweep
        wi = sc[LS_UF] * sk;
        pi = rhohat0 > 0.0 ? (rho / rhohat0) * rt0 : 0.0;
        ewi = eq0;
      }
      const double wh = wi - ewi;  // the second-projection coefficient used
      a.beta[(size_t)c * a.ldB + i] = pi + wh;
      a.w[i] = wi;
      a.what[i] = wh;
      a.coefW[i] = a.sigma[i] * wh;
    }
    alpha = sc[LS_FF];
  }
  __syncthreads();
  // 3. the new snapshot: first-projection coefficients on the final columns
  if (hn) {
    const double sk = hu ? a.sigma[q0] : 0.0;
    for (int i = tid; i < q; i += NT) {
      const double zi = i < q0 ? red1[i] * a.sigma[i] : sc[LS_UX] * sk;
      a.z[i] = zi;
      a.coefZ[i] = a.sigma[i] * zi;
    }
  }
  __syncthreads();
  // 4. scalars of the next sweep
  const int nu = hf ? 1 : 0;
  const int nx = hn ? 1 : 0;
  double wz = 0.0;
  if (nu) {
    // ||u - Q w_hat||^2 = ||u||^2 - w^T w_hat and the R_tilde identity with
    // w_hat (w_hat = w with an FP64 basis)
    double t = 0.0, t2 = 0.0;
    for (int i = tid; i < q; i += NT) {
      t = fma(a.w[i], a.what[i], t);
      if (nx) t2 = fma(a.what[i], a.z[i], t2);
    }
    wn2 = ls_block_sum<NT>(t, sh);
    wz = ls_block_sum<NT>(t2, sh);
  }
  if (tid == 0) {
    st->q = q;
    st->ls_u = nu;
    st->ls_x = nx;
    if (nu) st->ls_alpha = alpha;
    if (nx) {
      const double xn2 = sc[LS_XX];
      const int k = st->ls_nx;
      a.xpre[k] = (k > 0 ? a.xpre[k - 1] : 0.0) + xn2;
      st->ls_nx = k + 1;
      st->xfro2 += xn2;
      st->ls_gamma = nu ? sc[LS_FX] : 0.0;
    }
    double rh = 0.0, rt = 0.0, cq = 0.0;
    if (nu) {
      const double d = alpha - wn2;
      rh = d > 0.0 ? sqrt(d) : 0.0;
      if (nx && rh > 0.0) {
        rt = (st->ls_gamma - wz) / rh;
        cq = rt / rh;
      }
    }
    st->ls_rhohat = rh;
    st->ls_rt = rt;
    st->ls_cq = cq;
    if (push) st->pushes += 1;
  }
}

__global__ __launch_bounds__(512) void k_ls_finalize(LsSmall a) { ls_finalize_body<512>(a); }

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Tile shapes: FP32 basis 4 wavefronts up to 128 final columns, then 8
// wavefronts (8 groups up to 256 columns, 16 groups up to 512); FP64 basis 8
// wavefronts (up to 16 groups, 256 columns).
int ls_nw(bool tv_f64, int q, int nw_opt) {
  if (tv_f64) return 8;
  if (q <= 128) return 4;
  return (nw_opt == 16 && q <= 256) ? 16 : 8;
}

// Groups per wavefront: the smallest power of two that covers q, except for
// the FP32 sweep of eight wavefronts, which has 6- and 12-group tiles for
// 129-192 and 257-384 columns (a power-of-two tile is a third to a half
// empty there; measured 7-11% faster per sweep at n = 2^24).
int ls_qw(bool tv_f64, int q, int nw_opt) {
  if (!tv_f64 && ls_nw(tv_f64, q, nw_opt) == 8) {
    if (q > 128 && q <= 192) return 6;
    if (q > 256 && q <= 384) return 12;
  }
  return pick_qw(q > 0 ? q : 1, ls_nw(tv_f64, q, nw_opt) * (tv_f64 ? 2 : 4));
}


bool ls_supported(bool tv_f64, int q) { return tv_f64 ? q <= 256 : q <= 512; }

template <typename TV, typename TX, int NW>
static hipError_t launch_ls_q(int qw, int grid, const LsArgs &a, hipStream_t s) {
  constexpr int NT = NW * 64;
  switch (qw) {
    case 1: hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 1>), dim3(grid), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 2>), dim3(grid), dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 4>), dim3(grid), dim3(NT), 0, s, a); break;
    case 8:
      if constexpr (NW < 16) {  // the 16-wavefront tile covers at most 256 columns with 4 groups
        hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 8>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case 16:
      if constexpr (NW == 8) {
        hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 16>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case 6:
      if constexpr (NW == 8 && sizeof(TV) == 4) {
        hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 6>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case 12:
      if constexpr (NW == 8 && sizeof(TV) == 4) {
        hipLaunchKernelGGL((k_ls_pass<TV, TX, NW, 12>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ls_pass(bool tv_f64, bool tx_f64, int q, int nw_opt, int grid, const LsArgs &a, hipStream_t s) {
  if (!ls_supported(tv_f64, q)) return hipErrorInvalidValue;
  const int nw = ls_nw(tv_f64, q, nw_opt);
  const int qw = ls_qw(tv_f64, q, nw_opt);
  if (qw * nw * (tv_f64 ? 2 : 4) < q) return hipErrorInvalidValue;
  if (tv_f64) return tx_f64 ? launch_ls_q<double, double, 8>(qw, grid, a, s) : launch_ls_q<double, float, 8>(qw, grid, a, s);
  if (nw == 4) return tx_f64 ? launch_ls_q<float, double, 4>(qw, grid, a, s) : launch_ls_q<float, float, 4>(qw, grid, a, s);
  if (nw == 16)
    return tx_f64 ? launch_ls_q<float, double, 16>(qw, grid, a, s) : launch_ls_q<float, float, 16>(qw, grid, a, s);
  return tx_f64 ? launch_ls_q<float, double, 8>(qw, grid, a, s) : launch_ls_q<float, float, 8>(qw, grid, a, s);
}

template <typename TV, typename TX, int NW, int QW>
static int ls_occ_q() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_ls_pass<TV, TX, NW, QW>),
                                                   NW * 64, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <typename TV, typename TX, int NW>
static int ls_occ_m(int qw) {
  switch (qw) {
    case 1: return ls_occ_q<TV, TX, NW, 1>();
    case 2: return ls_occ_q<TV, TX, NW, 2>();
    case 4: return ls_occ_q<TV, TX, NW, 4>();
    case 8:
      if constexpr (NW < 16) return ls_occ_q<TV, TX, NW, 8>();
      return 1;
    case 6:
      if constexpr (NW == 8 && sizeof(TV) == 4) return ls_occ_q<TV, TX, NW, 6>();
      return 1;
    case 12:
      if constexpr (NW == 8 && sizeof(TV) == 4) return ls_occ_q<TV, TX, NW, 12>();
      return 1;
    default:
      if constexpr (NW == 8) return ls_occ_q<TV, TX, NW, 16>();
      return 1;
  }
}

int ls_occupancy(bool tv_f64, bool tx_f64, int q, int nw_opt) {
  const int nw = ls_nw(tv_f64, q, nw_opt), qw = ls_qw(tv_f64, q, nw_opt);
  if (tv_f64) return tx_f64 ? ls_occ_m<double, double, 8>(qw) : ls_occ_m<double, float, 8>(qw);
  if (nw == 4) return tx_f64 ? ls_occ_m<float, double, 4>(qw) : ls_occ_m<float, float, 4>(qw);
  if (nw == 16) return tx_f64 ? ls_occ_m<float, double, 16>(qw) : ls_occ_m<float, float, 16>(qw);
  return tx_f64 ? ls_occ_m<float, double, 8>(qw) : ls_occ_m<float, float, 8>(qw);
}

hipError_t launch_ls_reduce(const LsSmall &a, hipStream_t s) {
  const int waves = (a.gram ? 3 : 2) * a.nt + LS_NSC;
  hipLaunchKernelGGL(k_ls_reduce, dim3((waves + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ls_finalize(const LsSmall &a, hipStream_t s) {
  // the H_bar product for the column the finalize finishes (1 <= q <= nt;
  // for q = 1 it writes the empty product 0)
  if (a.nt >= 1) {
    hipLaunchKernelGGL(k_ls_hprod, dim3((a.nt + 63) / 64), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ls_finalize, dim3(1), dim3(512), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched one-reduction form.  The per-step plan of the three-sweep batched
// form (k_batch_plan with ls_mode) buckets the streams by final columns q
// and cuts each bucket's panels into workgroup ranges; here each bucket runs
// one sweep over its ranges, then every active stream its reduction, H_bar
// product and finalize.
// ---------------------------------------------------------------------------
__device__ __forceinline__ LsSmall ls_small_of(const BatchStream &d, int flush) {
  LsSmall a{};
  a.st = d.st;
  a.H = d.H;
  a.beta = d.beta;
  a.sigma = d.sigma;
  a.w = d.h;
  a.z = d.s;
  a.coefW = d.coefA;
  a.coefZ = d.coefB;
  a.red = d.red;
  a.bvec = d.bvec;
  a.xpre = d.xpre;
  a.part0 = d.part;
  a.part1 = d.part1;
  a.part2 = d.part2;
  a.E = d.E;
  a.what = d.what;
  a.gram = d.E != nullptr ? 1 : 0;
  a.ldH = d.ldH;
  a.ldB = d.ldB;
  a.n_max = d.n_max;
  a.ldg = d.ldg;
  a.G = d.st->nseg;
  a.nt = d.st->jstep;
  a.flush = flush;
  return a;
}

template <typename TV, typename TX, int NW, int QW, int BK>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(ls_waves<TV, NW, QW>()))) void k_ls_pass_batch(
    BatchArgs b) {
  __shared__ double lds[ls_lds_doubles<TV, NW, QW>()];
  const int G = uniform(b.meta[2 * BK + 1]);
  if ((int)blockIdx.x >= G) return;
  const int cnt = uniform(b.meta[2 * BK]);
  const int64_t *pre = b.pre + (size_t)BK * (b.S + 1);
  const int *list = b.list + (size_t)BK * b.S;
  const int64_t T = pre[cnt];
  int64_t lo = uniform((int64_t)blockIdx.x * T / G);
  const int64_t hi = uniform((int64_t)(blockIdx.x + 1) * T / G);
  int i = uniform(b.first[BK * kMaxBatchGrid + blockIdx.x]);
  const int flush = b.ls_mode == 2 ? 1 : 0;
  while (lo < hi) {
    const int s = uniform(list[i]);
    const int64_t ps = uniform(pre[i]), pe = uniform(pre[i + 1]);
    const int64_t e = pe < hi ? pe : hi;
    const BatchStream &d = b.streams[s];
    const DevState *st = uniform(d.st);
    LsArgs a{};
    a.W = uniform(d.W);
    a.x = flush ? nullptr : uniform(b.xptrs[s]);
    a.coefW = uniform(d.coefA);
    a.coefZ = uniform(d.coefB);
    a.st = st;
    a.part0 = uniform(d.part);
    a.part1 = uniform(d.part1);
    a.part2 = uniform(d.part2);
    a.n = uniform(d.n);
    a.P = uniform(d.P);
    a.n_max = uniform(d.n_max);
    a.ldg = uniform(d.ldg);
    a.flush = flush;
    ls_pass_body<TV, TX, NW, QW, ls_pf<TV, NW, QW>()>(a, lo - ps, e - ps, 1, (int)blockIdx.x - uniform(st->seg0), lds);
    lo = e;
    ++i;
  }
}

__global__ __launch_bounds__(256) void k_ls_reduce_batch(BatchArgs b) {
  const BatchStream &d = b.streams[blockIdx.y];
  if (!d.st->act) return;
  const LsSmall a = ls_small_of(d, b.ls_mode == 2);
  if ((int)blockIdx.x * 4 >= (a.gram ? 3 : 2) * a.nt + LS_NSC) return;
  ls_reduce_body(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_ls_hprod_batch(BatchArgs b) {
  const BatchStream &d = b.streams[blockIdx.y];
  const LsSmall a = ls_small_of(d, b.ls_mode == 2);
  if (!d.st->act || !(d.st->ls_u || (a.gram && d.st->ls_x))) return;
  if ((int)blockIdx.x * 64 >= d.st->q && blockIdx.x > 0) return;
  if (d.st->ls_u) ls_hprod_body(a, blockIdx.x);
  if (a.gram && d.st->ls_x) {
    __syncthreads();
    ls_ew_body(a, blockIdx.x);
  }
}

__global__ __launch_bounds__(512) void k_ls_finalize_batch(BatchArgs b) {
  const int s = blockIdx.x;
  const BatchStream &d = b.streams[s];
  DevState *st = d.st;
  const int flush = b.ls_mode == 2 ? 1 : 0;
  if (!flush) {
    if (b.xptrs[s] == nullptr) return;  // idle this step
    if (!st->act) {                     // offered to a stream that takes no snapshot
      if (threadIdx.x == 0) st->pushes += 1;
      return;
    }
  } else if (!st->act) {
    return;
  }
  ls_finalize_body<512>(ls_small_of(d, flush));
}

// Kernel shape of bucket k (basis sizes up to 32, 64, 128, 256, 512 final
// columns; k = 0 for an empty basis takes the shape of k = 1).  FP32 basis:
// 1, 2, 4, 8, 8 wavefronts with 8, 8, 8, 8, 16 groups; FP64 basis: 8
// wavefronts with 2, 4, 8, 16 groups (at most 256 columns).
bool ls_batch_supported(bool tv_f64, int k) { return !tv_f64 || k <= 4; }

template <typename TV, typename TX, int BK>
static const void *ls_batch_fn(int *nt) {
  if constexpr (sizeof(TV) == 4) {
    constexpr int NW = BK <= 1 ? 1 : (BK == 2 ? 2 : (BK == 3 ? 4 : 8));
    constexpr int QW = BK == 5 ? 16 : 8;
    *nt = NW * 64;
    return reinterpret_cast<const void *>(&k_ls_pass_batch<TV, TX, NW, QW, BK>);
  } else {
    constexpr int QW = BK <= 1 ? 2 : (BK == 2 ? 4 : (BK == 3 ? 8 : 16));
    *nt = 8 * 64;
    return reinterpret_cast<const void *>(&k_ls_pass_batch<TV, TX, 8, QW, BK>);
  }
}

template <typename TV, typename TX>
static const void *ls_batch_fn_k(int k, int *nt) {
  switch (k) {
    case 0: return ls_batch_fn<TV, TX, 0>(nt);
    case 1: return ls_batch_fn<TV, TX, 1>(nt);
    case 2: return ls_batch_fn<TV, TX, 2>(nt);
    case 3: return ls_batch_fn<TV, TX, 3>(nt);
    case 4: return ls_batch_fn<TV, TX, 4>(nt);
    default:
      if constexpr (sizeof(TV) == 4) return ls_batch_fn<TV, TX, 5>(nt);
      return nullptr;
  }
}

static const void *ls_batch_kernel(bool tv_f64, bool tx_f64, int k, int *nt) {
  if (tv_f64) return tx_f64 ? ls_batch_fn_k<double, double>(k, nt) : ls_batch_fn_k<double, float>(k, nt);
  return tx_f64 ? ls_batch_fn_k<float, double>(k, nt) : ls_batch_fn_k<float, float>(k, nt);
}

int ls_batch_occupancy(bool tv_f64, int k) {
  int nt = 0, nb = 0;
  const void *f = ls_batch_kernel(tv_f64, false, k, &nt);
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, nt, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_ls_batch_pass(bool tv_f64, bool tx_f64, int k, int grid, const BatchArgs &b, hipStream_t s) {
  int nt = 0;
  const void *f = ls_batch_kernel(tv_f64, tx_f64, k, &nt);
  if (!f) return hipErrorInvalidValue;
  void *args[] = {const_cast<BatchArgs *>(&b)};
  return hipLaunchKernel(f, dim3(grid), dim3(nt), args, 0, s);
}

hipError_t launch_ls_batch_small(const BatchArgs &b, hipStream_t s) {
  const int vblocks = (3 * b.max_nmax + LS_NSC + 3) / 4;
  hipLaunchKernelGGL(k_ls_reduce_batch, dim3(vblocks, b.S), dim3(256), 0, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_hprod_batch, dim3((b.max_nmax + 63) / 64, b.S), dim3(256), 0, s, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_finalize_batch, dim3(b.S), dim3(512), 0, s, b);
  return hipGetLastError();
}

}  // namespace foa
