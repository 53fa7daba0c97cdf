// Blocked form of the FOA push: BPK snapshots per step.
//
// The modified FOA builds the thin QR factorisation X = V beta together with
// H_bar, where beta_{:,c+1} = H_bar_{:,1:c} beta_{1:c,c} (eq. betacolumnupdate;
// the QR view of Section 3.1).  The blocked form reaches the same factors in
// exact arithmetic with a block Y of snapshots at a time:
//   R1 = V^T Y;  Z = Y - V R1;  R2 = V^T Z;  Z = Z - V R2     (block CGS2)
//   [R3 = V^T Z;  Z = Z - V R3]    when two projections may not be enough
//   Z = Q S by shifted CholeskyQR3 (Fukaya et al., SIAM J. Sci. Comput. 2020)
//   beta's new columns [R1 + R2 (+ R3); S], V's new columns Q, and H_bar's new
//   columns from the recurrence above solved column by column.
// So the basis is swept three times per block instead of three times per
// snapshot.  The third projection: a stored FP32 basis is orthonormal only to
// E = V^T V - I, the part of Z left along V after two passes is about E R2,
// and where the block's new directions are as small as ||E|| ||Y|| (noise-
// floor snapshots at small n) that part is as large as Z itself.  The test
// estimates ||E|| by ||R2||_F / ||R1||_F and takes the third pass when
// ||E|| ||R2_k|| > u_V ||Z_k|| / 10 for some k (u_V the basis's unit
// roundoff); its kernels are always enqueued and return at once otherwise.  A block is committed only if its Cholesky steps succeed and every
// new diagonal entry of beta is above the breakdown threshold; otherwise the
// device state is left as it was and the host takes those snapshots one at a
// time (the sequential kernels then apply the paper's breakdown rule).
//
// Kernels (all on the context stream, all no-ops once the block is rejected):
//   k_bpass   : the block row passes over V (FP64 accumulation, BPK right-hand
//               sides; same panel walk and tile layout as the single push);
//   k_zgram   : passes over the n x BPK block (||y||^2, Z^T Z, Z <- Z T with
//               its Gram matrix, the final Q written into V);
//   k_breduce : fixed-order reduction of the pass partials into R1 / R2 and
//               the next pass's coefficients;
//   k_bthird  : the test for the third projection (sets the gate of its
//               BP_D pass, reduction, BP_Z2 pass and Gram pass);
//   k_bchol   : Gram reduction, (shifted) Cholesky and triangular inverse;
//   k_bcommit : breakdown test, beta, H_bar, sigma and the scalar state.
#include <mutex>

#include "foa.h"
#include "foa_device.h"
#include "foa_tile.h"

// Block workspace of foa_push_blocked_static, for callers that cannot
// allocate device memory: one copy per device the library runs on, held
// until the process ends.  Host code never uses this name as an address:
// block_static_scratch() looks the device address up once per device and
// every launch takes that address.
static __device__ __align__(256) char scratch[FOA_BLOCK_STATIC_BYTES];

namespace foa {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

hipError_t block_static_scratch(int device, char **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *addr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    g_scratch_addr[device] = e == hipSuccess ? static_cast<char *>(addr) : nullptr;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
  }
  *ptr = g_scratch_addr[device];
  return g_scratch_err[device];
}

enum { BP_R1 = 0, BP_Z1 = 1, BP_Z2 = 2, BP_D = 3, BP_Z0 = 4, BP_ZD = 5, BP_ZR = 6 };
bool block_supported(bool tv_f64, int qw);
enum { ZG_YNORM = 0, ZG_GRAM = 1, ZG_WRITEV = 2, ZG_YNQ = 3 };

// ---------------------------------------------------------------------------
// Block row pass over the basis columns c0 .. c0 + j - 1 (a.c0, a.j; the
// whole basis unless an FP64 basis is split in two windows).  MODE BP_R1:
// D = W^T Y (column sums only).  BP_Z1: Z = Y - W C, D = W^T Z.  BP_Z2:
// Z = Z - W C.  BP_D: D = W^T Z (column sums of the block: the split form of
// BP_Z1's second phase and the third projection).  BP_Z0: Z = Y - W C, and
// BP_ZD: Z = Z - W C, D = W^T Z (the first and last window of BP_Z1 over a
// split basis).  BP_ZR: Z = Z - W C and D = W^T Y' for the next block's
// snapshots Y' (a.xn) in the same sweep (the next block's first projection
// over these columns; the two phases are independent, so Y' goes to LDS at
// phase 1's barrier).  W is the stored basis (the
// sigma scaling of its columns is folded into C and into the reduction of D).
// Per panel, the BPK right-hand sides of a row are spread over the update
// lanes (row, k); phase 1 and phase 2 are those of the single push with BPK
// values per row.
// ---------------------------------------------------------------------------
// PF: groups of the next panel's tile loaded ahead (0 .. QW; the rest load at
// the start of their panel).
// Register budget as waves per SIMD: the 8-group FP32 tile of the passes
// with one phase over the basis rows (BP_R1, BP_D) is held to 128 VGPRs, so
// two 8-wavefront workgroups share a CU (without prefetch: measured 22%
// faster than one workgroup with it); the others take what they need.
template <typename TV, int QW, int MODE>
constexpr int bp_waves() {
  return (sizeof(TV) == 4 && (MODE == BP_R1 || MODE == BP_D) && QW == 8) ? 4 : 1;
}

template <typename TV, typename TX, int NW, int QW, int MODE, int PF>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(bp_waves<TV, QW, MODE>()))) void k_bpass(
    BlockArgs a) {
  constexpr int EPL = Vec<TV>::EPL;
  constexpr int LPC = 64 / EPL;
  constexpr int CPW = EPL;
  constexpr int JCAP = QW * NW * CPW;
  constexpr int RPW = PANEL / NW;
  constexpr int GSTRIDE = NW * CPW;
  constexpr bool NEXT_Y = MODE == BP_ZR;
  constexpr bool HAS_P1 = MODE == BP_Z1 || MODE == BP_Z2 || MODE == BP_Z0 || MODE == BP_ZD || NEXT_Y;
  constexpr bool HAS_P2 = MODE == BP_R1 || MODE == BP_Z1 || MODE == BP_D || MODE == BP_ZD || NEXT_Y;
  constexpr bool SRC_X = MODE == BP_R1 || MODE == BP_Z1 || MODE == BP_Z0;
  constexpr bool STORE_Z = MODE == BP_Z1 || MODE == BP_Z2 || MODE == BP_Z0 || MODE == BP_ZD || NEXT_Y;
  static_assert(RPW * BPK <= 64, "update lanes");

  if (a.st->status != ST_ACTIVE || *a.flag || (a.gate && !*a.gate)) return;

  __shared__ double s_coef[HAS_P1 ? JCAP * BPK : 1];
  __shared__ double s_red[2][NW][PANEL * BPK];
  __shared__ double s_w[2][PANEL * BPK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cs = lane / LPC;
  const int rg = lane % LPC;
  const int j = a.j;
  const int slot = blockIdx.x;

  if (HAS_P1)
    for (int c = tid; c < JCAP * BPK; c += NW * 64) s_coef[c] = (c < j * BPK) ? a.coef[a.c0 * BPK + c] : 0.0;
  __syncthreads();

  const int cbase = wave * CPW + cs;
  const unsigned goff0 = (unsigned)((wave * CPW * PANEL + lane * EPL) * sizeof(TV));
  constexpr unsigned GBYTES = (unsigned)(GSTRIDE * PANEL * sizeof(TV));
  const unsigned tile_bytes = (unsigned)(j * PANEL * sizeof(TV));
  // update lanes: (row, right-hand side) pairs of this wavefront's rows
  const bool uact = lane < RPW * BPK;
  const int urow = wave * RPW + (lane % (RPW * BPK)) / BPK;
  const int uk = lane % BPK;

  double acc[QW][BPK];
#pragma unroll
  for (int g = 0; g < QW; ++g)
#pragma unroll
    for (int k = 0; k < BPK; ++k) acc[g][k] = 0.0;

  // the window's first column within each panel
  const char *Wb = static_cast<const char *>(a.W) + (size_t)a.c0 * PANEL * sizeof(TV);
  const size_t pbytes = (size_t)a.n_max * PANEL * sizeof(TV);
  TV t[QW][EPL];
  TV tn[PF > 0 ? PF : 1][EPL];

  const int64_t pend = a.P, pstep = gridDim.x;
  int64_t p = blockIdx.x;
  if (PF > 0 && p < pend) {
    load_tile_groups<TV, 0, PF, 0>(make_rsrc(Wb + (size_t)p * pbytes, tile_bytes), goff0, GBYTES, t);
#pragma unroll
    for (int g = 0; g < PF; ++g)
#pragma unroll
      for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
  }
  int par = 0;
  for (; p < pend; p += pstep) {
    double y;
    if (SRC_X) {
      const int64_t rem = a.n - p * PANEL;
      const int valid = (int)(rem >= PANEL ? PANEL : (rem > 0 ? rem : 0));
      const __amdgpu_buffer_rsrc_t rx = make_rsrc(static_cast<const TX *>(a.x) + p * PANEL,
                                                  (unsigned)(((BPK - 1) * a.ldx + valid) * sizeof(TX)));
      const unsigned off = (uact && urow < valid) ? (unsigned)((uk * a.ldx + urow) * sizeof(TX)) : kOOR;
      y = buf_load_scalar<TX>(rx, off);
    } else {
      const __amdgpu_buffer_rsrc_t rz = make_rsrc(a.Z + p * PANEL * BPK, PANEL * BPK * 8);
      y = buf_load_scalar<double>(rz, uact ? (unsigned)((uk * PANEL + urow) * 8) : kOOR);
    }
    double yn = 0.0;
    if constexpr (NEXT_Y) {
      const int64_t rem = a.n - p * PANEL;
      const int valid = (int)(rem >= PANEL ? PANEL : (rem > 0 ? rem : 0));
      const __amdgpu_buffer_rsrc_t rx = make_rsrc(static_cast<const TX *>(a.xn) + p * PANEL,
                                                  (unsigned)(((BPK - 1) * a.ldx + valid) * sizeof(TX)));
      yn = buf_load_scalar<TX>(rx, (uact && urow < valid) ? (unsigned)((uk * a.ldx + urow) * sizeof(TX)) : kOOR);
    }
    if constexpr (PF < QW)  // the groups not prefetched, straight into their place
      load_tile_groups<TV, PF, QW, PF>(make_rsrc(Wb + (size_t)p * pbytes, tile_bytes), goff0, GBYTES, t);
    if constexpr (PF > 0) {
      const bool more = p + pstep < pend;
      load_tile_groups<TV, 0, PF, 0>(make_rsrc(Wb + (size_t)(more ? p + pstep : p) * pbytes, more ? tile_bytes : 0u),
                                     goff0, GBYTES, tn);
    }

    double us = 0.0;
    if (HAS_P1) {
      double u[EPL][BPK];
#pragma unroll
      for (int e = 0; e < EPL; ++e)
#pragma unroll
        for (int k = 0; k < BPK; ++k) u[e][k] = 0.0;
#pragma unroll
      for (int g = 0; g < QW; ++g) {
#pragma unroll
        for (int k = 0; k < BPK; ++k) {
          const double cf = s_coef[(cbase + g * GSTRIDE) * BPK + k];
#pragma unroll
          for (int e = 0; e < EPL; ++e) u[e][k] = fma((double)t[g][e], cf, u[e][k]);
        }
      }
#pragma unroll
      for (int e = 0; e < EPL; ++e)
#pragma unroll
        for (int k = 0; k < BPK; ++k) {
          if constexpr (LPC <= 16) u[e][k] = xor_sum<16>(u[e][k]);
          u[e][k] = xor_sum<32>(u[e][k]);
        }
      if (cs == 0) {
#pragma unroll
        for (int e = 0; e < EPL; ++e)
#pragma unroll
          for (int k = 0; k < BPK; ++k) s_red[par][wave][(rg * EPL + e) * BPK + k] = u[e][k];
      }
      if (NEXT_Y && uact) s_w[par][urow * BPK + uk] = yn;
      __syncthreads();
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) us += s_red[par][w2][urow * BPK + uk];
    }
    const double wv = y - us;
    if (STORE_Z) {
      const __amdgpu_buffer_rsrc_t rz = make_rsrc(a.Z + p * PANEL * BPK, PANEL * BPK * 8);
      buf_store_scalar<double>(wv, rz, uact ? (unsigned)((uk * PANEL + urow) * 8) : kOOR);
    }
    if (HAS_P2) {
      if (!NEXT_Y) {
        if (uact) s_w[par][urow * BPK + uk] = wv;
        __syncthreads();
      }
      if constexpr (sizeof(TV) == 4) {
#pragma unroll
        for (int g = 0; g < QW; ++g)
#pragma unroll
          for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(t[g][e]));
      }
      // one row's right-hand sides at a time, which keeps fewer values live
      // (each accumulator takes its rows in order e = 0 .. EPL-1)
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        double wr[BPK];
#pragma unroll
        for (int k = 0; k < BPK; ++k) wr[k] = s_w[par][(rg * EPL + e) * BPK + k];
#pragma unroll
        for (int g = 0; g < QW; ++g)
#pragma unroll
          for (int k = 0; k < BPK; ++k) acc[g][k] = fma((double)t[g][e], wr[k], acc[g][k]);
      }
    }
    if constexpr (PF > 0) {
#pragma unroll
      for (int g = 0; g < PF; ++g)
#pragma unroll
        for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(tn[g][e]));
#pragma unroll
      for (int g = 0; g < PF; ++g)
#pragma unroll
        for (int e = 0; e < EPL; ++e) t[g][e] = tn[g][e];
    }
    par ^= 1;
  }

  if (HAS_P2) {
#pragma unroll
    for (int g = 0; g < QW; ++g) {
      const int c = cbase + g * GSTRIDE;
#pragma unroll
      for (int k = 0; k < BPK; ++k) {
        double v = acc[g][k];
#pragma unroll
        for (int m = 1; m < LPC; m <<= 1) v += xor_shfl(v, m);
        if (rg == 0 && c < j) a.partb[((size_t)(a.c0 + c) * BPK + k) * a.ldg + slot] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Passes over the n x BPK block, one thread per row (rows grid-strided).
// ZG_YNORM: partial ||y_k||^2 of the snapshots.  ZG_YNQ: the same and the
// partial products q_c^T y_k of the previous block's new columns with the
// snapshots (partq), when the sweep before formed V^T Y over the older
// columns (BP_ZR).  ZG_GRAM: the partial Gram
// matrix of Z T_0 .. T_{tlev-1} (T_t upper triangular, the inverses of the
// Cholesky steps so far), formed row by row from Z, which is never
// rewritten: the products are those a pass that stored Z T_0, then read it
// back for T_1, ... would form, in the same order, without the write streams.
// ZG_WRITEV: V's columns j .. j+BPK-1 <- Z T_0 T_1 T_2, rounded to the
// storage type.  Partials: partg[slot * GSLOT + (k * BPK + l)], slot =
// workgroup.
// ---------------------------------------------------------------------------
constexpr int GSLOT = BPK * BPK;

template <typename TV, typename TX, int MODE>
__global__ __launch_bounds__(256) void k_zgram(BlockArgs a) {
  if (a.st->status != ST_ACTIVE || *a.flag || (a.gate && !*a.gate)) return;
  __shared__ double sh[256];
  __shared__ double sT[3 * BPK * BPK];
  const int tid = threadIdx.x;
  const int tlev = a.tlev;
  if (MODE != ZG_YNORM && MODE != ZG_YNQ && tlev > 0) {
    if (tid < tlev * BPK * BPK) sT[tid] = a.sm[SM_T + tid];
    __syncthreads();
  }
  double g[BPK][BPK];
#pragma unroll
  for (int k = 0; k < BPK; ++k)
#pragma unroll
    for (int l = 0; l < BPK; ++l) g[k][l] = 0.0;
  const int64_t npad = a.P * PANEL;
  if constexpr (MODE == ZG_YNQ) {
    // ||y_k||^2 and h[c][k] = q_c^T y_k for the previous block's new columns
    // q_c = V(:, j - BPK + c): one row per grid stride
    const TX *x = static_cast<const TX *>(a.x);
    const TV *W = static_cast<const TV *>(a.W);
    double h[BPK][BPK];
#pragma unroll
    for (int c = 0; c < BPK; ++c)
#pragma unroll
      for (int k = 0; k < BPK; ++k) h[c][k] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + tid; r < a.n; r += (int64_t)gridDim.x * 256) {
      const TV *qr = W + ((r / PANEL) * a.n_max + (a.j - BPK)) * PANEL + r % PANEL;
      double y[BPK], q[BPK];
#pragma unroll
      for (int k = 0; k < BPK; ++k) y[k] = (double)x[(int64_t)k * a.ldx + r];
#pragma unroll
      for (int c = 0; c < BPK; ++c) q[c] = (double)qr[c * PANEL];
#pragma unroll
      for (int k = 0; k < BPK; ++k) g[k][k] = fma(y[k], y[k], g[k][k]);
#pragma unroll
      for (int c = 0; c < BPK; ++c)
#pragma unroll
        for (int k = 0; k < BPK; ++k) h[c][k] = fma(q[c], y[k], h[c][k]);
    }
#pragma unroll
    for (int c = 0; c < BPK; ++c)
#pragma unroll
      for (int k = 0; k < BPK; ++k) {
        const double v = block_sum_256(h[c][k], sh);
        if (tid == 0) a.partq[(size_t)blockIdx.x * GSLOT + c * BPK + k] = v;
      }
  }
  if constexpr (MODE == ZG_YNORM) {
    // the snapshots' rows, four grid strides in flight per thread (each sum
    // still takes its rows in the order of the plain loop below)
    const int64_t stride = (int64_t)gridDim.x * 256;
    const TX *x = static_cast<const TX *>(a.x);
    int64_t r = (int64_t)blockIdx.x * 256 + tid;
    for (; r + 3 * stride < a.n; r += 4 * stride) {
      double v[4][BPK];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < BPK; ++k) v[u][k] = (double)x[(int64_t)k * a.ldx + r + u * stride];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < BPK; ++k) g[k][k] = fma(v[u][k], v[u][k], g[k][k]);
    }
    for (; r < a.n; r += stride) {
#pragma unroll
      for (int k = 0; k < BPK; ++k) {
        const double v = (double)x[(int64_t)k * a.ldx + r];
        g[k][k] = fma(v, v, g[k][k]);
      }
    }
  }
  // the other passes take one row per grid stride (four in flight, as for
  // the snapshots above, measured 6-12% slower here)
  constexpr bool NORMS = MODE == ZG_YNORM || MODE == ZG_YNQ;
  for (int64_t r = (int64_t)blockIdx.x * 256 + tid; !NORMS && r < npad; r += (int64_t)gridDim.x * 256) {
    const int64_t p = r / PANEL;
    const int rr = (int)(r % PANEL);
    double z[BPK];
    const double *zr = a.Z + p * PANEL * BPK + rr;
#pragma unroll
    for (int k = 0; k < BPK; ++k) z[k] = zr[k * PANEL];
    for (int t = 0; t < tlev; ++t) {  // z <- z T_t
      const double *T = sT + t * BPK * BPK;
      double o[BPK];
#pragma unroll
      for (int l = 0; l < BPK; ++l) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= l; ++k) s = fma(z[k], T[k * BPK + l], s);  // T[k][l], k <= l
        o[l] = s;
      }
#pragma unroll
      for (int l = 0; l < BPK; ++l) z[l] = o[l];
    }
    if (MODE == ZG_WRITEV) {
      TV *vc = static_cast<TV *>(a.W) + (size_t)p * a.n_max * PANEL + (size_t)a.j * PANEL + rr;
#pragma unroll
      for (int k = 0; k < BPK; ++k) vc[k * PANEL] = (TV)z[k];
      continue;
    }
#pragma unroll
    for (int k = 0; k < BPK; ++k)
#pragma unroll
      for (int l = 0; l < BPK; ++l) g[k][l] = fma(z[k], z[l], g[k][l]);
  }
  if (MODE == ZG_WRITEV) return;
#pragma unroll
  for (int k = 0; k < BPK; ++k)
#pragma unroll
    for (int l = 0; l < BPK; ++l) {
      if (NORMS && k != l) continue;
      const double s = block_sum_256(g[k][l], sh);
      if (tid == 0) a.partg[(size_t)blockIdx.x * GSLOT + k * BPK + l] = s;
    }
}

// ---------------------------------------------------------------------------
// Reduction of the block-pass partials: one wavefront per (column, rhs) pair
// in a fixed order.  MODE 1 (after BP_R1): R = sigma o D, coef = sigma o R,
// and (extra wavefronts) ||y_k||^2 from the ZG_YNORM partials.  MODE 2 (after
// BP_Z1): R2 = sigma o D, R += R2, coef = sigma o R2.  MODE 3 (after BP_D):
// R += sigma o D, coef = sigma o (sigma o D).  MODE 1 with a.qy: D of the
// columns before the previous block's from dnext (summed by MODE 4 during
// that block), of the previous block's 4 from the ZG_YNQ partials.  MODE 4
// (after BP_ZR): the raw sums D into dnext, for the next block.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_breduce(BlockArgs a) {
  if (a.st->status != ST_ACTIVE || *a.flag || (a.gate && !*a.gate)) return;
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int npairs = a.j * BPK;
  if (wv < npairs) {
    const int c = wv / BPK, k = wv % BPK;
    double t = 0.0;
    if (MODE == 1 && a.qy && c < a.j - BPK) {
      t = a.dnext[wv];
    } else if (MODE == 1 && a.qy) {
      const int e = (c - (a.j - BPK)) * BPK + k;
      for (int g = lane; g < a.Gz; g += 64) t += a.partq[(size_t)g * GSLOT + e];
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    } else {
      const double *pc = a.partb + (size_t)wv * a.ldg;
      for (int g = lane; g < a.G; g += 64) t += pc[g];
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    }
    if (MODE == 4) {
      if (lane == 0) a.dnext[wv] = t;
      return;
    }
    if (lane == 0) {
      const double r = a.sigma[c] * t;
      const size_t idx = (size_t)c * BPK + k;
      if (MODE == 1) {
        a.sm[SM_R + idx] = r;
      } else {
        a.sm[SM_R + idx] += r;
      }
      if (MODE == 2) a.sm[SM_R2 + idx] = r;
      a.coef[idx] = a.sigma[c] * r;
    }
  } else if (MODE == 1 && wv < npairs + BPK) {
    const int k = wv - npairs;
    double t = 0.0;
    for (int g = lane; g < a.Gz; g += 64) t += a.partg[(size_t)g * GSLOT + k * BPK + k];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) t += xor_shfl(t, m);
    if (lane == 0) a.sm[SM_YN2 + k] = t;
  }
}

// ---------------------------------------------------------------------------
// The Gram partials of the workgroups of a block pass, reduced in a fixed
// order into sG[0 .. GSLOT): thread t sums entry t % GSLOT over the slots
// t / GSLOT, + 16, + 32, ... (eight interleaved sums, so eight loads are in
// flight, then added in order); the 16 partial sums of an entry are then
// added in slot order.  One workgroup of 256 threads; sG is complete on
// return.
// ---------------------------------------------------------------------------
static_assert(GSLOT == 16, "256 threads as 16 entries x 16 slot lanes");
__device__ inline void gram_reduce(const BlockArgs &a, int tid, double *sh, double *sG) {
  constexpr int SL = 256 / GSLOT;  // slot lanes per entry
  const int e = tid % GSLOT, s0 = tid / GSLOT;
  double t8[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) t8[m] = 0.0;
  int g = s0;
  for (; g + 7 * SL < a.Gz; g += 8 * SL) {
#pragma unroll
    for (int m = 0; m < 8; ++m) t8[m] += a.partg[(size_t)(g + m * SL) * GSLOT + e];
  }
  double t = 0.0;
#pragma unroll
  for (int m = 0; m < 8; ++m) t += t8[m];
  for (; g < a.Gz; g += SL) t += a.partg[(size_t)g * GSLOT + e];
  sh[tid] = t;
  __syncthreads();
  if (tid < GSLOT) {
    double v = 0.0;
    for (int j = 0; j < 256 / GSLOT; ++j) v += sh[j * GSLOT + tid];
    sG[tid] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Cholesky step ROUND (0: shifted; 0, 1, 2) of the block QR: reduce the Gram
// partials (fixed order), factor G (+ s I) = S^T S, store T_ROUND = S^{-1}
// and accumulate S_total = S S_total.  A non-finite Gram matrix or a non-positive pivot
// rejects the block.  One workgroup; the 4 x 4 algebra runs in thread 0.
// ---------------------------------------------------------------------------
template <int ROUND>
__global__ __launch_bounds__(256) void k_bchol(BlockArgs a) {
  if (a.st->status != ST_ACTIVE || *a.flag) return;
  __shared__ double sh[256];
  __shared__ double sG[GSLOT];
  const int tid = threadIdx.x;
  gram_reduce(a, tid, sh, sG);
  if (tid != 0) return;
  double G[BPK][BPK], S[BPK][BPK], T[BPK][BPK];
  bool ok = true;
  for (int k = 0; k < BPK; ++k)
    for (int l = 0; l < BPK; ++l) {
      // symmetric part (the two triangles are sums of the same products)
      G[k][l] = 0.5 * (sG[k * BPK + l] + sG[l * BPK + k]);
      ok = ok && isfinite(G[k][l]);
    }
  if (ROUND == 0) {
    double tr = 0.0;
    for (int k = 0; k < BPK; ++k) tr += G[k][k];
    const double s = 11.0 * ((double)a.n * BPK + BPK * (BPK + 1)) * 0x1p-53 * tr;
    for (int k = 0; k < BPK; ++k) G[k][k] += s;
  }
  // G = S^T S, S upper triangular with a positive diagonal
  for (int k = 0; k < BPK; ++k)
    for (int l = 0; l < BPK; ++l) S[k][l] = 0.0;
  for (int k = 0; k < BPK && ok; ++k) {
    double d = G[k][k];
    for (int i = 0; i < k; ++i) d -= S[i][k] * S[i][k];
    if (!(d > 0.0) || !isfinite(d)) {
      ok = false;
      break;
    }
    S[k][k] = sqrt(d);
    for (int l = k + 1; l < BPK; ++l) {
      double v = G[k][l];
      for (int i = 0; i < k; ++i) v -= S[i][k] * S[i][l];
      S[k][l] = v / S[k][k];
    }
  }
  if (!ok) {
    *a.flag = 1;
    return;
  }
  // T = S^{-1} (upper triangular), column by column: S T_{:,l} = e_l
  for (int l = 0; l < BPK; ++l) {
    for (int k = BPK - 1; k >= 0; --k) {
      double v = (k == l) ? 1.0 : 0.0;
      for (int i = k + 1; i <= l; ++i) v -= S[k][i] * T[i][l];
      T[k][l] = (k <= l) ? v / S[k][k] : 0.0;
    }
  }
  double *Stot = a.sm + SM_S;
  double P[BPK][BPK];
  for (int k = 0; k < BPK; ++k)
    for (int l = 0; l < BPK; ++l) {
      double v = 0.0;
      if (ROUND == 0) {
        v = S[k][l];
      } else {
        for (int i = k; i <= l; ++i) v += S[k][i] * Stot[i * BPK + l];
      }
      P[k][l] = v;
    }
  for (int k = 0; k < BPK; ++k)
    for (int l = 0; l < BPK; ++l) {
      Stot[k * BPK + l] = P[k][l];
      a.sm[SM_T + ROUND * GSLOT + k * BPK + l] = T[k][l];
    }
}

// ---------------------------------------------------------------------------
// Commit of an accepted block (one workgroup): breakdown test on the new
// diagonal of beta, then beta's columns j .. j+BPK-1, sigma and the scalar
// state.  On rejection nothing is written except the flag.  H_bar follows in
// k_bcommit_h.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bcommit(BlockArgs a) {
  DevState *st = a.st;
  if (st->status != ST_ACTIVE || *a.flag) return;
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  const int j = a.j;
  const double *Stot = a.sm + SM_S;
  int bad = 0;
  for (int e = tid; e < j * BPK; e += 256) bad |= !isfinite(a.sm[SM_R + e]);
  bad = __syncthreads_or(bad);
  if (tid == 0) {
    bool ok = !bad;
    double xf = st->xfro2;
    for (int k = 0; k < BPK; ++k) {
      const double yk = a.sm[SM_YN2 + k];
      ok = ok && isfinite(yk);
      xf += yk;
      const double skk = Stot[k * BPK + k];
      ok = ok && isfinite(skk) && skk > st->tol * sqrt(xf);
    }
    s_ok = ok ? 1 : 0;
    if (!ok) *a.flag = 1;
  }
  __syncthreads();
  if (!s_ok) return;
  // beta's new columns: rows 0..j-1 from R, rows j..j+BPK-1 from S
  for (int e = tid; e < j * BPK; e += 256) {
    const int c = e / BPK, k = e % BPK;
    a.beta[(size_t)(j + k) * a.ldB + c] = a.sm[SM_R + e];
  }
  if (tid < BPK * BPK) {
    const int k = tid / BPK, l = tid % BPK;
    if (k <= l) a.beta[(size_t)(j + l) * a.ldB + (j + k)] = Stot[k * BPK + l];
  }
  if (tid < BPK) a.sigma[j + tid] = 1.0;
  if (tid == 0) {
    double xf = st->xfro2;
    for (int k = 0; k < BPK; ++k) xf += a.sm[SM_YN2 + k];
    st->xfro2 = xf;
    st->q = j + BPK;
    st->pushes += BPK;
  }
}

// ---------------------------------------------------------------------------
// H_bar's new columns c = j-1 .. j+BPK-2 (0-based) of an accepted block, from
// H_bar_{:,c} beta_{c,c} = beta_{:,c+1} - H_bar_{:,0:c-1} beta_{0:c-1,c}.  The
// part of the sum over the old columns (l < j-1) is the same kind of product
// for all BPK new columns, so it is formed first, for every row at once (64
// rows x 4 l-slices per workgroup, slices combined in order); then each row
// runs the BPK-step recurrence over the new columns by itself.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bcommit_h(BlockArgs a) {
  DevState *st = a.st;
  if (*a.flag || st->q != a.j + BPK) return;  // rejected, or nothing committed
  __shared__ double sh[4][64][BPK];
  const int j = a.j;
  const int r = threadIdx.x & 63;
  const int sl = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;  // 0-based row
  const int rows = j + BPK;           // rows 0 .. j+BPK-1 carry the new columns
  double t[BPK];
#pragma unroll
  for (int k = 0; k < BPK; ++k) t[k] = 0.0;
  if (i < rows) {
    const int lo = i > 0 ? i - 1 : 0;
    const int hi = j - 1;  // old columns l < j-1
    const int len = hi > lo ? hi - lo : 0;
    const int a0 = lo + (len * sl) / 4;
    const int a1 = lo + (len * (sl + 1)) / 4;
    for (int l = a0; l < a1; ++l) {
      const double h = a.H[(size_t)l * a.ldH + i];
#pragma unroll
      for (int k = 0; k < BPK; ++k) t[k] = fma(h, a.beta[(size_t)(j - 1 + k) * a.ldB + l], t[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < BPK; ++k) sh[sl][r][k] = t[k];
  __syncthreads();
  if (sl != 0 || i >= rows) return;
  double hn[BPK];
#pragma unroll
  for (int k = 0; k < BPK; ++k) {
    const int c = j - 1 + k;
    double v = a.beta[(size_t)(c + 1) * a.ldB + i];
    v -= ((sh[0][r][k] + sh[1][r][k]) + sh[2][r][k]) + sh[3][r][k];
    for (int kk = 0; kk < k; ++kk) v -= hn[kk] * a.beta[(size_t)c * a.ldB + (j - 1 + kk)];
    hn[k] = (i <= c + 1) ? v / a.beta[(size_t)c * a.ldB + c] : 0.0;
    a.H[(size_t)c * a.ldH + i] = hn[k];
  }
  if (i == rows - 1) st->hlast = hn[BPK - 1];
}

__global__ void k_bflag_clear(int *flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

// ---------------------------------------------------------------------------
// Test for the third projection, after the Gram pass of Z = Y - V (R1 + R2):
// ||Z_k||^2 from the Gram partials (fixed order), ||R2||_F, ||R2_k|| and
// ||R1||_F = ||R - R2||_F from the small area.  *gate = 1 when
// (||R2||_F / ||R1||_F) ||R2_k|| > unit ||Z_k|| / 10 for some k, else 0
// (also for a rejected block).  One workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bthird(BlockArgs a, int *gate, double unit) {
  __shared__ double sh[256];
  __shared__ double sG[GSLOT];
  __shared__ double s_z2[BPK], s_r2[BPK];
  const int tid = threadIdx.x;
  if (a.st->status != ST_ACTIVE || *a.flag) {
    if (tid == 0) *gate = 0;
    return;
  }
  const int npairs = a.j * BPK;
  double r1 = 0.0;
  double r2k[BPK];
#pragma unroll
  for (int k = 0; k < BPK; ++k) r2k[k] = 0.0;
  for (int e = tid; e < npairs; e += 256) {
    const double v2 = a.sm[SM_R2 + e];
    const double v1 = a.sm[SM_R + e] - v2;
    r1 = fma(v1, v1, r1);
#pragma unroll
    for (int k = 0; k < BPK; ++k)
      if (e % BPK == k) r2k[k] = fma(v2, v2, r2k[k]);
  }
  const double r1s = block_sum_256(r1, sh);
#pragma unroll
  for (int k = 0; k < BPK; ++k) {
    const double v = block_sum_256(r2k[k], sh);
    if (tid == 0) s_r2[k] = v;
  }
  gram_reduce(a, tid, sh, sG);
  if (tid < BPK) s_z2[tid] = sG[tid * BPK + tid];
  __syncthreads();
  if (tid != 0) return;
  int third = 0;
  if (r1s > 0.0) {
    double r2f = 0.0;
    for (int k = 0; k < BPK; ++k) r2f += s_r2[k];
    const double e = sqrt(r2f) / sqrt(r1s);
    for (int k = 0; k < BPK; ++k) third |= e * sqrt(s_r2[k]) > 0.1 * unit * sqrt(s_z2[k]);
  }
  *gate = third;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Prefetched groups of a block pass (what fits beside the BPK accumulators).
// FP32 basis: the whole tile, except 6 of 12 groups in BP_Z1, none at 14 and
// 16 groups in BP_Z1, BP_R1 and BP_D (the 16-group BP_Z1 spills even without;
// 2 of 14 in BP_Z1 and 8 of 14 or 16 in BP_R1 fit and were no faster), and
// none at 8 groups in BP_R1 and BP_D (their 128-VGPR budget); FP64 basis: up
// to 4 groups, in BP_Z2 up to 8.
template <typename TV, int QW, int MODE>
constexpr int bp_pf() {
  if constexpr (sizeof(TV) == 8) {
    return (QW <= 4 || MODE == BP_Z2 || MODE == BP_Z0) ? QW : 0;  // BP_ZD as BP_Z1
  } else {
    if (QW == 8 && (MODE == BP_R1 || MODE == BP_D)) return 0;
    if (QW <= 8) return QW;
    if (QW == 12) return (MODE == BP_Z1 || MODE == BP_ZR) ? 6 : 12;
    return MODE == BP_Z2 ? QW : 0;  // 14 and 16 groups
  }
}

template <typename TV, typename TX, int NW, int MODE>
static hipError_t launch_bpass_q(int qw, int grid, const BlockArgs &a, hipStream_t s) {
  constexpr int NT = NW * 64;
  switch (qw) {
    case 1: hipLaunchKernelGGL((k_bpass<TV, TX, NW, 1, MODE, bp_pf<TV, 1, MODE>()>), dim3(grid), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_bpass<TV, TX, NW, 2, MODE, bp_pf<TV, 2, MODE>()>), dim3(grid), dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_bpass<TV, TX, NW, 4, MODE, bp_pf<TV, 4, MODE>()>), dim3(grid), dim3(NT), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_bpass<TV, TX, NW, 8, MODE, bp_pf<TV, 8, MODE>()>), dim3(grid), dim3(NT), 0, s, a); break;
    case 12:
      if constexpr (sizeof(TV) == 4 && NW == 8) {
        hipLaunchKernelGGL((k_bpass<TV, TX, NW, 12, MODE, bp_pf<TV, 12, MODE>()>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case 14:
      if constexpr (sizeof(TV) == 4 && NW == 8) {
        hipLaunchKernelGGL((k_bpass<TV, TX, NW, 14, MODE, bp_pf<TV, 14, MODE>()>), dim3(grid), dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default:
      if constexpr (NW * 16 * Vec<TV>::EPL <= 512)
        hipLaunchKernelGGL((k_bpass<TV, TX, NW, 16, MODE, bp_pf<TV, 16, MODE>()>), dim3(grid), dim3(NT), 0, s, a);
      else
        return hipErrorInvalidValue;
      break;
  }
  return hipGetLastError();
}

template <typename TV, typename TX, int NW>
static hipError_t launch_bpass_m(int mode, int qw, int grid, const BlockArgs &a, hipStream_t s) {
  if (!block_supported(sizeof(TV) == 8, qw)) return hipErrorInvalidValue;
  switch (mode) {
    case BP_R1: return launch_bpass_q<TV, TX, NW, BP_R1>(qw, grid, a, s);
    case BP_Z1: return launch_bpass_q<TV, TX, NW, BP_Z1>(qw, grid, a, s);
    case BP_D: return launch_bpass_q<TV, double, NW, BP_D>(qw, grid, a, s);
    case BP_Z0:
      if constexpr (sizeof(TV) == 8) return launch_bpass_q<TV, TX, NW, BP_Z0>(qw, grid, a, s);
      return hipErrorInvalidValue;
    case BP_ZD:
      if constexpr (sizeof(TV) == 8) return launch_bpass_q<TV, double, NW, BP_ZD>(qw, grid, a, s);
      return hipErrorInvalidValue;
    case BP_ZR: return launch_bpass_q<TV, TX, NW, BP_ZR>(qw, grid, a, s);
    default: return launch_bpass_q<TV, double, NW, BP_Z2>(qw, grid, a, s);
  }
}

// Tile widths the block passes take: an FP64 window beyond 256 columns needs
// more accumulator registers than a 16-wavefront workgroup has (a wider FP64
// basis goes through the passes in windows of at most 256 columns).
bool block_supported(bool tv_f64, int qw) { return !tv_f64 || qw <= 8; }

hipError_t launch_bpass(int mode, bool tv_f64, bool tx_f64, int nw, int qw, int grid, const BlockArgs &a,
                        hipStream_t s) {
  if (tv_f64)
    return tx_f64 ? launch_bpass_m<double, double, 16>(mode, qw, grid, a, s)
                  : launch_bpass_m<double, float, 16>(mode, qw, grid, a, s);
  if (nw == 4)
    return tx_f64 ? launch_bpass_m<float, double, 4>(mode, qw, grid, a, s)
                  : launch_bpass_m<float, float, 4>(mode, qw, grid, a, s);
  return tx_f64 ? launch_bpass_m<float, double, 8>(mode, qw, grid, a, s)
                : launch_bpass_m<float, float, 8>(mode, qw, grid, a, s);
}

template <typename TV, typename TX>
static hipError_t launch_zgram_t(int mode, int grid, const BlockArgs &a, hipStream_t s) {
  switch (mode) {
    case ZG_YNORM: hipLaunchKernelGGL((k_zgram<TV, TX, ZG_YNORM>), dim3(grid), dim3(256), 0, s, a); break;
    case ZG_GRAM: hipLaunchKernelGGL((k_zgram<TV, TX, ZG_GRAM>), dim3(grid), dim3(256), 0, s, a); break;
    case ZG_YNQ: hipLaunchKernelGGL((k_zgram<TV, TX, ZG_YNQ>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_zgram<TV, TX, ZG_WRITEV>), dim3(grid), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_zgram(int mode, bool tv_f64, bool tx_f64, int grid, const BlockArgs &a, hipStream_t s) {
  if (tv_f64)
    return tx_f64 ? launch_zgram_t<double, double>(mode, grid, a, s) : launch_zgram_t<double, float>(mode, grid, a, s);
  return tx_f64 ? launch_zgram_t<float, double>(mode, grid, a, s) : launch_zgram_t<float, float>(mode, grid, a, s);
}

hipError_t launch_breduce(int mode, const BlockArgs &a, hipStream_t s) {
  const int waves = a.j * BPK + (mode == 1 ? BPK : 0);
  const int blocks = (waves + 3) / 4;
  if (mode == 1)
    hipLaunchKernelGGL(k_breduce<1>, dim3(blocks), dim3(256), 0, s, a);
  else if (mode == 2)
    hipLaunchKernelGGL(k_breduce<2>, dim3(blocks), dim3(256), 0, s, a);
  else if (mode == 3)
    hipLaunchKernelGGL(k_breduce<3>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_breduce<4>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bchol(int round, const BlockArgs &a, hipStream_t s) {
  if (round == 0)
    hipLaunchKernelGGL(k_bchol<0>, dim3(1), dim3(256), 0, s, a);
  else if (round == 1)
    hipLaunchKernelGGL(k_bchol<1>, dim3(1), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_bchol<2>, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bcommit(const BlockArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_bcommit, dim3(1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_bcommit_h, dim3((a.j + BPK + 63) / 64), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bflag_clear(int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_bflag_clear, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_bthird(const BlockArgs &a, int *gate, double unit, hipStream_t s) {
  hipLaunchKernelGGL(k_bthird, dim3(1), dim3(256), 0, s, a, gate, unit);
  return hipGetLastError();
}

}  // namespace foa
