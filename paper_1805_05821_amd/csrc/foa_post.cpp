// Host FP64 post-processing of the FOA state (Algorithm 1 after its snapshot
// loop): rank truncation, eigenpairs of the projected matrix, error
// indicators (Section 3.2.3), coefficients of the first snapshot and mode
// ordering (Section 3.2.4), and the mode matrix V B on the device.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "foa.h"
#include "foa_ctx.h"
#include "hostla.h"

using namespace foa;
using cd = std::complex<double>;

namespace {

double spacing_at(double x, bool f32) {
  x = std::fabs(x);
  if (f32) {
    const float xf = (float)x;
    return (double)(std::nextafter(xf, INFINITY) - xf);
  }
  return std::nextafter(x, INFINITY) - x;
}

// Unit 2-norm, entry of largest modulus real positive (column of length m).
void unit_phase(cd *z, int m) {
  double nrm = 0.0;
  int kmax = 0;
  double amax = -1.0;
  for (int i = 0; i < m; ++i) {
    nrm += std::norm(z[i]);
    const double a = std::abs(z[i]);
    if (a > amax) {
      amax = a;
      kmax = i;
    }
  }
  nrm = std::sqrt(nrm);
  if (nrm == 0.0 || amax == 0.0) return;
  const cd ph = std::conj(z[kmax]) / amax;
  for (int i = 0; i < m; ++i) z[i] = z[i] * ph / nrm;
}

// Eigen-decomposition and derived quantities of the (possibly truncated)
// projected matrix; cached in c->dmd.
foa_status compute_dmd(foa_ctx_s *c) {
  foa_status r = refresh_mirror(c);
  if (r != FOA_OK) return r;
  if (c->dmd.valid) return FOA_OK;
  const int m = projected_order(c);
  if (m < 1) return set_err(c, FOA_E_STATE, "need a projected matrix of order >= 1 (q = %d)", c->q_host);
  if (c->trunc_r > 0 && c->trunc_m != m) {
    c->trunc_r = 0;  // truncation was computed for another state
    c->Ur.clear();
  }
  const int ldH = c->L.ldH;
  const bool inv = c->dev_status == ST_INVARIANT;
  const double hlast = inv ? 0.0 : c->hH[(size_t)(m - 1) * ldH + m];
  const double b11 = c->hB[0];
  std::vector<double> Hm((size_t)m * m);
  // upper Hessenberg pattern only
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m && i <= j + 1; ++i) Hm[(size_t)j * m + i] = c->hH[(size_t)j * ldH + i];

  DmdCache &d = c->dmd;
  d = DmdCache();
  d.m = m;
  const int rr = c->trunc_r;
  std::vector<cd> Z;
  if (rr > 0) {
    // U_r^T H_m U_r (truncated DMD, Algorithm 1)
    const std::vector<double> &U = c->Ur;  // m x r
    std::vector<double> HU((size_t)m * rr, 0.0), Ht((size_t)rr * rr, 0.0);
    for (int j = 0; j < rr; ++j)
      for (int l = 0; l < m; ++l) {
        const double u = U[(size_t)j * m + l];
        if (u == 0.0) continue;
        for (int i = 0; i < m; ++i) HU[(size_t)j * m + i] += Hm[(size_t)l * m + i] * u;
      }
    for (int j = 0; j < rr; ++j)
      for (int i = 0; i < rr; ++i) {
        double s = 0.0;
        for (int l = 0; l < m; ++l) s += U[(size_t)i * m + l] * HU[(size_t)j * m + l];
        Ht[(size_t)j * rr + i] = s;
      }
    if (hla::eig_real(rr, Ht.data(), rr, d.lam, Z, d.is_real) != 0)
      return set_err(c, FOA_E_NUMERIC, "QR iteration did not converge (order %d)", rr);
    d.k = rr;
    d.r = rr;
  } else {
    if (hla::eig_real(m, Hm.data(), m, d.lam, Z, d.is_real) != 0)
      return set_err(c, FOA_E_NUMERIC, "QR iteration did not converge (order %d)", m);
    d.k = m;
  }
  const int k = d.k;
  for (int i = 0; i < k; ++i) unit_phase(Z.data() + (size_t)i * k, k);

  // B = U_r Z (truncated) or Z: coefficients of the modes in the V_{1:m} basis
  d.B.assign((size_t)m * k, cd(0, 0));
  if (rr > 0) {
    for (int i = 0; i < k; ++i)
      for (int l = 0; l < rr; ++l) {
        const cd z = Z[(size_t)i * k + l];
        for (int row = 0; row < m; ++row) d.B[(size_t)i * m + row] += c->Ur[(size_t)l * m + row] * z;
      }
  } else {
    d.B = Z;
  }

  // error indicators (Section 3.2.3)
  d.ind.assign(k, 0.0);
  for (int i = 0; i < k; ++i) {
    const cd *y = d.B.data() + (size_t)i * m;  // U_r z_i (or z_i)
    if (rr == 0) {
      d.ind[i] = std::fabs(hlast) * std::abs(y[m - 1]);
    } else {
      std::vector<cd> Hy(m, cd(0, 0)), t(rr, cd(0, 0));
      for (int l = 0; l < m; ++l)
        for (int row = 0; row < m; ++row) Hy[row] += Hm[(size_t)l * m + row] * y[l];
      for (int a = 0; a < rr; ++a)
        for (int row = 0; row < m; ++row) t[a] += c->Ur[(size_t)a * m + row] * Hy[row];
      double s2 = 0.0;
      for (int row = 0; row < m; ++row) {
        cd top = Hy[row];
        for (int a = 0; a < rr; ++a) top -= c->Ur[(size_t)a * m + row] * t[a];
        s2 += std::norm(top);
      }
      s2 += std::norm(hlast * y[m - 1]);
      d.ind[i] = std::sqrt(s2);
    }
  }

  // coefficients of psi_1: [z]{c} = ||psi_1|| e_1 or ||psi_1|| U_r^T e_1
  d.coef.assign(k, cd(0, 0));
  for (int a = 0; a < k; ++a) d.coef[a] = rr > 0 ? cd(b11 * c->Ur[(size_t)a * m + 0], 0.0) : cd(a == 0 ? b11 : 0.0, 0.0);
  if (hla::solve_complex(k, Z, d.coef) != 0)
    return set_err(c, FOA_E_NUMERIC, "eigenvector matrix is singular");

  // one entry per real eigenvalue and per conjugate pair; order by |c| desc,
  // then |lambda| desc, then index
  for (int i = 0; i < k; ++i)
    if (d.is_real[i] || d.lam[i].imag() > 0) d.entries.push_back(i);
  std::stable_sort(d.entries.begin(), d.entries.end(), [&](int a, int b) {
    const double ca = std::abs(d.coef[a]), cb = std::abs(d.coef[b]);
    if (ca != cb) return ca > cb;
    const double la = std::abs(d.lam[a]), lb = std::abs(d.lam[b]);
    if (la != lb) return la > lb;
    return a < b;
  });
  d.valid = true;
  return FOA_OK;
}

}  // namespace

extern "C" {

foa_status foa_truncate(foa_ctx c, double rel_tol, int32_t r_force, int32_t *r_out, double *h_sigma) {
  if (!c) return FOA_E_ARG;
  if (std::isnan(rel_tol) || r_force < -1) return set_err(c, FOA_E_ARG, "bad truncation arguments");
  foa_status r = refresh_mirror(c);
  if (r != FOA_OK) return r;
  c->dmd.valid = false;
  if (r_force == -1) {
    c->trunc_r = 0;
    c->trunc_m = 0;
    c->Ur.clear();
    if (r_out) *r_out = 0;
    return FOA_OK;
  }
  const int m = projected_order(c);
  if (m < 1) return set_err(c, FOA_E_STATE, "need at least two snapshots");
  std::vector<double> Bm((size_t)m * m, 0.0);  // upper triangular pattern only
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= j; ++i) Bm[(size_t)j * m + i] = c->hB[(size_t)j * c->L.ldB + i];
  std::vector<double> U, S;
  if (hla::svd_left(m, Bm.data(), m, U, S) != 0)
    return set_err(c, FOA_E_NUMERIC, "Jacobi SVD did not converge (order %d)", m);
  int rank;
  if (r_force > 0) {
    rank = std::min<int>(r_force, m);
  } else {
    const double thr = rel_tol >= 0 ? rel_tol * S[0]
                                    : (double)c->q_host * spacing_at(S[0], c->prec == FOA_PREC_F32);
    rank = 0;
    for (int i = 0; i < m; ++i) rank += S[i] > thr ? 1 : 0;
    rank = std::max(rank, 1);
  }
  c->Ur.assign(U.begin(), U.begin() + (size_t)m * rank);
  c->hsv = S;
  c->trunc_r = rank;
  c->trunc_m = m;
  if (r_out) *r_out = rank;
  if (h_sigma)
    for (int i = 0; i < m; ++i) h_sigma[i] = S[i];
  return FOA_OK;
}

foa_status foa_indicators(foa_ctx c, int32_t m_max, double *h_lambda, double *h_err, int32_t *m_out) {
  if (!c) return FOA_E_ARG;
  if (m_max < 0) return set_err(c, FOA_E_ARG, "m_max < 0");
  foa_status r = compute_dmd(c);
  if (r != FOA_OK) return r;
  const DmdCache &d = c->dmd;
  const int cnt = std::min<int>(m_max, (int)d.entries.size());
  for (int e = 0; e < cnt; ++e) {
    const int i = d.entries[e];
    if (h_lambda) {
      h_lambda[2 * e] = d.lam[i].real();
      h_lambda[2 * e + 1] = d.lam[i].imag();
    }
    if (h_err) h_err[e] = d.ind[i];
  }
  if (m_out) *m_out = cnt;
  return FOA_OK;
}

foa_status foa_modes(foa_ctx c, int32_t m_max, double *h_lambda, int8_t *h_kind, double *h_amp, double *h_err,
                     void *d_phi, int64_t ld_phi, int32_t phi_cols, foa_dtype phi_dtype, int32_t *m_out) {
  if (!c) return FOA_E_ARG;
  if (m_max < 0 || (d_phi && (ld_phi < c->n || (phi_dtype != FOA_F32 && phi_dtype != FOA_F64))))
    return set_err(c, FOA_E_ARG, "bad mode arguments");
  foa_status r = compute_dmd(c);
  if (r != FOA_OK) return r;
  const DmdCache &d = c->dmd;
  const int cnt = std::min<int>(m_max, (int)d.entries.size());
  int ncols = 0;
  for (int e = 0; e < cnt; ++e) ncols += d.is_real[d.entries[e]] ? 1 : 2;
  if (d_phi && ncols > phi_cols)
    return set_err(c, FOA_E_ARG, "mode matrix needs %d columns, phi_cols = %d", ncols, phi_cols);
  for (int e = 0; e < cnt; ++e) {
    const int i = d.entries[e];
    if (h_lambda) {
      h_lambda[2 * e] = d.lam[i].real();
      h_lambda[2 * e + 1] = d.lam[i].imag();
    }
    if (h_kind) h_kind[e] = d.is_real[i] ? 0 : 1;
    if (h_amp) h_amp[e] = std::abs(d.coef[i]);
    if (h_err) h_err[e] = d.ind[i];
  }
  if (m_out) *m_out = cnt;
  if (!d_phi || ncols == 0) return FOA_OK;
  // packed real coefficients, sigma folded in: V = W diag(sigma)
  const int m = d.m;
  const bool v64 = c->prec == FOA_PREC_F64, o64 = phi_dtype == FOA_F64;
  const bool mfma = modes_use_mfma(v64, o64);
  const size_t ldp = mfma ? (size_t)modes_rpad(ncols) : 1;   // stride between rows l
  const size_t cst = mfma ? 1 : (size_t)m;                    // stride between columns
  std::vector<double> Bp(mfma ? (size_t)modes_kpad(m) * ldp : (size_t)m * ncols, 0.0);
  int col = 0;
  for (int e = 0; e < cnt; ++e) {
    const int i = d.entries[e];
    const cd *b = d.B.data() + (size_t)i * m;
    for (int l = 0; l < m; ++l) Bp[col * cst + l * ldp] = c->hsigma[l] * b[l].real();
    ++col;
    if (!d.is_real[i]) {
      for (int l = 0; l < m; ++l) Bp[col * cst + l * ldp] = c->hsigma[l] * b[l].imag();
      ++col;
    }
  }
  void *dB = static_cast<char *>(c->ws) + c->L.mcoef;
  hipError_t e;
  if (mfma) {
    std::vector<float> Bf(Bp.begin(), Bp.end());
    e = hipMemcpy(dB, Bf.data(), Bf.size() * sizeof(float), hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(dB, Bp.data(), Bp.size() * sizeof(double), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_err(c, e, "hipMemcpy mode coefficients");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, c->stream);
  }
  e = launch_modes_gemm(v64, c->W, c->n, c->n_max, m, dB, ncols, d_phi, ld_phi, o64, c->stream);
  if (c->profile && e0 && e1) {
    (void)hipEventRecord(e1, c->stream);
    c->ev_pending.push_back({e0, e1, 2.0 * (double)c->n * m * ncols, 1});
  }
  return hip_err(c, e, "mode GEMM");
}

}  // extern "C"
