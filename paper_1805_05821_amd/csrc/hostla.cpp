// Host FP64 dense linear algebra (see hostla.h).
//
// svd_left: one-sided (Hestenes) Jacobi: plane rotations applied to pairs of
//   columns until all pairs are orthogonal to working precision; the column
//   norms are the singular values and the normalised columns the left
//   singular vectors.
// eig_real: Householder reduction to upper Hessenberg form, then the Francis
//   implicit double-shift QR iteration (Golub & Van Loan, Sec. 7.5) with
//   deflation, accumulating the orthogonal similarity, to a real Schur form T
//   (1x1 blocks for real eigenvalues, 2x2 blocks for conjugate pairs).
//   Eigenvectors of T come from back substitution through the block
//   structure in complex arithmetic and are mapped back with the accumulated
//   orthogonal matrix.
#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace hla {

namespace {
constexpr double kEps = 2.220446049250313e-16;
}

int svd_left(int m, const double *A, int lda, std::vector<double> &U, std::vector<double> &S) {
  std::vector<double> G((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) G[(size_t)j * m + i] = A[(size_t)j * lda + i];
  auto col = [&](int j) { return G.data() + (size_t)j * m; };
  auto dot = [&](const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
  };
  const double tol = std::sqrt((double)m) * kEps;
  std::vector<double> nrm(m);
  bool converged = (m <= 1);
  for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
    for (int j = 0; j < m; ++j) nrm[j] = dot(col(j), col(j));
    bool rotated = false;
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const double a = nrm[p], b = nrm[q];
        if (a == 0.0 || b == 0.0) continue;
        double *gp = col(p), *gq = col(q);
        const double g = dot(gp, gq);
        if (std::fabs(g) <= tol * std::sqrt(a) * std::sqrt(b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        double t;
        if (std::fabs(zeta) > 1e150)
          t = 0.5 / zeta;
        else
          t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = gp[i], y = gq[i];
          gp[i] = c * x - s * y;
          gq[i] = s * x + c * y;
        }
        nrm[p] = a - t * g;
        nrm[q] = b + t * g;
      }
    }
    converged = !rotated;
  }
  if (!converged) return -1;
  std::vector<double> sv(m);
  for (int j = 0; j < m; ++j) sv[j] = std::sqrt(dot(col(j), col(j)));
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return sv[a] > sv[b]; });
  U.assign((size_t)m * m, 0.0);
  S.assign(m, 0.0);
  for (int k = 0; k < m; ++k) {
    const int j = idx[k];
    S[k] = sv[j];
    if (sv[j] > 0)
      for (int i = 0; i < m; ++i) U[(size_t)k * m + i] = col(j)[i] / sv[j];
  }
  return 0;
}

namespace {

// Column-major element access.
struct Mat {
  int m;
  std::vector<double> a;
  explicit Mat(int m_) : m(m_), a((size_t)m_ * m_, 0.0) {}
  double &operator()(int i, int j) { return a[(size_t)j * m + i]; }
  double operator()(int i, int j) const { return a[(size_t)j * m + i]; }
};

// Householder reduction of H to upper Hessenberg form, H <- Q^T H Q, Q <- Q Q_k.
void hessenberg(Mat &H, Mat &Q) {
  const int m = H.m;
  std::vector<double> v(m);
  for (int k = 0; k + 2 < m; ++k) {
    double tail = 0.0;
    for (int i = k + 2; i < m; ++i) tail = std::max(tail, std::fabs(H(i, k)));
    if (tail == 0.0) continue;  // column already in Hessenberg form
    double alpha = 0.0;
    for (int i = k + 1; i < m; ++i) alpha += H(i, k) * H(i, k);
    alpha = std::sqrt(alpha);
    if (H(k + 1, k) > 0) alpha = -alpha;
    const int len = m - k - 1;
    for (int l = 0; l < len; ++l) v[l] = H(k + 1 + l, k);
    v[0] -= alpha;
    double vn = 0.0;
    for (int l = 0; l < len; ++l) vn += v[l] * v[l];
    if (vn == 0.0) continue;
    const double beta = 2.0 / vn;
    for (int j = k; j < m; ++j) {  // H <- P H
      double s = 0.0;
      for (int l = 0; l < len; ++l) s += v[l] * H(k + 1 + l, j);
      s *= beta;
      for (int l = 0; l < len; ++l) H(k + 1 + l, j) -= s * v[l];
    }
    for (int i = 0; i < m; ++i) {  // H <- H P, Q <- Q P
      double s = 0.0, t = 0.0;
      for (int l = 0; l < len; ++l) {
        s += H(i, k + 1 + l) * v[l];
        t += Q(i, k + 1 + l) * v[l];
      }
      s *= beta;
      t *= beta;
      for (int l = 0; l < len; ++l) {
        H(i, k + 1 + l) -= s * v[l];
        Q(i, k + 1 + l) -= t * v[l];
      }
    }
    H(k + 1, k) = alpha;
    for (int i = k + 2; i < m; ++i) H(i, k) = 0.0;
  }
}

// Apply the reflector I - beta v v^T (v of length nv, rows r0..r0+nv-1) from
// the left to columns c0..c1 of H, and from the right to columns r0.. of H
// (rows 0..rmax) and of Q (all rows).
void reflect3(Mat &H, Mat &Q, int r0, int nv, const double *v, double beta, int c0, int rmax) {
  const int m = H.m;
  for (int j = c0; j < m; ++j) {
    double s = 0.0;
    for (int l = 0; l < nv; ++l) s += v[l] * H(r0 + l, j);
    s *= beta;
    for (int l = 0; l < nv; ++l) H(r0 + l, j) -= s * v[l];
  }
  for (int i = 0; i <= rmax; ++i) {
    double s = 0.0;
    for (int l = 0; l < nv; ++l) s += H(i, r0 + l) * v[l];
    s *= beta;
    for (int l = 0; l < nv; ++l) H(i, r0 + l) -= s * v[l];
  }
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int l = 0; l < nv; ++l) s += Q(i, r0 + l) * v[l];
    s *= beta;
    for (int l = 0; l < nv; ++l) Q(i, r0 + l) -= s * v[l];
  }
}

// Householder vector of (x, y, z) (nv = 2 or 3): P x = alpha e_1.
bool house(double x, double y, double z, int nv, double *v, double &beta) {
  const double nrm = std::sqrt(x * x + y * y + (nv == 3 ? z * z : 0.0));
  if (nrm == 0.0) return false;
  const double alpha = x > 0 ? -nrm : nrm;
  v[0] = x - alpha;
  v[1] = y;
  if (nv == 3) v[2] = z;
  double vn = v[0] * v[0] + v[1] * v[1] + (nv == 3 ? v[2] * v[2] : 0.0);
  if (vn == 0.0) return false;
  beta = 2.0 / vn;
  return true;
}

// Rotate a 2x2 diagonal block with real eigenvalues to upper triangular form.
void split_real_block(Mat &H, Mat &Q, int k) {
  const int m = H.m;
  const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
  if (c == 0.0) return;
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  const double sq = std::sqrt(std::max(disc, 0.0));
  const double z = p + (p >= 0 ? sq : -sq);  // lambda_1 - d
  double cs = z, sn = c;
  const double r = std::hypot(cs, sn);
  if (r == 0.0) return;
  cs /= r;
  sn /= r;
  // G = [[cs, -sn], [sn, cs]]; H <- G^T H G, Q <- Q G
  for (int j = k; j < m; ++j) {
    const double x = H(k, j), y = H(k + 1, j);
    H(k, j) = cs * x + sn * y;
    H(k + 1, j) = -sn * x + cs * y;
  }
  for (int i = 0; i <= k + 1; ++i) {
    const double x = H(i, k), y = H(i, k + 1);
    H(i, k) = cs * x + sn * y;
    H(i, k + 1) = -sn * x + cs * y;
  }
  for (int i = 0; i < m; ++i) {
    const double x = Q(i, k), y = Q(i, k + 1);
    Q(i, k) = cs * x + sn * y;
    Q(i, k + 1) = -sn * x + cs * y;
  }
  H(k + 1, k) = 0.0;
}

// Francis double-shift QR iteration to real Schur form (T in H, vectors in Q).
int schur(Mat &H, Mat &Q) {
  const int m = H.m;
  double anorm = 0.0;
  for (double x : H.a) anorm = std::max(anorm, std::fabs(x));
  if (anorm == 0.0) anorm = 1.0;
  int hi = m - 1;
  int iter = 0, total = 0;
  const int max_total = 60 * std::max(m, 1);
  double v[3], beta;
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(H(l, l - 1)) <= kEps * s) {
        H(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {  // 1x1 block converged
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {  // 2x2 block converged
      const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      const double p = 0.5 * (a - d);
      if (p * p + b * c >= 0.0) split_real_block(H, Q, hi - 1);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++total > max_total) return -1;
    ++iter;
    double s, t;
    if (iter % 11 == 10) {  // exceptional shift
      const double e = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
      s = 1.5 * e;
      t = e * e;
    } else {
      s = H(hi - 1, hi - 1) + H(hi, hi);
      t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
    }
    // first column of (H - s1 I)(H - s2 I) restricted to the active block
    double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
    double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
    double z = H(l + 1, l) * H(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      if (house(x, y, z, 3, v, beta)) {
        const int c0 = k > l ? k - 1 : l;
        reflect3(H, Q, k, 3, v, beta, c0, std::min(k + 3, hi));
        if (k > l) {
          H(k + 1, k - 1) = 0.0;
          H(k + 2, k - 1) = 0.0;
        }
      }
      x = H(k + 1, k);
      y = H(k + 2, k);
      if (k < hi - 2) z = H(k + 3, k);
    }
    if (house(x, y, 0.0, 2, v, beta)) {
      reflect3(H, Q, hi - 1, 2, v, beta, hi - 2, hi);
      H(hi, hi - 2) = 0.0;
    }
  }
  return 0;
}

}  // namespace

int eig_real(int m, const double *A, int lda, std::vector<cd> &lam, std::vector<cd> &Z,
             std::vector<int> &is_real) {
  lam.assign(m, cd(0, 0));
  Z.assign((size_t)m * m, cd(0, 0));
  is_real.assign(m, 1);
  if (m == 0) return 0;
  Mat H(m), Q(m);
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < m; ++i) H(i, j) = A[(size_t)j * lda + i];
    Q(j, j) = 1.0;
  }
  hessenberg(H, Q);
  if (schur(H, Q) != 0) return -1;
  // blocks of the real Schur form
  std::vector<int> bstart, bsize;
  for (int k = 0; k < m;) {
    if (k + 1 < m && H(k + 1, k) != 0.0) {
      bstart.push_back(k);
      bsize.push_back(2);
      const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
      const double re = 0.5 * (a + d);
      const double p = 0.5 * (a - d);
      const double im = std::sqrt(std::max(-(p * p + b * c), 0.0));
      lam[k] = cd(re, im);
      lam[k + 1] = cd(re, -im);
      is_real[k] = is_real[k + 1] = 0;
      k += 2;
    } else {
      bstart.push_back(k);
      bsize.push_back(1);
      lam[k] = cd(H(k, k), 0.0);
      k += 1;
    }
  }
  double tn = 0.0;
  for (double x : H.a) tn += x * x;
  const double smin = std::max(kEps * std::sqrt(tn), 1e-300);
  const int nb = (int)bstart.size();
  std::vector<cd> x(m);
  for (int bi = 0; bi < nb; ++bi) {
    const int k = bstart[bi], sz = bsize[bi];
    for (int e = 0; e < sz; ++e) {
      const int col = k + e;
      const cd L = lam[col];
      std::fill(x.begin(), x.end(), cd(0, 0));
      if (sz == 1) {
        x[k] = 1.0;
      } else {
        const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
        const cd u1(b), u2 = L - a;          // (T - L) u = 0, first-row form
        const cd w1 = L - d, w2(c);          // second-row form
        if (std::abs(u1) + std::abs(u2) >= std::abs(w1) + std::abs(w2)) {
          x[k] = u1;
          x[k + 1] = u2;
        } else {
          x[k] = w1;
          x[k + 1] = w2;
        }
      }
      for (int bj = bi - 1; bj >= 0; --bj) {
        const int r = bstart[bj], rs = bsize[bj];
        cd rhs[2];
        for (int e2 = 0; e2 < rs; ++e2) {
          cd acc(0, 0);
          for (int jj = r + rs; jj < k + sz; ++jj) acc += H(r + e2, jj) * x[jj];
          rhs[e2] = -acc;
        }
        if (rs == 1) {
          cd dg = H(r, r) - L;
          if (std::abs(dg) < smin) dg = smin;
          x[r] = rhs[0] / dg;
        } else {
          const cd a11 = H(r, r) - L, a12 = H(r, r + 1), a21 = H(r + 1, r), a22 = H(r + 1, r + 1) - L;
          cd det = a11 * a22 - a12 * a21;
          if (std::abs(det) < smin * smin) det = smin * smin;
          x[r] = (rhs[0] * a22 - a12 * rhs[1]) / det;
          x[r + 1] = (a11 * rhs[1] - a21 * rhs[0]) / det;
        }
        double big = 0.0;
        for (int i = r; i < k + sz; ++i) big = std::max(big, std::abs(x[i]));
        if (big > 1e100)
          for (int i = r; i < k + sz; ++i) x[i] /= big;
      }
      // z = Q x, unit 2-norm
      cd *zc = Z.data() + (size_t)col * m;
      double nrm = 0.0;
      for (int i = 0; i < m; ++i) {
        cd acc(0, 0);
        for (int jj = 0; jj < k + sz; ++jj) acc += Q(i, jj) * x[jj];
        zc[i] = acc;
        nrm += std::norm(acc);
      }
      nrm = std::sqrt(nrm);
      if (nrm > 0)
        for (int i = 0; i < m; ++i) zc[i] /= nrm;
    }
  }
  return 0;
}

int solve_complex(int m, std::vector<cd> M, std::vector<cd> &b) {
  std::vector<int> piv(m);
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = std::abs(M[(size_t)k * m + k]);
    for (int i = k + 1; i < m; ++i) {
      const double v = std::abs(M[(size_t)k * m + i]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (best == 0.0) return -1;
    if (p != k) {
      for (int j = 0; j < m; ++j) std::swap(M[(size_t)j * m + k], M[(size_t)j * m + p]);
      std::swap(b[k], b[p]);
    }
    const cd pk = M[(size_t)k * m + k];
    for (int i = k + 1; i < m; ++i) {
      const cd f = M[(size_t)k * m + i] / pk;
      if (f == cd(0, 0)) continue;
      for (int j = k + 1; j < m; ++j) M[(size_t)j * m + i] -= f * M[(size_t)j * m + k];
      b[i] -= f * b[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    cd acc = b[k];
    for (int j = k + 1; j < m; ++j) acc -= M[(size_t)j * m + k] * b[j];
    b[k] = acc / M[(size_t)k * m + k];
  }
  return 0;
}

}  // namespace hla
