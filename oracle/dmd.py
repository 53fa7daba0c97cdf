"""DMD eigenvalues, modes, error indicators and coefficients from the FOA
state: the post-processing of Algorithm 1 and Algorithm 3, Section 3.2.3
(error indicators) and Section 3.2.4 (coefficients of the first snapshot,
eqs. exrecon / exreconwrt).  Plain NumPy float64; test infrastructure only.

Parity status: pinned by tests/test_oracle_pins.py (exact eigenvalue
recovery on exact-rank data, indicator = true residual for a known map A,
exact reconstruction of snapshots 1..N-1, truncation reproducing the
breakdown eigenvalues on rank-deficient data).

Readings where the paper is silent:
* eigenvectors z are scaled to unit 2-norm (Section 3.2.3 assumes unit DMD
  eigenvectors) and their phase is fixed so the entry of largest modulus is
  real and positive;
* modes are ordered by decreasing |c_j| (Section 4.1), ties by decreasing
  |lambda|, then by index;
* truncation rank: r = #{sigma_i(beta_m) > N eps_s(sigma_1)}, N the number of
  snapshots taken, eps_s the spacing at sigma_1 in the storage precision
  (numerical rank rule of Section 4.1).
"""

import numpy as np

from .foa import INVARIANT


def projected_size(st) -> int:
    """Order m of the projected matrix: q-1 normally (H_{q-1}), q after an
    invariant breakdown (the square H_q is then complete)."""
    return st.q if st.status == INVARIANT else st.q - 1


def spacing(x: float, storage: str = "f64") -> float:
    """eps(x): distance from |x| to the next larger number of the storage type."""
    if storage == "f32":
        return float(np.spacing(np.float32(abs(x))))
    return float(np.spacing(np.float64(abs(x))))


def kappa2(M) -> float:
    s = np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")


def truncation_rank(sigma, nsnap: int, storage: str = "f64") -> int:
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.size == 0:
        return 0
    thr = nsnap * spacing(sigma[0], storage)
    return int(np.count_nonzero(sigma > thr))


def _unit_phase(Z):
    Z = Z.astype(np.complex128, copy=True)
    for i in range(Z.shape[1]):
        z = Z[:, i]
        z /= np.linalg.norm(z)
        k = int(np.argmax(np.abs(z)))
        z *= np.conj(z[k]) / abs(z[k])
        Z[:, i] = z
    return Z


def _order(lam, c):
    idx = np.arange(lam.shape[0])
    keys = sorted(idx, key=lambda i: (-abs(c[i]), -abs(lam[i]), i))
    return np.asarray(keys, dtype=np.int64)


def dmd_untruncated(st):
    """Untruncated DMD of Algorithm 1: eig(H_m); indicators |h_{m+1,m}| |e_m^T z_i| (eq. errordmdvec);
    coefficients [z]{c} = ||psi_1|| e_1 (eq. exrecon)."""
    m = projected_size(st)
    Hm = st.H[:m, :m].copy()
    lam, Z = np.linalg.eig(Hm)
    Z = _unit_phase(Z)
    hlast = 0.0 if st.status == INVARIANT else float(st.H[m, m - 1])
    ind = abs(hlast) * np.abs(Z[m - 1, :])
    rhs = np.zeros(m, dtype=np.complex128)
    rhs[0] = st.beta[0, 0]
    c = np.linalg.solve(Z, rhs)
    order = _order(lam, c)
    return {
        "m": m,
        "lam": lam,
        "Z": Z,            # eigenvectors in the V_{1:m} basis
        "B": Z,            # coefficients of the modes in the V_{1:m} basis
        "indicators": ind,
        "coef": c,
        "order": order,
    }


def dmd_truncated(st, r: int):
    """Truncated DMD of Algorithm 1: SVD of beta_m, U_r^T H_m U_r, its eigenpairs; indicators
    ||[(I - U_r U_r^T) H_m ; h_{m+1,m} e_m^T] U_r z_i||_2 (Section 3.2.3);
    coefficients [z]{c} = ||psi_1|| U_r^T e_1 (eq. exreconwrt)."""
    m = projected_size(st)
    Hm = st.H[:m, :m].copy()
    U, S, _ = np.linalg.svd(st.beta[:m, :m])
    Ur = U[:, :r]
    Ht = Ur.T @ Hm @ Ur
    lam, Z = np.linalg.eig(Ht)
    Z = _unit_phase(Z)
    hlast = 0.0 if st.status == INVARIANT else float(st.H[m, m - 1])
    P = np.eye(m) - Ur @ Ur.T
    ind = np.empty(r)
    for i in range(r):
        y = Ur @ Z[:, i]
        top = P @ (Hm @ y)
        bot = hlast * y[m - 1]
        ind[i] = np.sqrt(np.linalg.norm(top) ** 2 + abs(bot) ** 2)
    rhs = st.beta[0, 0] * Ur[0, :].astype(np.complex128)
    c = np.linalg.solve(Z, rhs)
    order = _order(lam, c)
    return {
        "m": m,
        "r": r,
        "sigma": S,
        "Ur": Ur,
        "lam": lam,
        "Z": Z,
        "B": Ur @ Z,
        "indicators": ind,
        "coef": c,
        "order": order,
    }


def packed_modes(res, V):
    """Modes V_{1:m} B as packed real columns in the mode order: a real
    eigenvalue gives one column, a conjugate pair one (Re, Im) column pair
    for its member with Im > 0.  Returns (Phi, lam_list, kinds)."""
    m = res["m"]
    Phi_c = V[:, :m] @ res["B"]
    cols, lams, kinds = [], [], []
    for i in res["order"]:
        lam = res["lam"][i]
        if lam.imag < 0:
            continue
        if lam.imag == 0:
            cols.append(Phi_c[:, i].real)
            kinds.append(0)
        else:
            cols.append(Phi_c[:, i].real)
            cols.append(Phi_c[:, i].imag)
            kinds.append(1)
        lams.append(lam)
    Phi = np.stack(cols, axis=1) if cols else np.zeros((V.shape[0], 0))
    return Phi, np.asarray(lams), np.asarray(kinds, dtype=np.int8)
