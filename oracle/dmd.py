"""DMD eigenvalues, modes, error indicators and coefficients from the FOA
state: the post-processing of Algorithm 1 and Algorithm 3, Section 3.2.3
(error indicators) and Section 3.2.4 (coefficients of the first snapshot,
eqs. exrecon / exreconwrt).  Plain NumPy float64; test infrastructure only.

Parity status: pinned by tests/test_oracle_pins.py: exact eigenvalue
recovery on exact-rank data; untruncated and truncated indicators equal to
the true residual ||A phi - lambda phi|| for a known map A; truncated
coefficients equal to the least-squares fit of psi_1 by the explicit modes;
exact reconstruction of snapshots 1..N-1 from the packed real mode columns;
the rank rule on hand-computed singular values in both storage precisions;
truncation reproducing the breakdown eigenvalues on rank-deficient data.

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
    """Numerical rank of beta_m (the rule of Section 4.1 read with the storage
    precision): singular values above nsnap times the spacing at sigma_1."""
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
    """Untruncated DMD (Algorithm 1 without rank truncation): eigenpairs of the
    square leading block H_m.  The error indicator of an eigenpair is the size
    of the Arnoldi residual term, |h_{m+1,m}| times the last entry of the unit
    eigenvector (Section 3.2.3, eq. errordmdvec).  The coefficients c of
    psi_1 in the mode basis solve [z] c = V^T psi_1 = ||psi_1|| e_1, since
    psi_1 = ||psi_1|| v_1 (eq. exrecon)."""
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
    """Rank-truncated DMD (Algorithm 1 with rank truncation): beta_m = U S W^T,
    the projection U_r^T H_m U_r onto the r dominant left singular directions,
    and its eigenpairs (lambda, z); the modes are V_{1:m} U_r z.

    Indicator (Section 3.2.3): with A V_{1:m} = V_{1:m} H_m + h_{m+1,m}
    v_{m+1} e_m^T and lambda U_r z = U_r U_r^T H_m U_r z, the residual
    A V U_r z - lambda V U_r z has coordinates (I - U_r U_r^T) H_m U_r z in
    V_{1:m} and h_{m+1,m} (U_r z)_m along v_{m+1}; its norm is the indicator.

    Coefficients (eq. exreconwrt): V_{1:m} U_r has orthonormal columns, so
    the least-squares fit of psi_1 = ||psi_1|| v_1 by the modes solves
    [z] c = ||psi_1|| U_r^T e_1."""
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
        inside = P @ (Hm @ y)          # coordinates in V_{1:m}
        along = hlast * y[m - 1]       # coordinate along v_{m+1}
        ind[i] = np.sqrt(np.linalg.norm(inside) ** 2 + abs(along) ** 2)
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


def packed_coefficients(res):
    """Coefficients c_j of psi_1 for the entries of packed_modes, in the same
    order (one per real eigenvalue, one per conjugate pair: that of its Im > 0
    member; the other member's is the conjugate for real snapshots)."""
    return np.asarray([res["coef"][i] for i in res["order"] if res["lam"][i].imag >= 0],
                      dtype=np.complex128)
