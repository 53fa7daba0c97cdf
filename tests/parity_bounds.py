"""Tolerances of the GPU-vs-oracle parity tests, derived from the paper's
error analysis (Section 3.2.2) and first-order perturbation theory.  Every
quantity here is computed from the oracle's FP64 results, never from the HIP
path's.

Notation: eps is the unit roundoff scale of the basis storage (2^-52 or
2^-23), kappa_2 = sigma_1 / sigma_min of beta_m, kappa_r = sigma_1 / sigma_r
for a truncation to rank r (the truncated backward error of eq.
foabaseddmdrtkberr is C eps ||X||_2 ||Sigma_r^-1||_2 = C eps kappa_r in the
scale of ||H||), C = 10 (the constant the precision gate states).
"""

import numpy as np
from scipy.optimize import linear_sum_assignment

C = 10.0
EPS64 = 2.0 ** -52


def column_gate_f64(g, st, c=C):
    """Element-wise FP64 gate, column by column: column j of H_bar and of
    beta against c (j+2) eps64 kappa_2 of the leading (j+2) x (j+2) block of
    the oracle's beta (the snapshots column j depends on), relative to the
    largest entry of the leading block.  Returns the largest error / bound
    (columns whose leading block is singular, after a breakdown, are
    skipped)."""
    m, q = g["m"], g["q"]
    worst = 0.0
    for j in range(m):
        k = min(j + 2, q)
        s = np.linalg.svd(st.beta[:k, :k], compute_uv=False)
        if not s[-1] > 0.0:
            continue
        kap = s[0] / s[-1]
        scale = np.abs(st.H[:k, :j + 1]).max()
        eH = np.abs(g["H"][:k, j] - st.H[:k, j]).max() / scale
        sb = np.abs(st.beta[:k, :k]).max()
        eB = np.abs(g["beta"][:k, j + 1] - st.beta[:k, j + 1]).max() / sb if j + 1 < q else 0.0
        tol = c * k * EPS64 * kap
        worst = max(worst, eH / tol, eB / tol)
    return worst


def svals(beta_m):
    return np.linalg.svd(beta_m, compute_uv=False)


def kappa_r(sig, r):
    return float(sig[0] / sig[r - 1])


def gap_factor(sig, r):
    """sigma_r / (sigma_r - sigma_{r+1}): how much a perturbation of beta of
    size eps ||beta|| can turn the r-dimensional dominant subspace (Wedin):
    sin-theta <= ||d beta|| / (sigma_r - sigma_{r+1}) = eps kappa_r * gap_factor."""
    if r >= len(sig):
        return 1.0
    return float(sig[r - 1] / max(sig[r - 1] - sig[r], 1e-300))


def eig_condition(T):
    """Eigenvalues, unit right eigenvectors Z, and per eigenvalue
    cond_i = 1 / |y_i^H z_i| with unit left eigenvectors y_i."""
    lam, Z = np.linalg.eig(T)
    Z = Z / np.linalg.norm(Z, axis=0)
    Y = np.linalg.inv(Z).conj().T          # columns: left eigenvectors, y_i^H z_j = delta_ij
    Yn = Y / np.linalg.norm(Y, axis=0)
    cond = 1.0 / np.abs(np.sum(Yn.conj() * Z, axis=0))
    return lam, Z, Yn, cond


def eigvec_sensitivity(lam, Z, Yn):
    """s_i = sum_{j != i} 1 / (|lambda_i - lambda_j| |y_j^H z_j|): first-order
    bound ||dz_i|| <= ||dT||_2 s_i for a perturbation dT of the matrix."""
    r = lam.shape[0]
    yz = np.abs(np.sum(Yn.conj() * Z, axis=0))
    s = np.empty(r)
    for i in range(r):
        d = np.abs(lam[i] - lam)
        d[i] = np.inf
        s[i] = float(np.sum(1.0 / (np.maximum(d, 1e-300) * yz)))
    return s


def match(a, b):
    """Index pairs (ia, ib) of a min-cost matching of two eigenvalue sets."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    Cm = np.abs(a[:, None] - b[None, :])
    ia, ib = linear_sum_assignment(Cm)
    return ia, ib


def truncated_projection(H_m, beta_m, r):
    """U_r U_r^T H_m U_r U_r^T (basis-free form of U_r^T H_m U_r) and the
    r x r matrix itself."""
    U, _, _ = np.linalg.svd(beta_m)
    Ur = U[:, :r]
    T = Ur.T @ H_m @ Ur
    return Ur @ T @ Ur.T, T, Ur


def eig_gate(lam_gpu, lam_ref, cond, eps, kap):
    """Per matched eigenvalue: |d lambda_i| <= C eps kappa cond_i (Bauer-Fike
    to first order with the backward error C eps kappa ||H||, ||H|| ~ 1 for
    these data: |lambda| <= 1 and H is the projection of a map of norm ~1).
    Returns (max ratio error / bound, max error, per-entry bounds)."""
    ia, ib = match(lam_gpu, lam_ref)
    err = np.abs(np.asarray(lam_gpu)[ia] - np.asarray(lam_ref)[ib])
    bnd = C * eps * kap * np.maximum(1.0, cond[ib])
    return float(np.max(err / bnd)) if len(err) else 0.0, float(err.max()) if len(err) else 0.0, bnd


def phase_aligned_error(phi, ref):
    """min over unit complex a of ||phi - a ref|| / ||ref|| (eigenvectors are
    unique up to a unit factor; the phase convention can pick another)."""
    ip = np.vdot(ref, phi)
    a = ip / abs(ip) if abs(ip) > 0 else 1.0
    return float(np.linalg.norm(phi - a * ref) / np.linalg.norm(ref))


def unpack(Phi, kinds):
    """Complex modes from packed real columns (one per real eigenvalue,
    (Re, Im) per pair)."""
    out, col = [], 0
    for k in kinds:
        if k == 1:
            out.append(Phi[:, col] + 1j * Phi[:, col + 1])
            col += 2
        else:
            out.append(Phi[:, col].astype(np.complex128))
            col += 1
    return out
