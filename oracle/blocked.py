"""Blocked form of the modified FOA: p snapshots per step, in plain NumPy
float64.

Test infrastructure only: imported by tests/, never by the product path.

What it computes.  The modified FOA builds the thin QR factorisation
X_1^N = V_1^N beta_N and the Hessenberg matrix H_bar with
beta_{:,c+1} = H_bar_{:,1:c} beta_{1:c,c} (eq. betacolumnupdate; the QR view
of the factorisation discussed after eq. betacolumnupdate and in Section 3.1).
The blocked form reaches the same factors in exact arithmetic, taking the
snapshots Y = [psi_{q+1} .. psi_{q+p}] of a block together:

1. classical Gram-Schmidt of the whole block against V, twice:
   R1 = V^T Y, Z = Y - V R1, R2 = V^T Z, Z = Z - V R2; and a third time,
   R3 = V^T Z, Z = Z - V R3, when the part of Z still along V after two
   passes may exceed a tenth of the basis's unit roundoff u_V relative to
   ||Z_k|| (see third_projection_needed; R = R1 + R2 (+ R3));
2. the block's own QR, Z = Q S, by one shifted Cholesky QR step followed by
   two plain Cholesky QR steps ("shifted CholeskyQR3": Fukaya, Kannan,
   Nakatsukasa, Yamamoto and Yanagisawa, SIAM J. Sci. Comput. 42 (2020)),
   with the published shift s = 11 (n p + p (p + 1)) u ||Z||_2^2, u = 2^-53,
   and trace(Z^T Z) >= ||Z||_2^2 in its place;
3. beta's new columns [R; S] and V's new columns Q;
4. H_bar's columns c = q .. q+p-1 (1-based) from the recurrence above solved
   for H_bar_{:,c}: H_bar_{:,c} beta_{c,c} = beta_{:,c+1} - H_bar_{:,1:c-1} beta_{1:c-1,c}.

A block is committed only when every new diagonal entry S_kk of beta lies
above the breakdown threshold of the sequential form (tol * ||X_1^{q+k}||_F)
and the three Cholesky factorisations succeed; otherwise its snapshots are
taken one at a time by the sequential oracle (foa.py), which applies the
paper's breakdown and non-finite rules.  The first snapshot (its
normalisation in Algorithm 1) is always taken by the sequential oracle, and
so are the (N - 1) mod p snapshots after it that do not fill a block: first,
while the basis is smallest.

With storage="f32" every stored column of V is rounded to FP32 once it is
final (the FP32 basis of the device form); all arithmetic stays FP64.  Two
projections are then not always enough: V^T V = I + E with E of order
u_32 sqrt(q / n), the part of Z left along V after the passes is about
E^2 R1, and where the block's new directions are as small as ||E|| ||Y||
(noise-floor snapshots, small n) that part is of the size of Z itself and
the basis loses orthogonality block after block.  A third pass multiplies it
by E once more.  ||E|| is estimated by ||R2||_F / ||R1||_F (R2 = -E R1 up to
rounding), so the test costs no extra pass over V.

Parity status: pinned against the sequential oracle (the same exact-arithmetic
factors: tests compare H_bar and beta with foa.foa_batch within O(eps kappa))
and against orthogonality and the factorisation residual.
"""

import numpy as np

from . import foa

PB = 4          # snapshots per block
UNIT = 2.0 ** -53
THIRD_ETA = 0.1  # third projection when the estimated remainder exceeds THIRD_ETA * u_V * ||Z_k||


def _chol_upper(G):
    """Upper-triangular S with G = S^T S, or None when G is not numerically
    positive definite."""
    if not np.all(np.isfinite(G)):
        return None
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(L)) or np.any(np.diag(L) <= 0.0):
        return None
    return L.T


def _right_solve_upper(Z, S):
    """Z S^{-1} for upper-triangular S."""
    return np.linalg.solve(S.T, Z.T).T


def block_qr(Z):
    """Shifted CholeskyQR3 of the n x p block Z: (Q, S) with Z = Q S, or None."""
    n, p = Z.shape
    G = Z.T @ Z
    s = 11.0 * (n * p + p * (p + 1)) * UNIT * np.trace(G)
    S0 = _chol_upper(G + s * np.eye(p))
    if S0 is None:
        return None
    Z1 = _right_solve_upper(Z, S0)
    S1 = _chol_upper(Z1.T @ Z1)
    if S1 is None:
        return None
    Z2 = _right_solve_upper(Z1, S1)
    S2 = _chol_upper(Z2.T @ Z2)
    if S2 is None:
        return None
    Q = _right_solve_upper(Z2, S2)
    return Q, S2 @ S1 @ S0


def third_projection_needed(R1, R2, Z, unit):
    """True when some column of Z (after two projections) may keep a part
    along V larger than THIRD_ETA * unit * ||Z_k||: that part is about E R2_k,
    with ||E|| estimated by ||R2||_F / ||R1||_F."""
    r1 = np.linalg.norm(R1)
    if not r1 > 0.0:
        return False
    e = np.linalg.norm(R2) / r1
    return bool(np.any(e * np.linalg.norm(R2, axis=0) > THIRD_ETA * unit * np.linalg.norm(Z, axis=0)))


def storage_unit(storage):
    return 2.0 ** -24 if storage == "f32" else UNIT


def block_step(st, Y, unit=UNIT):
    """One block of p snapshots (columns of Y) on a state with q >= 1; unit:
    the unit roundoff of V's storage.  Returns True when the block was
    committed, False when it was not (the state is then unchanged)."""
    n, p = Y.shape
    j = st.q
    V = st.V[:, :j]
    yn2 = np.einsum("ij,ij->j", Y, Y)
    if not np.all(np.isfinite(yn2)):
        return False
    R1 = V.T @ Y
    Z = Y - V @ R1
    R2 = V.T @ Z
    Z = Z - V @ R2
    R = R1 + R2
    third = third_projection_needed(R1, R2, Z, unit)
    if third:
        R3 = V.T @ Z
        Z = Z - V @ R3
        R = R + R3
    res = block_qr(Z)
    if res is None:
        return False
    Q, S = res
    xf = st.xfro2 + np.cumsum(yn2)
    if np.any(np.diag(S) <= st.tol * np.sqrt(xf)):
        return False
    beta, H = st.beta, st.H
    beta[:j, j:j + p] = R
    beta[j:j + p, j:j + p] = S
    st.V[:, j:j + p] = Q
    for c in range(j - 1, j + p - 1):      # 0-based column of H_bar
        H[:c + 2, c] = (beta[:c + 2, c + 1] - H[:c + 2, :c] @ beta[:c, c]) / beta[c, c]
        st.hist_h.append(float(H[c + 1, c]))
    st.xfro2 = float(xf[-1])
    st.q = j + p
    st.pushes += p
    st.third_projections = getattr(st, "third_projections", 0) + int(third)
    return True


def round_new_columns(st, q0, storage):
    """FP32 storage: round V's columns q0 .. q-1 (final from now on)."""
    if storage == "f32" and st.q > q0:
        st.V[:, q0:st.q] = st.V[:, q0:st.q].astype(np.float32).astype(np.float64)


def foa_blocked(X, p=PB, tol=None, capacity=None, storage="f64"):
    """The blocked form over X = [psi_1 .. psi_N] (n x N); storage "f64" or
    "f32" (V's final columns rounded to FP32)."""
    X = np.asarray(X, dtype=np.float64)
    n, N = X.shape
    cap = N if capacity is None else int(capacity)
    unit = storage_unit(storage)
    st = foa.foa_stream_init(n, cap, tol)
    st.third_projections = 0
    foa.foa_stream_update(st, X[:, :1])
    round_new_columns(st, 0, storage)
    k = 1
    lead = (N - k) % p
    if lead and st.status == foa.ACTIVE:
        q0 = st.q
        foa.foa_stream_update(st, X[:, k:k + lead])
        round_new_columns(st, q0, storage)
        k += lead
    while k < N:
        q0 = st.q
        if (st.status == foa.ACTIVE and k + p <= N and st.q + p <= cap
                and block_step(st, np.ascontiguousarray(X[:, k:k + p]), unit)):
            round_new_columns(st, q0, storage)
            k += p
            continue
        m = min(p, N - k)
        foa.foa_stream_update(st, X[:, k:k + m])
        round_new_columns(st, q0, storage)
        k += m
    return st
