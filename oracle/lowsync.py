"""One-reduction form of the FOA step: the factorisation X_1^q = V beta and
H_bar of the modified FOA reached with one sweep over the basis and one global
reduction per snapshot, in plain NumPy float64 (test infrastructure only;
never imported by the product path).

The modified FOA is the thin QR factorisation of the snapshots with H_bar
following from beta (the QR view of Section 3.1: beta_{:,j+1} =
H_bar_{:,1:j} beta_{1:j,j}, eq. betacolumnupdate, solved for H_bar's column
j).  Algorithm 1 orthogonalises with classical Gram-Schmidt applied twice;
each of its two projections needs a global reduction before the next can
start, which is the message count the paper weighs in Section 3.2.5.  This
form orthogonalises the snapshots themselves with the two projections of
CGS2 spread over consecutive pushes (the delayed reorthogonalisation of
Bielich, Langou, Thomas, Swirydowicz, Yamazaki and Boman, "Low-synch
Gram-Schmidt with delayed reorthogonalization for Krylov solvers", Parallel
Computing 2022).  The sweep of push t+1 over the rows:
  * finishes column t-1: its second projection u - Q w (w = Q^T u from the
    previous reduction);
  * gives snapshot t its first projection: x_t - Q z - q_hat R_tilde, where z
    = Q^T x_t and the coefficient R_tilde on the column just finished come
    from the previous reduction (the latter through the identity
    (u - Q w)^T x = u^T x - w^T z, with the column's norm estimated as
    sqrt(||u||^2 - ||w||^2));
  * takes in snapshot t+1 (copied into the next basis column, so the caller
    may reuse its buffer after the push);
and the one reduction of its column sums gives the exact norm of column
t-1, w for column t, and z for snapshot t+1.  Coefficients computed against
the estimated norm are rescaled once the exact norm is known, so the
estimate only affects the first projection, which the second corrects.  A
column is therefore final two pushes after its snapshot; ``flush`` finishes
the pending columns (two sweeps without a new snapshot).

Storage: columns hold unnormalised vectors; q_c = sigma_c column_c with
sigma_c = 1 / ||column_c||.  With storage="f32" every stored column is
rounded to float32 (all arithmetic stays float64), the precision form of the
library's FP32 basis.

Non-orthogonality of the stored basis.  A stored column is rounded after it
is orthogonalised, so the final columns are orthonormal only up to
E = Q^T Q - I (entries of order eps32 / sqrt(n) with an FP32 basis).  Two
projections that treat Q as orthonormal leave components of order ||E|| ||x||
along Q; once that reaches the residual of a new snapshot (snapshots near the
noise floor of the data, small n) the error compounds from column to column.
The second projection (the reorthogonalisation) therefore uses the
coefficients (I - E) w in place of w: the projector Q (I - E) Q^T differs from
the orthogonal projector onto span(Q) by O(||E||^2), so the column it leaves
is orthogonal to the stored basis to O(||E||^2) whatever the first projection
left.  E gains a column when a column becomes final: its inner products with
the earlier final columns, from the same sweep's column sums.  With an FP64
basis E is of order eps64 and the correction changes results at rounding
level only.

Breakdown (the reading of the exact-arithmetic condition h_{j+1,j} = 0 used
for the sequential form): column c is dependent when its exact norm
beta_{c,c} <= tol ||X_1^c||_F.  The stream then becomes invariant with the c-1
columns before it; its beta column c (rows 1..c-1) and H_bar column c-1 (with
h_{c,c-1} = 0) are kept.  A snapshot with a non-finite entry is dropped and
the stream stops; the snapshots before it are completed by the flush.

Parity status: pinned by tests/test_oracle_lowsync.py against Householder QR
(QR uniqueness), the sequential oracle, orthogonality and factorisation bounds
with both storage precisions, exact-rank breakdown, the flush rules and the
one-sweep access count.
"""

from dataclasses import dataclass, field

import numpy as np

from .foa import EPS64, default_breakdown_tol

ACTIVE = "active"
INVARIANT = "invariant"
NONFINITE = "nonfinite"
ZERO_FIRST = "zero_first"


@dataclass
class LowSyncState:
    V: np.ndarray                 # (n, cap + 2): final columns 0..q-1, then pending ones
    H: np.ndarray                 # (cap, cap) H_bar
    beta: np.ndarray              # (cap, cap)
    sigma: np.ndarray             # scales of the final columns
    storage: str = "f64"
    q: int = 0                    # final columns
    status: str = ACTIVE
    tol: float = 0.0
    xn2: list = field(default_factory=list)   # ||x_c||^2 of the accepted snapshots
    # pending column under its second projection (at index q): w = Q^T u, alpha = ||u||^2
    has_u: bool = False
    w: np.ndarray = None
    alpha: float = 0.0
    # pending snapshot copy (at index q + has_u): z = Q^T x (first projection
    # coefficients on the final columns); gamma = u^T x when a column is pending
    has_x: bool = False
    z: np.ndarray = None
    gamma: float = 0.0
    pushes: int = 0
    sweeps: int = 0
    E: np.ndarray = None          # Q^T Q - I of the final columns (cap x cap)
    w_hat: np.ndarray = None      # (I - E) w, the second-projection coefficients used


def init(n, capacity, tol=None, storage="f64") -> LowSyncState:
    tol = default_breakdown_tol(capacity) if tol is None or tol < 0 else float(tol)
    return LowSyncState(V=np.zeros((n, capacity + 2), order="F"), H=np.zeros((capacity, capacity), order="F"),
                        beta=np.zeros((capacity, capacity), order="F"), sigma=np.zeros(capacity + 2),
                        storage=storage, tol=tol, E=np.zeros((capacity, capacity)))


def _store(st, v):
    return v.astype(np.float32).astype(np.float64) if st.storage == "f32" else v


def _hbar_column(st, c):
    """H_bar's column c-1 (0-based) once beta's column c is final: solve
    beta_{:,c} = H_bar_{:,0:c} beta_{0:c,c-1} (eq. betacolumnupdate) for it."""
    b = st.H[:c, :c - 1] @ st.beta[:c - 1, c - 1]
    col = st.beta[:c + 1, c].copy()
    col[:c] -= b
    st.H[:c + 1, c - 1] = col / st.beta[c - 1, c - 1]


def _sweep(st, x):
    """One sweep over the rows (x: the new snapshot, or None for a flush
    sweep), then the quantities of its one reduction."""
    q = st.q
    Q = st.V[:, :q] * st.sigma[:q]              # final columns, normalised
    st.sweeps += 1
    # ||u - Q w_hat||^2 = ||u||^2 - w^T w_hat + O(||E||^2)
    rho_hat = np.sqrt(max(st.alpha - float(st.w @ st.w_hat), 0.0)) if st.has_u else 0.0
    # 1. second projection of the pending column (index q)
    if st.has_u:
        ut = _store(st, st.V[:, q] - Q @ st.w_hat)
        st.V[:, q] = ut
    # 2. first projection of the pending snapshot copy
    iu = q + (1 if st.has_u else 0)           # where the snapshot copy sits
    if st.has_x:
        r_t = 0.0
        if st.has_u and rho_hat > 0.0:
            r_t = (st.gamma - float(st.w_hat @ st.z)) / rho_hat
        u = st.V[:, iu] - Q @ st.z
        if st.has_u and rho_hat > 0.0:
            u = u - ut * (r_t / rho_hat)    # q_hat R_tilde with q_hat = ut / rho_hat
        u = _store(st, u)
        st.V[:, iu] = u
    # 3. the new snapshot, copied into the next column
    ix = iu + (1 if st.has_x else 0)
    if x is not None:
        xs = _store(st, x)
        st.V[:, ix] = xs
        xn2 = float(x @ x)
    # ---- the one reduction: column sums against Q and the pending vectors ----
    if st.has_u:
        nu2 = float(ut @ ut)
        gq = Q.T @ ut                    # the finished (stored) column against Q
    if st.has_x:
        wq, alpha = Q.T @ u, float(u @ u)
        wu = float(ut @ u) if st.has_u else None
    if x is not None:
        zq = Q.T @ xs
        zu = float(ut @ xs) if st.has_u else None
        gx = float(u @ xs) if st.has_x else None
    # ---- finalize -----------------------------------------------------------
    if x is not None and not np.isfinite(xn2):
        st.status = NONFINITE           # x dropped; what came before is kept
        x = None
    if x is not None and q == 0 and not st.has_u and not st.has_x and xn2 == 0.0:
        st.status = ZERO_FIRST
        return
    if st.has_u:
        rho = np.sqrt(nu2)
        c = q                            # column c (0-based) is now complete
        xf = np.sqrt(sum(st.xn2[:c + 1]))
        if rho <= st.tol * xf:
            st.beta[c, c] = 0.0
            if c > 0:
                _hbar_column(st, c)
            st.status = INVARIANT
            st.has_u = st.has_x = False
            return
        st.beta[c, c] = rho
        st.sigma[c] = 1.0 / rho
        st.E[:c, c] = st.E[c, :c] = gq / rho     # E gains the new final column
        if c > 0:
            _hbar_column(st, c)
        st.q = q = c + 1
        st.has_u = False
    if st.has_x:
        # the snapshot copy became the pending column: its coefficients on the
        # final columns are the first projection plus the second one
        k = st.q - 1                     # column just finished, if any (index q-1)
        wfull = wq.copy()
        p = st.z.copy()
        if wu is not None:               # a column was finished in this sweep
            wfull = np.append(wfull, wu * st.sigma[k])
            p = np.append(p, (rho / rho_hat) * r_t if rho_hat > 0.0 else 0.0)
        c = st.q                         # 0-based index of this column
        w_hat = wfull - st.E[:c, :c] @ wfull
        st.beta[:c, c] = p + w_hat       # the coefficients actually subtracted
        st.has_u, st.w, st.w_hat, st.alpha = True, wfull, w_hat, alpha
        st.has_x = False
    if x is not None:
        zfull = zq.copy()
        if zu is not None:
            zfull = np.append(zfull, zu * st.sigma[st.q - 1])
        st.has_x, st.z = True, zfull
        st.gamma = gx if gx is not None else 0.0
        st.xn2.append(xn2)


def push(st: LowSyncState, x):
    """Take one snapshot (one sweep and one reduction)."""
    st.pushes += 1
    if st.status != ACTIVE:
        return st
    pend = st.q + int(st.has_u) + int(st.has_x)
    if pend >= st.H.shape[0]:
        raise ValueError("capacity exceeded")
    _sweep(st, np.asarray(x, dtype=np.float64))
    return st


def flush(st: LowSyncState):
    """Finish the pending columns: sweeps without a new snapshot until none
    is pending (at most two)."""
    while st.status in (ACTIVE, NONFINITE) and (st.has_u or st.has_x):
        _sweep(st, None)
    return st


def run(X, tol=None, storage="f64", capacity=None):
    """All columns of X (n x N) pushed, then flushed."""
    X = np.asarray(X, dtype=np.float64)
    n, N = X.shape
    st = init(n, N if capacity is None else capacity, tol, storage)
    for j in range(N):
        push(st, np.ascontiguousarray(X[:, j]))
    return flush(st)


def basis(st):
    """Normalised final columns V_{1:q}."""
    return st.V[:, :st.q] * st.sigma[:st.q]
