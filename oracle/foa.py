"""Modified FOA (the factorisation X_1^N = V_1^N beta_N with the projected
Hessenberg matrix H_bar_N) in plain NumPy float64.

Test infrastructure only: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Parity status: pinned.  tests/test_oracle_pins.py checks it against
Householder QR of the snapshots (QR uniqueness, Section 3.1 factorisation
view), the closed form H_bar = beta_{1:N,2:N} beta_{N-1}^{-1}
(eq. betacolumnupdate), exact recovery of generating eigenvalues on
exact-rank data (Section 3.2.4 breakdown argument), Algorithm 2 on a known
map A (eq. avarnoldi), the orthogonality and backward-error bounds of
eqs. qrfactorth / errorinfact / matmulhbeta, and a hand-derived example
(tests/golden/diag2_worked.json).

Index convention: paper indices are 1-based; arrays here are 0-based, so the
paper's h_{i,j} is ``H[i-1, j-1]`` and beta_{i,j} is ``beta[i-1, j-1]``.

Reading of the breakdown rule (the paper states only the exact-arithmetic
condition h_{j+1,j} = 0 for a snapshot in the span of its predecessors, and
that N is then reduced to the independent prefix): in iteration j the
snapshot psi_{j+1} is declared dependent when
    beta_{j+1,j+1} = h_{j+1,j} beta_{j,j} <= tol * ||X_1^{j+1}||_F,
with tol defaulting to capacity * 2^-52 (the numerical-rank scale of
Section 4.1, N eps(.)).  On breakdown column j of H_bar (rows 1..j) and
column j+1 of beta (rows 1..j) are kept, h_{j+1,j} is set to 0, no v_{j+1}
is appended, q stays j and the state becomes invariant: the square H_q then
holds the exact Ritz pairs.  A snapshot with a non-finite entry stops the
run with nothing of it kept.
"""

from dataclasses import dataclass, field

import numpy as np

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23

ACTIVE = "active"
INVARIANT = "invariant"
NONFINITE = "nonfinite"
ZERO_FIRST = "zero_first"


def default_breakdown_tol(capacity: int) -> float:
    """tol = N eps with N the snapshot capacity (numerical rank scale, Section 4.1)."""
    return float(capacity) * EPS64


@dataclass
class FOAState:
    """The state tuple (H, V, beta, q) of Algorithm 4 plus bookkeeping."""

    V: np.ndarray          # (n, cap) Arnoldi vectors in columns 0..q-1
    H: np.ndarray          # (cap, cap) H_bar: rows 0..q-1, columns 0..q-2 (q-1 with invariant)
    beta: np.ndarray       # (cap, cap) upper triangular, columns 0..q-1 (q with invariant)
    q: int = 0
    status: str = ACTIVE
    tol: float = 0.0
    xfro2: float = 0.0     # ||X_1^q||_F^2 of the snapshots taken so far
    pushes: int = 0        # snapshots offered, including ignored ones
    hist_h: list = field(default_factory=list)  # h_{j+1,j} per iteration


def _new_state(n: int, cap: int, tol) -> FOAState:
    tol = default_breakdown_tol(cap) if tol is None or tol < 0 else float(tol)
    return FOAState(
        V=np.zeros((n, cap), dtype=np.float64, order="F"),
        H=np.zeros((cap, cap), dtype=np.float64, order="F"),
        beta=np.zeros((cap, cap), dtype=np.float64, order="F"),
        tol=tol,
    )


# ---------------------------------------------------------------------------
# One iteration j (1-based) of Algorithm 1 / Algorithm 4, split into the
# paper's stages in its order: partial beta column, w from the snapshot,
# CGS2, normalisation, beta completion.  Each helper does exactly the
# operations of its stage.
# ---------------------------------------------------------------------------

def _beta_partial(H, beta, j):
    """Partial beta column (eq. betacolumnupdate without its last term):
    beta_{1,j+1} = h_{1,1:j-1} beta_{1:j-1,j};
    beta_{i,j+1} = h_{i,i-1:j-1} beta_{i-1:j-1,j}, i = 2..j."""
    beta[0, j] = H[0, 0:j - 1] @ beta[0:j - 1, j - 1]
    for i in range(2, j + 1):
        beta[i - 1, j] = H[i - 1, i - 2:j - 1] @ beta[i - 2:j - 1, j - 1]


def _form_w(V, beta, psi, j):
    """w from the snapshot: w = (psi_{j+1} - sum_{i<=j} beta_{i,j+1} v_i) / beta_{j,j},
    which equals A v_j (eq. avpsijp1beta)."""
    return (psi - V[:, :j] @ beta[:j, j]) / beta[j - 1, j - 1]


def _cgs2(V, w, j):
    """Classical Gram-Schmidt with one reorthogonalisation (Algorithm 1)."""
    h = V[:, :j].T @ w          # projection
    w = w - V[:, :j] @ h        # first orthogonalisation
    s = V[:, :j].T @ w          # reprojection
    h = h + s                   # corrected Hessenberg column
    w = w - V[:, :j] @ s        # second orthogonalisation
    return h, w


def _norm(w):
    """2-norm (the normalisation of w, and of the first snapshot)."""
    return float(np.sqrt(w @ w))


def _beta_complete(H, beta, j):
    """Beta completion: beta_{i,j+1} += h_{i,j} beta_{j,j}, i = 1..j+1."""
    for i in range(1, j + 2):
        beta[i - 1, j] = beta[i - 1, j] + H[i - 1, j - 1] * beta[j - 1, j - 1]


def _first(st: FOAState, psi1):
    """First snapshot of Algorithm 1 / Algorithm 4: beta_11 = ||psi_1||, v_1 = psi_1 / beta_11."""
    nrm2 = float(psi1 @ psi1)
    st.pushes += 1
    if not np.isfinite(nrm2):
        st.status = NONFINITE
        return
    b11 = float(np.sqrt(nrm2))
    if b11 == 0.0:
        st.status = ZERO_FIRST
        return
    st.beta[0, 0] = b11
    st.V[:, 0] = psi1 / b11
    st.xfro2 = nrm2
    st.q = 1


def _iteration(st: FOAState, psi, j):
    """Iteration j (1-based) of the loop of Algorithm 1: consumes psi_{j+1}."""
    V, H, beta = st.V, st.H, st.beta
    st.pushes += 1
    xn2 = float(psi @ psi)
    if not np.isfinite(xn2):
        st.status = NONFINITE
        return
    saved = beta[:j + 1, j].copy()
    _beta_partial(H, beta, j)
    w = _form_w(V, beta, psi, j)
    h, w = _cgs2(V, w, j)
    hn = _norm(w)
    if not (np.all(np.isfinite(h)) and np.isfinite(hn)):
        beta[:j + 1, j] = saved
        st.status = NONFINITE
        return
    st.xfro2 += xn2
    H[:j, j - 1] = h
    bnew = hn * beta[j - 1, j - 1]
    st.hist_h.append(hn)
    if bnew <= st.tol * np.sqrt(st.xfro2):
        # psi_{j+1} lies in span(v_1..v_j): exact Ritz pairs, stop (Section 3.2.4)
        H[j, j - 1] = 0.0
        _beta_complete(H, beta, j)
        st.status = INVARIANT
        return
    H[j, j - 1] = hn              # normalisation
    V[:, j] = w / hn
    _beta_complete(H, beta, j)
    st.q = j + 1


def foa_batch(X, tol=None, capacity=None) -> FOAState:
    """Algorithm 1 up to the basis (its snapshot loop), for X = [psi_1 .. psi_N] (n x N)."""
    X = np.asarray(X, dtype=np.float64)
    n, N = X.shape
    cap = N if capacity is None else int(capacity)
    st = _new_state(n, cap, tol)
    _first(st, np.ascontiguousarray(X[:, 0]))
    for j in range(1, N):
        if st.status != ACTIVE:
            st.pushes += 1
            continue
        _iteration(st, np.ascontiguousarray(X[:, j]), j)
    return st


def foa_stream_init(n: int, capacity: int, tol=None) -> FOAState:
    """Initial state of Algorithm 3 (q = 0) with storage for ``capacity`` snapshots."""
    return _new_state(int(n), int(capacity), tol)


def foa_stream_update(st: FOAState, Xp) -> FOAState:
    """Algorithm 4: process the p new snapshots in the columns of ``Xp``.

    The storage is preallocated to the capacity, so 'expanding' H, V and beta
    for new snapshots only widens the logical extent.  For a given total number of
    snapshots the result equals Algorithm 1 bit for bit (same operations in
    the same order, Section 3.1).
    """
    Xp = np.asarray(Xp, dtype=np.float64)
    if Xp.ndim == 1:
        Xp = Xp[:, None]
    n, p = Xp.shape
    if st.q + p > st.V.shape[1] and st.status == ACTIVE:
        raise ValueError("capacity exceeded")
    k = 0
    if st.q == 0 and st.status == ACTIVE and st.pushes == 0:
        _first(st, np.ascontiguousarray(Xp[:, 0]))
        k = 1
    for c in range(k, p):
        if st.status != ACTIVE:
            st.pushes += 1
            continue
        j = st.q  # iteration index: consumes psi_{q+1}
        _iteration(st, np.ascontiguousarray(Xp[:, c]), j)
    return st


# ---------------------------------------------------------------------------
# Algorithm 2: Rayleigh-Ritz with the standard Arnoldi method (known A).
# Used only as a reference for the known-A tests.
# ---------------------------------------------------------------------------

def arnoldi_known_A(A, psi1, N):
    """Algorithm 2's Arnoldi loop with CGS2 orthogonalisation.

    Returns (V (n x N), H_bar (N x (N-1)))."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    V = np.zeros((n, N), order="F")
    H = np.zeros((N, N - 1), order="F")
    V[:, 0] = psi1 / _norm(psi1)
    for j in range(1, N):
        w = A @ V[:, j - 1]                 # Krylov step
        h = V[:, :j].T @ w                  # projection
        w = w - V[:, :j] @ h                # first orthogonalisation
        s = V[:, :j].T @ w                  # reprojection
        h = h + s
        w = w - V[:, :j] @ s                # second orthogonalisation
        hn = _norm(w)
        H[:j, j - 1] = h
        H[j, j - 1] = hn
        V[:, j] = w / hn
    return V, H
