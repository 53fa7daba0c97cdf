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
# One iteration j (1-based) of the loop of Algorithm 1 / Algorithm 4, in the
# order the method needs its quantities:
#   * the part of beta's column j+1 that the known columns of H_bar give,
#   * the vector A v_j recovered from the snapshot psi_{j+1},
#   * its orthogonalisation against V_1^j (classical Gram-Schmidt, twice),
#     which yields H_bar's column j,
#   * the normalisation that appends v_{j+1},
#   * the rest of beta's column j+1 from the new Hessenberg column.
# ---------------------------------------------------------------------------

def _partial_beta_column(H, beta, j):
    """Expansion coefficients of psi_{j+1} in V_1^j, minus the contribution
    of the Hessenberg column not yet known.

    psi_{j+1} = A psi_j = A V_1^j beta_{1:j,j}; A maps v_1..v_{j-1} through the
    first j-1 columns of H_bar (eq. avarnoldi), so the known part is the
    product of the j x (j-1) leading block of H_bar with beta_{1:j-1,j}
    (eq. betacolumnupdate; H_bar is upper Hessenberg, so the product is
    banded).  Returns a vector of length j."""
    return H[:j, :j - 1] @ beta[:j - 1, j - 1]


def _arnoldi_vector(V, b, bjj, psi, j):
    """A v_j from the snapshot: psi_{j+1} = V_1^j b + beta_{jj} A v_j, with b
    the partial column above (eq. avpsijp1beta)."""
    return (psi - V[:, :j] @ b) / bjj


def _cgs2(V, w, j):
    """Classical Gram-Schmidt against V_1^j with one reorthogonalisation:
    two projection passes, each removing V_1^j V_1^jT w from w and adding
    its coefficients to the Hessenberg column.  Returns (H_bar[0:j, j-1], w)."""
    Vj = V[:, :j]
    h = np.zeros(j)
    for _ in range(2):
        s = Vj.T @ w
        w = w - Vj @ s
        h = h + s
    return h, w


def _norm(w):
    """2-norm (the normalisation of w, and of the first snapshot)."""
    return float(np.sqrt(w @ w))


def _completed_beta_column(b, hcol, bjj):
    """Column j+1 of beta (rows 1..j+1): the partial column plus A v_j's share,
    beta_{jj} times H_bar's column j (eq. betacolumnupdate)."""
    col = np.zeros(hcol.shape[0])
    col[:b.shape[0]] = b
    return col + hcol * bjj


def _first(st: FOAState, psi1):
    """First snapshot: beta_11 = ||psi_1|| and v_1 = psi_1 / beta_11."""
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
    """Iteration j (1-based) of the loop of Algorithm 1: consumes psi_{j+1}.
    Nothing is written to the state before every new quantity is finite."""
    V, H, beta = st.V, st.H, st.beta
    st.pushes += 1
    xn2 = float(psi @ psi)
    if not np.isfinite(xn2):
        st.status = NONFINITE
        return
    bjj = beta[j - 1, j - 1]
    b = _partial_beta_column(H, beta, j)
    w = _arnoldi_vector(V, b, bjj, psi, j)
    h, w = _cgs2(V, w, j)
    hn = _norm(w)
    if not (np.all(np.isfinite(h)) and np.isfinite(hn)):
        st.status = NONFINITE
        return
    st.xfro2 += xn2
    st.hist_h.append(hn)
    # psi_{j+1} in span(v_1..v_j) (the reading of h_{j+1,j} = 0 stated above):
    # the exact Ritz pairs are in the square H_j (Section 3.2.4), stop
    dependent = hn * bjj <= st.tol * np.sqrt(st.xfro2)
    hcol = np.append(h, 0.0 if dependent else hn)
    H[:j + 1, j - 1] = hcol
    beta[:j + 1, j] = _completed_beta_column(b, hcol, bjj)
    if dependent:
        st.status = INVARIANT
        return
    V[:, j] = w / hn
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
    """Arnoldi's method with the map A known (Algorithm 2), orthogonalising
    with two classical Gram-Schmidt passes (its own code, so that a mistake in
    the FOA helpers does not carry over to this reference).

    Returns (V (n x N), H_bar (N x (N-1)))."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    V = np.zeros((n, N), order="F")
    H = np.zeros((N, N - 1), order="F")
    V[:, 0] = psi1 / _norm(psi1)
    for j in range(1, N):
        w = A @ V[:, j - 1]                 # Krylov step
        Vj = V[:, :j]
        h = np.zeros(j)
        for _ in range(2):                  # written out here, independent of _cgs2
            c = Vj.T @ w
            w = w - Vj @ c
            h = h + c
        hn = _norm(w)
        H[:j, j - 1] = h
        H[j, j - 1] = hn
        V[:, j] = w / hn
    return V, H
