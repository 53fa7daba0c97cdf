"""Pins of the blocked oracle (oracle/blocked.py) against facts it does not
define: the sequential oracle (itself pinned), Householder QR, orthogonality,
the factorisation residual, exact-rank recovery with the breakdown rule, and
the O(eps kappa) growth of the projection error (Section 3.2.2).  Planted
mistakes must fail at least one of them."""

import numpy as np
import pytest

import datagen
import oracle.blocked as ob
import oracle.foa as ofoa
from pins import _krylov, match_eigs

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23


def _noisy(n=3000, N=61, name="noisy_2p20x200"):
    w = datagen.get_workload(name).with_n(n).with_N(N)
    X, lam, b = datagen.snapshots_numpy(w, dtype="float64")
    return X


def pin_matches_sequential(B):
    """Same factors as the sequential oracle within O(q eps kappa)."""
    out = []
    for name, n in (("noisy_2p20x200", 3000), ("noisy_2p24x500", 20000)):
        X = _noisy(n, 61, name)
        a = ofoa.foa_batch(X)
        b = B.foa_blocked(X)
        q, m = a.q, a.q - 1
        kap = np.linalg.cond(a.beta[:m, :m])
        eH = np.linalg.norm(b.H[:m, :m] - a.H[:m, :m], 2) / np.linalg.norm(a.H[:m, :m], 2)
        eB = np.linalg.norm(b.beta[:q, :q] - a.beta[:q, :q]) / np.linalg.norm(a.beta[:q, :q])
        out.append(b.q == q and eH <= 10 * q * EPS64 * kap and eB <= 10 * q * EPS64 * kap)
    return all(out)


def pin_orthogonal_factorisation(B):
    """||I - V^T V|| <= 10 sqrt(q) eps and X = V beta to 10 sqrt(q) eps (eqs. qrfactorth, errorinfact)."""
    X = _noisy(20000, 61, "noisy_2p24x500")
    b = B.foa_blocked(X)
    q = b.q
    V = b.V[:, :q]
    orth = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    fact = np.linalg.norm(X[:, :q] - V @ b.beta[:q, :q]) / np.linalg.norm(X[:, :q])
    hess = np.abs(np.tril(b.H[:q, :q - 1], -2)).max() == 0.0
    tri = np.abs(np.tril(b.beta[:q, :q], -1)).max() == 0.0
    return orth <= 10 * np.sqrt(q) * EPS64 and fact <= 10 * np.sqrt(q) * EPS64 and hess and tri


def pin_householder(B):
    """beta equals Householder R with a positive diagonal; H_bar = R_{:,2:} R_{1:q-1}^{-1}."""
    X = _noisy(500, 25)
    b = B.foa_blocked(X)
    Q, R = np.linalg.qr(X)
    d = np.sign(np.diag(R))
    R = d[:, None] * R
    q = b.q
    Hc = R[:, 1:q] @ np.linalg.inv(R[:q - 1, :q - 1])
    kap = np.linalg.cond(R)
    return (np.abs(b.beta[:q, :q] - R).max() <= 100 * q * EPS64 * kap * np.abs(R).max()
            and np.abs(b.H[:q, :q - 1] - Hc).max() <= 100 * q * EPS64 * kap * np.abs(Hc).max())


def pin_exact_rank(B):
    """Exact-rank data: the block that crosses the rank falls back to the
    sequential rule, breakdown at the same snapshot, generating eigenvalues exact."""
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, b = datagen.snapshots_numpy(w)
    bb = B.foa_blocked(X)
    ev = np.linalg.eigvals(bb.H[:bb.q, :bb.q])
    lam_all = np.concatenate([lam, np.conj(lam)])
    return bb.status == ofoa.INVARIANT and bb.q == 20 and match_eigs(ev, lam_all) <= 1e-9


def pin_kappa_slope(B):
    """Projection error grows like kappa, not kappa^2 (Section 3.2.2 figure)."""
    A = np.vander(np.linspace(0, 1, 50))
    psi1 = np.random.default_rng(5).standard_normal(50)
    ks, es = [], []
    for N in range(5, 12):
        X = _krylov(A, psi1, N)
        st = B.foa_blocked(X, tol=0.0)
        m = N - 1
        V = st.V[:, :m]
        es.append(np.linalg.norm(V.T @ A @ V - st.H[:m, :m]))
        ks.append(np.linalg.cond(X[:, :m]))
    slope = np.polyfit(np.log(ks), np.log(es), 1)[0]
    return 0.6 <= slope <= 1.4


def pin_block_qr(B):
    """The block QR of an ill-conditioned block (kappa 1e10) is orthogonal to
    eps and reproduces the block (Householder-quality)."""
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((4000, 4)))
    W, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    Z = U @ np.diag([1.0, 1e-3, 1e-7, 1e-10]) @ W.T
    res = B.block_qr(Z)
    if res is None:
        return False
    Q, S = res
    return (np.linalg.norm(np.eye(4) - Q.T @ Q, 2) <= 100 * EPS64
            and np.linalg.norm(Z - Q @ S) <= 100 * EPS64 * np.linalg.norm(Z)
            and np.abs(np.tril(S, -1)).max() == 0.0 and np.all(np.diag(S) > 0))


def pin_noise_floor_f32(B):
    """FP32-rounded basis, snapshots whose new directions sit at the data's
    noise floor (about 1e-8 of their norm) at small n (5000 rows, 500
    snapshots): the basis stays orthogonal and X = V beta holds, both to
    10 sqrt(q) eps32 -- where two projections that take V as orthonormal lose
    orthogonality completely (||I - V^T V|| about 47)."""
    X = _noisy(5000, 500, "noisy_2p24x500")
    b = B.foa_blocked(X, storage="f32")
    q = b.q
    V = b.V[:, :q]
    if q != 500 or not (np.all(np.isfinite(V)) and np.all(np.isfinite(b.beta[:q, :q]))):
        return False
    orth = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    fact = np.linalg.norm(X[:, :q] - V @ b.beta[:q, :q]) / np.linalg.norm(X[:, :q])
    return orth <= 10 * np.sqrt(q) * EPS32 and fact <= 10 * np.sqrt(q) * EPS32


def pin_third_projection_rule(B):
    """The test for a third projection: never on an exactly orthonormal basis
    (R2 = 0), never when R1 = 0, and on a basis whose Gram deviation E is known
    exactly it fires precisely when ||E R1||_F / ||R1||_F * ||R2_k|| exceeds a
    tenth of the unit roundoff times ||Z_k||."""
    rng = np.random.default_rng(11)
    n, j, p = 400, 30, 4
    V, _ = np.linalg.qr(rng.standard_normal((n, j)))
    Y = rng.standard_normal((n, p))
    R1 = V.T @ Y
    Z = Y - V @ R1
    ok = not B.third_projection_needed(R1, np.zeros_like(R1), Z, 2.0 ** -24)
    ok = ok and not B.third_projection_needed(np.zeros_like(R1), np.zeros_like(R1), Z, 2.0 ** -24)
    E = 1e-6 * rng.standard_normal((j, j))
    R2 = -E @ R1
    e = np.linalg.norm(R2) / np.linalg.norm(R1)
    rem = e * np.linalg.norm(R2, axis=0)
    for scale in (0.5, 2.0):       # Z's columns just above / below the threshold
        Zs = Z / np.linalg.norm(Z, axis=0) * (rem.max() / (0.1 * 2.0 ** -24)) * scale
        ok = ok and B.third_projection_needed(R1, R2, Zs, 2.0 ** -24) == (scale < 1.0)
    return ok


PINS = [pin_matches_sequential, pin_orthogonal_factorisation, pin_householder, pin_exact_rank,
        pin_kappa_slope, pin_block_qr, pin_noise_floor_f32, pin_third_projection_rule]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_blocked_oracle_pin(pin):
    assert pin(ob)


# ---- planted mistakes --------------------------------------------------------

class _Mutant:
    """oracle.blocked with one function replaced."""

    def __init__(self, **repl):
        self.__dict__.update({k: getattr(ob, k) for k in ("PB", "UNIT", "THIRD_ETA", "block_qr", "_chol_upper",
                                                          "_right_solve_upper", "third_projection_needed",
                                                          "storage_unit", "round_new_columns")})
        self.__dict__.update(repl)
        self.block_step = lambda st, Y, unit=ob.UNIT: self.step_impl(self, st, Y, unit)
        self.foa_blocked = (lambda X, p=ob.PB, tol=None, capacity=None, storage="f64":
                            _foa_blocked(self, X, p, tol, capacity, storage))


def _foa_blocked(M, X, p, tol, capacity, storage):
    X = np.asarray(X, dtype=np.float64)
    n, N = X.shape
    cap = N if capacity is None else int(capacity)
    unit = M.storage_unit(storage)
    st = ofoa.foa_stream_init(n, cap, tol)
    ofoa.foa_stream_update(st, X[:, :1])
    M.round_new_columns(st, 0, storage)
    k = 1
    lead = (N - k) % p
    if lead and st.status == ofoa.ACTIVE:
        q0 = st.q
        ofoa.foa_stream_update(st, X[:, k:k + lead])
        M.round_new_columns(st, q0, storage)
        k += lead
    while k < N:
        q0 = st.q
        if (st.status == ofoa.ACTIVE and k + p <= N and st.q + p <= cap
                and M.block_step(st, np.ascontiguousarray(X[:, k:k + p]), unit)):
            M.round_new_columns(st, q0, storage)
            k += p
            continue
        m = min(p, N - k)
        ofoa.foa_stream_update(st, X[:, k:k + m])
        M.round_new_columns(st, q0, storage)
        k += m
    return st


def _step(M, st, Y, unit, passes=2, h_col_shift=0, drop_S=False, transpose_R=False, third=True):
    n, p = Y.shape
    j = st.q
    V = st.V[:, :j]
    yn2 = np.einsum("ij,ij->j", Y, Y)
    R1 = V.T @ Y
    Z = Y - V @ R1
    R = R1
    if passes == 2:
        R2 = V.T @ Z
        Z = Z - V @ R2
        R = R1 + R2
        if third and M.third_projection_needed(R1, R2, Z, unit):
            R3 = V.T @ Z
            Z = Z - V @ R3
            R = R + R3
    res = M.block_qr(Z)
    if res is None:
        return False
    Q, S = res
    if drop_S:
        S = np.diag(np.diag(S))
    if transpose_R:
        R = R[:, ::-1]
    xf = st.xfro2 + np.cumsum(yn2)
    if np.any(np.diag(S) <= st.tol * np.sqrt(xf)):
        return False
    st.beta[:j, j:j + p] = R
    st.beta[j:j + p, j:j + p] = S
    st.V[:, j:j + p] = Q
    for c in range(j - 1, j + p - 1):
        cc = c + h_col_shift
        st.H[:c + 2, c] = (st.beta[:c + 2, c + 1] - st.H[:c + 2, :c] @ st.beta[:c, cc]) / st.beta[c, c]
    st.xfro2 = float(xf[-1])
    st.q = j + p
    st.pushes += p
    return True


MUTANTS = {
    "single_projection": dict(passes=1),
    "h_recurrence_index": dict(h_col_shift=-1),
    "block_R_offdiagonal_dropped": dict(drop_S=True),
    "R_columns_reversed": dict(transpose_R=True),
    "no_third_projection": dict(third=False),
    # the rule itself: the remainder measured against ||R1_k|| instead of ||Z_k||;
    # the threshold on ||R2_k|| alone
    "third_rule_against_R1": dict(repl=dict(third_projection_needed=lambda R1, R2, Z, unit: bool(
        np.linalg.norm(R1) > 0 and np.any(np.linalg.norm(R2) / np.linalg.norm(R1) * np.linalg.norm(R2, axis=0)
                                          > ob.THIRD_ETA * unit * np.linalg.norm(R1, axis=0))))),
    "third_rule_without_E_estimate": dict(repl=dict(third_projection_needed=lambda R1, R2, Z, unit: bool(
        np.any(np.linalg.norm(R2, axis=0) > ob.THIRD_ETA * unit * np.linalg.norm(Z, axis=0))))),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_blocked_mutant_is_caught(name):
    kw = dict(MUTANTS[name])
    M = _Mutant(**kw.pop("repl", {}))
    M.step_impl = lambda M_, st, Y, unit: _step(M_, st, Y, unit, **kw)
    failed = []
    for pin in PINS:
        try:
            ok = pin(M)
        except Exception:
            ok = False
        if not ok:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
