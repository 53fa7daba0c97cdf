"""Pins of the one-reduction oracle (oracle/lowsync.py) against facts it does
not define: Householder QR of the snapshots (QR uniqueness), the sequential
oracle of Algorithm 1, orthogonality and factorisation bounds (eqs.
qrfactorth, errorinfact) in both storage precisions, recovery of generating
eigenvalues with the breakdown stop (Section 3.2.4), the flush and
non-finite rules, and one sweep over the basis per snapshot.  Planted
mistakes must each fail a pin by value."""

import types

import numpy as np
import pytest

import datagen
import oracle
import oracle.lowsync as LS
from pins import _random_X, match_eigs

EPS = 2.0 ** -52
EPS32 = 2.0 ** -23


def _headline_small(n=4096, N=200):
    """The noisy_2p24x500 recipe (120 pairs over 1e0..1e-7, noise 1e-8) at
    n = 4096, N = 200: kappa_2 ~ 1e8-1e9, beyond 1/eps32."""
    w = datagen.get_workload("noisy_2p24x500").with_n(n).with_N(N)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    return X


def _noisy_small(n=3000, N=60):
    w = datagen.get_workload("noisy_2p20x200").with_n(n).with_N(N)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    return X


def pin_ls_householder_qr(L, n=60, N=12, seed=3):
    """Thin QR with positive diagonal, unique for full-rank X: V and beta
    against Householder QR; H_bar = R_{:,2:N} R_{N-1}^{-1} (eq.
    betacolumnupdate)."""
    X = _random_X(n, N, seed)
    st = L.run(X, tol=0.0)
    if st.q != N:
        return False, f"q={st.q}"
    Q, R = np.linalg.qr(X)
    sgn = np.sign(np.diag(R))
    Q, R = Q * sgn, (R.T * sgn).T
    kap = np.linalg.cond(X)
    tol = 100 * N * EPS * kap
    ev = np.abs(L.basis(st) - Q).max()
    eb = np.abs(st.beta[:N, :N] - R).max() / np.abs(R).max()
    Hc = np.linalg.solve(R[:N - 1, :N - 1].T, R[:, 1:N].T).T
    eh = np.abs(st.H[:N, :N - 1] - Hc).max() / np.abs(Hc).max()
    return ev <= tol and eb <= tol and eh <= tol, f"|dV|={ev:.1e} |dbeta|={eb:.1e} |dH|={eh:.1e} tol={tol:.1e}"


def pin_ls_vs_sequential(L):
    """Same factors as the sequential oracle up to rounding: H_bar, beta and V
    within 100 q eps kappa_2 (the two differ in the order of operations)."""
    X = _noisy_small()
    a = L.run(X)
    b = oracle.foa_batch(X)
    q = b.q
    if a.q != q:
        return False, f"q {a.q} vs {q}"
    kap = oracle.kappa2(b.beta[:q, :q])
    tol = 100 * q * EPS * kap
    eH = np.linalg.norm(a.H[:q, :q - 1] - b.H[:q, :q - 1]) / np.linalg.norm(b.H[:q, :q - 1])
    eB = np.linalg.norm(a.beta[:q, :q] - b.beta[:q, :q]) / np.linalg.norm(b.beta[:q, :q])
    eV = np.abs(L.basis(a) - b.V[:, :q]).max()
    return max(eH, eB, eV) <= tol, f"kappa={kap:.1e} relH={eH:.1e} relB={eB:.1e} maxV={eV:.1e} tol={tol:.1e}"


def pin_ls_orthogonality(L):
    """||I - V^T V||_2 <= 10 q eps64 (FP64 storage) and 10 sqrt(q) eps32 (FP32
    storage) at kappa_2 ~ 1e9 (eq. qrfactorth: twice is enough)."""
    X = _headline_small()
    msgs, ok = [], True
    for storage, bound in (("f64", lambda q: 10 * q * EPS), ("f32", lambda q: 10 * np.sqrt(q) * EPS32)):
        st = L.run(X, storage=storage)
        V = L.basis(st)
        e = np.linalg.norm(np.eye(st.q) - V.T @ V, 2)
        ok = ok and st.q == X.shape[1] and e <= bound(st.q)
        msgs.append(f"{storage}: q={st.q} ||I-V^TV||={e:.1e} (bound {bound(st.q):.1e})")
    return ok, "; ".join(msgs)


def pin_ls_noise_floor_f32(L):
    """FP32 storage where new snapshots lie at the noise floor of the data and
    the stored basis is far from orthonormal at working precision (the
    noisy_2p24x500 recipe at n = 5000, N = 384: 240 signal directions, then
    residuals of ~1e-8 ||x||, against an ||I - Q^T Q|| of a few 1e-8 from the
    rounding of the stored columns): orthogonality and factorisation stay at
    10 sqrt(q) eps32 (eqs. qrfactorth, errorinfact), and beta is the
    factorisation of the snapshots.  Without the Gram correction of the
    second projection the basis loses orthogonality entirely here."""
    w = datagen.get_workload("noisy_2p24x500").with_n(5000).with_N(384)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    st = L.run(X, storage="f32")
    q = st.q
    V = L.basis(st)
    if not (np.all(np.isfinite(V)) and np.all(np.isfinite(st.beta[:q, :q]))):
        return False, f"q={q}: non-finite basis or beta"
    e = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    r = np.linalg.norm(X[:, :q] - V @ st.beta[:q, :q]) / np.linalg.norm(X[:, :q])
    b = 10 * np.sqrt(q) * EPS32
    return (q == X.shape[1] and e <= b and r <= b,
            f"q={q} ||I-V^TV||={e:.1e}, factorisation {r:.1e} (bound {b:.1e})")


def pin_ls_factorisation(L):
    """||X - V beta||_F / ||X||_F <= 10 sqrt(q) eps of the storage precision
    (eq. errorinfact's leading term) at kappa_2 ~ 1e9."""
    X = _headline_small()
    msgs, ok = [], True
    for storage, eps in (("f64", EPS), ("f32", EPS32)):
        st = L.run(X, storage=storage)
        q = st.q
        r = np.linalg.norm(X[:, :q] - L.basis(st) @ st.beta[:q, :q]) / np.linalg.norm(X[:, :q])
        ok = ok and r <= 10 * np.sqrt(q) * eps
        msgs.append(f"{storage}: {r:.1e} (bound {10 * np.sqrt(q) * eps:.1e})")
    return ok, "; ".join(msgs)


def pin_ls_shift_relation(L):
    """beta_{1:q,2:q} = H_bar_q beta_{q-1} to rounding (eq. matmulhbeta)."""
    X = _noisy_small()
    st = L.run(X)
    q = st.q
    lhs = np.linalg.norm(st.beta[:q, 1:q] - st.H[:q, :q - 1] @ st.beta[:q - 1, :q - 1])
    bound = 10 * q * EPS * np.linalg.norm(st.H[:q, :q - 1]) * np.linalg.norm(st.beta[:q - 1, :q - 1])
    return lhs <= bound, f"{lhs:.1e} <= {bound:.1e}"


def pin_ls_exact_rank(L):
    """Exact-rank data: the stream becomes invariant with q = 2M (the
    dependent snapshot is found two pushes later) and the eigenvalues of
    H_{2M} are the generating ones (Section 3.2.4)."""
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, _ = datagen.snapshots_numpy(w)
    st = L.run(X)
    M2 = 2 * w.pairs
    if st.q != M2 or st.status != "invariant":
        return False, f"q={st.q} status={st.status}"
    err = match_eigs(np.linalg.eigvals(st.H[:M2, :M2]), np.concatenate([lam, lam.conj()]))
    return err <= 1e-8, f"max |dlambda| {err:.1e}"


def pin_ls_nonfinite_and_zero(L):
    """A snapshot with a NaN is dropped and stops the stream; the snapshots
    before it are completed by the flush, bitwise as if the stream had ended
    there.  A zero first snapshot leaves q = 0."""
    X = _noisy_small(n=400, N=12)
    Xb = X.copy()
    Xb[5, 7] = np.nan
    a = L.run(Xb)
    b = L.run(X[:, :7], capacity=12)
    same = (a.status == "nonfinite" and a.q == b.q == 7 and np.array_equal(a.beta, b.beta)
            and np.array_equal(a.H, b.H) and np.array_equal(L.basis(a), L.basis(b)))
    z = L.run(np.zeros((5, 3)))
    return same and z.q == 0 and z.status == "zero_first", f"nonfinite q={a.q} status={a.status}; zero q={z.q}"


def pin_ls_flush_midway(L):
    """A flush in the middle of the stream finishes the pending columns; the
    stream goes on from there and the result is the same factorisation to
    rounding."""
    X = _noisy_small()
    st = L.init(X.shape[0], X.shape[1])
    for j in range(X.shape[1]):
        L.push(st, X[:, j])
        if j in (0, 1, 9, 30):
            L.flush(st)
    L.flush(st)
    ref = L.run(X)
    q = ref.q
    kap = oracle.kappa2(ref.beta[:q, :q])
    e = np.linalg.norm(st.H[:q, :q - 1] - ref.H[:q, :q - 1]) / np.linalg.norm(ref.H[:q, :q - 1])
    return st.q == q and e <= 100 * q * EPS * kap, f"q={st.q} relH={e:.1e}"


class _CountingArray(np.ndarray):
    """ndarray that counts the elements read from it by matrix products and
    column slices taken for arithmetic."""

    reads = [0]

    def __array_ufunc__(self, ufunc, method, *inputs, **kw):
        args = []
        for x in inputs:
            if isinstance(x, _CountingArray):
                _CountingArray.reads[0] += x.size
                x = np.asarray(x)
            args.append(x)
        return getattr(ufunc, method)(*args, **kw)


def pin_ls_one_sweep(L):
    """The basis storage is read once per push: at most n (q + 3) elements
    (the final columns once, the pending columns), where the literal schedule
    of Algorithm 1 reads the basis five times."""
    X = _noisy_small(n=500, N=40)
    n = X.shape[0]
    st = L.init(n, 40)
    worst = 0.0
    for j in range(40):
        st.V = st.V.view(_CountingArray)
        _CountingArray.reads[0] = 0
        L.push(st, X[:, j])
        st.V = np.asarray(st.V)
        q = st.q
        worst = max(worst, _CountingArray.reads[0] / (n * (q + 3)))
    return worst <= 1.0, f"max basis reads per push / (n (q + 3)) = {worst:.2f}"


LS_PINS = [pin_ls_householder_qr, pin_ls_vs_sequential, pin_ls_orthogonality, pin_ls_factorisation,
           pin_ls_noise_floor_f32, pin_ls_shift_relation, pin_ls_exact_rank, pin_ls_nonfinite_and_zero,
           pin_ls_flush_midway, pin_ls_one_sweep]


def run_all(L):
    out = {}
    for f in LS_PINS:
        try:
            ok, d = f(L)
            out[f.__name__] = (bool(ok), d, False)
        except Exception as e:
            out[f.__name__] = (False, f"raised {type(e).__name__}: {e}", True)
    return out


@pytest.mark.parametrize("pin", LS_PINS, ids=lambda f: f.__name__)
def test_lowsync_pin(pin):
    ok, detail = pin(LS)
    assert ok, detail


# ---- planted mistakes ---------------------------------------------------------

def _mutant(edit):
    """A copy of the oracle module with one source edit."""
    import inspect

    src = inspect.getsource(LS)
    assert edit[0] in src, edit[0]
    m = types.ModuleType("lowsync_mutant")
    m.__dict__["__name__"] = "oracle.lowsync_mutant"
    m.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(edit[0], edit[1], 1), "lowsync_mutant", "exec"), m.__dict__)
    return m


# Not listed (equivalent within the method's O(eps kappa) error): leaving out
# the second projection's coefficients from beta, keeping the estimated norm
# on beta's diagonal, and leaving out the rescale of the first-pass
# coefficient to the exact norm.  The second projection measures and removes
# whatever the first left, so each of these changes beta only by the
# rounding-size second-pass coefficients (the counterpart of the excluded
# mutant of the sequential oracle).
LS_MUTANTS = {
    "first_projection_skips_last_column": ("u = u - ut * (r_t / rho_hat)", "u = u"),
    "second_projection_sign": ("ut = _store(st, st.V[:, q] - Q @ st.w_hat)",
                               "ut = _store(st, st.V[:, q] + Q @ st.w_hat)"),
    "gamma_without_w_z_term": ("(st.gamma - float(st.w_hat @ st.z)) / rho_hat", "st.gamma / rho_hat"),
    "second_projection_ignores_gram": ("w_hat = wfull - st.E[:c, :c] @ wfull", "w_hat = wfull"),
    "gram_column_unscaled": ("st.E[:c, c] = st.E[c, :c] = gq / rho", "st.E[:c, c] = st.E[c, :c] = gq"),
    "gram_column_sign": ("st.E[:c, c] = st.E[c, :c] = gq / rho", "st.E[:c, c] = st.E[c, :c] = -gq / rho"),
    "hbar_divides_by_new_diagonal": ("st.H[:c + 1, c - 1] = col / st.beta[c - 1, c - 1]",
                                     "st.H[:c + 1, c - 1] = col / st.beta[c, c]"),
    "w_last_entry_unscaled": ("wfull = np.append(wfull, wu * st.sigma[k])", "wfull = np.append(wfull, wu)"),
    "z_last_entry_unscaled": ("zfull = np.append(zfull, zu * st.sigma[st.q - 1])", "zfull = np.append(zfull, zu)"),
    "final_columns_unnormalised": ("Q = st.V[:, :q] * st.sigma[:q]", "Q = st.V[:, :q]"),
}


@pytest.mark.parametrize("name", sorted(LS_MUTANTS))
def test_lowsync_mutant_is_caught(name):
    res = run_all(_mutant(LS_MUTANTS[name]))
    failed = [k for k, (ok, _, raised) in res.items() if not ok and not raised]
    assert failed, f"mutant {name} passed every pin"


def test_lowsync_unmutated_passes():
    res = run_all(_mutant(("ACTIVE = \"active\"", "ACTIVE = \"active\"")))
    bad = {k: d for k, (ok, d, _) in res.items() if not ok}
    assert not bad, bad
