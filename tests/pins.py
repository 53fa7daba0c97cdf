"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself.

Each ``pin_*`` returns (ok: bool, detail: str).  ``run_all`` runs every pin;
tests/test_oracle_pins.py requires all of them to pass, and
tests/test_oracle_mutants.py plants plausible mistakes in the oracle and
requires at least one pin to fail for each.

References used here are independent of the oracle's own arithmetic:
Householder QR (numpy.linalg.qr) for the QR-uniqueness pin, the generating
eigenvalues of the synthetic data, an explicitly known map A, the
hand-derived example in tests/golden/diag2_worked.json, and closed forms.
"""

import json
import math
import os

import numpy as np
from scipy.optimize import linear_sum_assignment

import datagen

EPS = 2.0 ** -52
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def match_eigs(a, b):
    """Max |a_i - b_pi(i)| over a min-cost matching (unordered sets)."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return float(C[r, c].max()) if len(r) else 0.0


def _krylov(A, psi1, N):
    X = np.empty((A.shape[0], N))
    X[:, 0] = psi1
    for j in range(1, N):
        X[:, j] = A @ X[:, j - 1]
    return X


def _known_A(n=40, seed=11):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / math.sqrt(n)
    A /= 1.05 * max(abs(np.linalg.eigvals(A)))
    psi1 = rng.standard_normal(n)
    return A, psi1


# --------------------------------------------------------------------------

def pin_golden_diag2(O):
    g = json.load(open(os.path.join(GOLDEN, "diag2_worked.json")))
    X = np.array(g["X"])
    st = O.foa_batch(X)
    tol = g["tol"]
    q = st.q
    ok = q == g["q"] and st.status == g["status"]
    Vg, Hg, Bg = np.array(g["V"]), np.array(g["H"]), np.array(g["beta"])
    e = max(np.abs(st.V[:, :q] - Vg).max(), np.abs(st.H[:3, :2] - Hg).max(),
            np.abs(st.beta[:2, :3] - Bg).max())
    res = O.dmd_untruncated(st)
    el = match_eigs(res["lam"], g["eigenvalues"])
    ec = np.abs(np.sort(np.abs(res["coef"])) - np.sort(g["abs_coef"])).max()
    ei = np.abs(res["indicators"]).max()
    ok = ok and e <= tol and el <= tol and ec <= 10 * tol and ei <= tol
    return ok, f"q={q} status={st.status} max|d|={e:.2e} eig={el:.2e} coef={ec:.2e}"


def pin_exact_rank_recovery(O):
    """Exact-rank data: breakdown at snapshot 2M+1 and the Ritz values of the
    square H_{2M} are the generating eigenvalues (Section 3.2.4)."""
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, _ = datagen.snapshots_numpy(w)
    st = O.foa_batch(X)
    M2 = 2 * w.pairs
    if st.q != M2 or st.status != "invariant":
        return False, f"q={st.q} status={st.status}, expected {M2} invariant"
    res = O.dmd_untruncated(st)
    err = match_eigs(res["lam"], np.concatenate([lam, lam.conj()]))
    return err <= 1e-8, f"max matched |dlambda| = {err:.2e}"


def _random_X(n, N, seed, cond_decades=2.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, N)))
    Wm, _ = np.linalg.qr(rng.standard_normal((N, N)))
    s = np.logspace(0, -cond_decades, N)
    return (U * s) @ Wm.T


def pin_householder_qr(O, n=60, N=12, seed=3):
    """X_1^N = V beta is the thin QR factorisation with positive diagonal
    (Section 3.1, factorisation view), unique for full-rank X: compare with
    Householder QR; then H_bar = R_{:,2:N} R_{N-1}^{-1} (eq. betacolumnupdate)."""
    X = _random_X(n, N, seed)
    st = O.foa_batch(X, tol=0.0)
    if st.q != N:
        return False, f"q={st.q}"
    Q, R = np.linalg.qr(X)
    sgn = np.sign(np.diag(R))
    Q, R = Q * sgn, (R.T * sgn).T
    kap = np.linalg.cond(X)
    tolv = 100 * N * EPS * kap
    ev = np.abs(st.V[:, :N] - Q).max()
    eb = np.abs(st.beta[:N, :N] - R).max() / np.abs(R).max()
    Hc = np.linalg.solve(R[:N - 1, :N - 1].T, R[:, 1:N].T).T
    eh = np.abs(st.H[:N, :N - 1] - Hc).max() / np.abs(Hc).max()
    ok = ev <= tolv and eb <= tolv and eh <= tolv
    return ok, f"kappa={kap:.1e} |dV|={ev:.1e} |dbeta|={eb:.1e} |dH|={eh:.1e} tol={tolv:.1e}"


def _noisy_small(n=3000, N=60):
    w = datagen.get_workload("noisy_2p20x200").with_n(n).with_N(N)
    X, lam, b = datagen.snapshots_numpy(w, dtype="float64")
    return X


def pin_orthogonality(O):
    """||I - V^T V||_2 <= c eps (eq. qrfactorth) on ill-conditioned data."""
    X = _noisy_small()
    st = O.foa_batch(X)
    V = st.V[:, :st.q]
    e = np.linalg.norm(np.eye(st.q) - V.T @ V, 2)
    k = O.kappa2(st.beta[:st.q, :st.q])
    return e <= 10 * st.q * EPS, f"q={st.q} kappa={k:.1e} ||I-V^TV||={e:.2e}"


def pin_factorisation(O):
    """||X_1^q - V beta||_F bounded as in eq. errorinfact (c_1 = 10 N)."""
    X = _noisy_small()
    st = O.foa_batch(X)
    q = st.q
    n = X.shape[0]
    V, B, Hb = st.V[:, :q], st.beta[:q, :q], st.H[:q + 1, :q]
    r = np.linalg.norm(X[:, :q] - V @ B)
    nx2 = np.linalg.norm(X[:, :q], 2)
    g = lambda k: k * EPS / (1 - k * EPS)
    c1 = 10 * q
    bound = (g(3 * n + 4) * np.linalg.norm(X[:, :q]) + (g(2) + c1 * EPS) * q * np.linalg.norm(Hb) * nx2
             + g(q + 1) * q * np.linalg.norm(Hb) * nx2)
    return r <= bound, f"residual={r:.2e} bound={bound:.2e} rel={r / np.linalg.norm(X[:, :q]):.1e}"


def pin_shift_relation(O):
    """||beta_{1:q,2:q} - H_bar_q beta_{q-1}||_F <= gamma_{q-1} ||H_bar||_F ||beta||_F
    (eq. matmulhbeta)."""
    X = _noisy_small()
    st = O.foa_batch(X)
    q = st.q
    lhs = np.linalg.norm(st.beta[:q, 1:q] - st.H[:q, :q - 1] @ st.beta[:q - 1, :q - 1])
    g = (q - 1) * EPS / (1 - (q - 1) * EPS)
    bound = g * np.linalg.norm(st.H[:q, :q - 1]) * np.linalg.norm(st.beta[:q - 1, :q - 1])
    return lhs <= bound, f"lhs={lhs:.2e} bound={bound:.2e}"


def pin_known_A(O, N=10):
    """Known A: ||V^T A V - H_{N-1}||_F <= C eps kappa_2(X) (eq. foabaseddmdberr)
    and agreement with Algorithm 2 (eq. avarnoldi)."""
    A, psi1 = _known_A()
    X = _krylov(A, psi1, N)
    st = O.foa_batch(X, tol=0.0)
    m = N - 1
    V = st.V[:, :m]
    kap = np.linalg.cond(X[:, :m])
    e1 = np.linalg.norm(V.T @ A @ V - st.H[:m, :m])
    V2, H2 = O.arnoldi_known_A(A, psi1, N)
    e2 = np.linalg.norm(st.H[:N, :m] - H2)
    C = 100.0
    ok = e1 <= C * EPS * kap and e2 <= C * EPS * kap
    return ok, f"kappa={kap:.1e} ||V^TAV-H||={e1:.2e} ||H-H_alg2||={e2:.2e} bound={C * EPS * kap:.1e}"


def pin_indicator_residual(O, N=12):
    """|h_{N,N-1}| |e_{N-1}^T z_i| = ||A V z_i - lambda_i V z_i||_2 for unit z_i
    (eq. errordmdvec), up to C eps ||X|| ||y_i|| (Section 3.2.3)."""
    A, psi1 = _known_A(seed=12)
    X = _krylov(A, psi1, N)
    st = O.foa_batch(X, tol=0.0)
    res = O.dmd_untruncated(st)
    m = res["m"]
    V = st.V[:, :m]
    worst = 0.0
    for i in range(m):
        phi = V @ res["Z"][:, i]
        true = np.linalg.norm(A @ phi - res["lam"][i] * phi)
        worst = max(worst, abs(true - res["indicators"][i]) / max(true, 1e-12))
    kap = np.linalg.cond(X[:, :m])
    return worst <= 1e-6, f"kappa={kap:.1e} max rel |indicator - residual| = {worst:.2e}"


def pin_reconstruction(O, N=12):
    """psi_k = sum_j lambda_j^(k-1) c_j phi_j for k <= N-1 and the last-snapshot
    error |h_{N,N-1}| |sum_j c_j lambda_j^(N-2) e_{N-1}^T z_j| (Section 3.2.4)."""
    A, psi1 = _known_A(seed=13)
    X = _krylov(A, psi1, N)
    st = O.foa_batch(X, tol=0.0)
    res = O.dmd_untruncated(st)
    m = res["m"]
    Phi = st.V[:, :m] @ res["Z"]
    c, lam = res["coef"], res["lam"]
    worst = 0.0
    for k in range(1, N):
        rec = (Phi @ (c * lam ** (k - 1))).real
        worst = max(worst, np.linalg.norm(rec - X[:, k - 1]) / np.linalg.norm(X[:, k - 1]))
    recN = (Phi @ (c * lam ** (N - 1))).real
    errN = np.linalg.norm(recN - X[:, N - 1])
    pred = abs(st.H[m, m - 1]) * abs(np.sum(c * lam ** (N - 2) * res["Z"][m - 1, :]))
    # A psi with psi = psi_{N-1}: the error of sum lambda_j c_j lambda_j^(N-2) phi_j
    eN = abs(errN - pred) / max(errN, 1e-300)
    ok = worst <= 1e-10 and eN <= 1e-6
    return ok, f"max rel recon err (k<N)={worst:.2e} last-snapshot err={errN:.3e} predicted={pred:.3e}"


def pin_truncation_rank(O):
    """Exact-rank data without the breakdown stop: the numerical-rank rule
    (Section 4.1) picks r = 2M and the truncated Ritz values of Algorithm 1 are
    the generating eigenvalues."""
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, _ = datagen.snapshots_numpy(w)
    st = O.foa_batch(X[:, :40], tol=0.0)
    m = O.projected_size(st)
    s = np.linalg.svd(st.beta[:m, :m], compute_uv=False)
    r = O.truncation_rank(s, st.q, "f64")
    if r != 2 * w.pairs:
        return False, f"rank rule gave r={r}, expected {2 * w.pairs}"
    res = O.dmd_truncated(st, r)
    err = match_eigs(res["lam"], np.concatenate([lam, lam.conj()]))
    return err <= 1e-8, f"r={r} max matched |dlambda|={err:.2e}"


def _known_A_truncated(N=14, seed=21):
    """Krylov data of a known map whose snapshot matrix has a wide spread of
    singular values, for the truncated pins (r < m)."""
    A, psi1 = _known_A(n=40, seed=seed)
    X = _krylov(A, psi1, N)
    return A, X


def pin_truncated_indicator_residual(O, N=14, r=9):
    """Truncated indicator = ||A phi - lambda phi||_2 for phi = V_{1:m} U_r z,
    r < m, on Krylov data of a known A (Section 3.2.3, the truncated form of
    the residual identity; the paper's indicator is exact in exact arithmetic)."""
    A, X = _known_A_truncated(N)
    st = O.foa_batch(X, tol=0.0)
    res = O.dmd_truncated(st, r)
    m = res["m"]
    V = st.V[:, :m]
    worst, smallest = 0.0, np.inf
    for i in range(r):
        phi = V @ res["B"][:, i]
        true = np.linalg.norm(A @ phi - res["lam"][i] * phi)
        smallest = min(smallest, true)
        worst = max(worst, abs(true - res["indicators"][i]) / true)
    ok = worst <= 1e-6 and smallest > 1e-8
    return ok, f"m={m} r={r} max rel |indicator - residual| = {worst:.2e} (smallest residual {smallest:.1e})"


def pin_truncated_coefficients_lstsq(O, N=14, r=9):
    """Truncated coefficients = the least-squares minimiser of
    ||psi_1 - [V U_r][z] c||_2 (eq. exreconwrt), computed here by lstsq on the
    explicit complex modes."""
    A, X = _known_A_truncated(N)
    st = O.foa_batch(X, tol=0.0)
    res = O.dmd_truncated(st, r)
    m = res["m"]
    Phi = st.V[:, :m] @ res["B"]
    c_ls = np.linalg.lstsq(Phi, X[:, 0].astype(np.complex128), rcond=None)[0]
    e = np.abs(res["coef"] - c_ls).max() / np.abs(c_ls).max()
    return e <= 1e-9, f"r={r} max rel |c - c_lstsq| = {e:.2e}"


def pin_truncation_rank_rule(O):
    """The rank rule on hand-computed thresholds: N times the spacing at
    sigma_1 of the storage type.  sigma_1 = 3 lies in [2, 4), so the spacing
    is 2^-22 in FP32 and 2^-51 in FP64; with N = 10 the thresholds are
    10 * 2^-22 = 2.384e-6 and 10 * 2^-51 = 4.441e-15."""
    sig = np.array([3.0, 1e-2, 2.5e-6, 2.3e-6, 1e-9, 4.5e-15, 4.4e-15])
    r32 = O.truncation_rank(sig, 10, "f32")
    r64 = O.truncation_rank(sig, 10, "f64")
    ok = r32 == 3 and r64 == 6 and O.truncation_rank(sig[:0], 10, "f32") == 0
    return ok, f"r(f32)={r32} (expect 3), r(f64)={r64} (expect 6)"


def pin_packed_reconstruction(O, N=12):
    """Snapshots 1..N-1 rebuilt from the packed real mode columns (one column
    per real eigenvalue, (Re, Im) for each conjugate pair's Im > 0 member) and
    the coefficients: psi_k = sum_real c lambda^(k-1) phi + sum_pairs
    2 Re(c lambda^(k-1) (phi_re + i phi_im)) (Section 3.2.4, exact
    reconstruction for k <= N-1); entries in decreasing |c|."""
    A, psi1 = _known_A(seed=14)
    X = _krylov(A, psi1, N)
    st = O.foa_batch(X, tol=0.0)
    res = O.dmd_untruncated(st)
    Phi, lams, kinds = O.packed_modes(res, st.V)
    cs = O.packed_coefficients(res)
    if not (len(lams) == len(kinds) == len(cs) and Phi.shape[1] == int(np.sum(np.where(kinds == 1, 2, 1)))):
        return False, "entry counts disagree"
    if np.any(np.diff(np.abs(cs)) > 1e-12 * np.abs(cs).max()):
        return False, "entries not in decreasing |c|"
    worst = 0.0
    for k in range(1, N):
        rec = np.zeros(X.shape[0])
        col = 0
        for lam, kind, c in zip(lams, kinds, cs):
            t = c * lam ** (k - 1)
            if kind == 0:
                rec += (t * Phi[:, col]).real
                col += 1
            else:
                rec += 2.0 * (t * (Phi[:, col] + 1j * Phi[:, col + 1])).real
                col += 2
        worst = max(worst, np.linalg.norm(rec - X[:, k - 1]) / np.linalg.norm(X[:, k - 1]))
    return worst <= 1e-9, f"{len(lams)} entries, max rel reconstruction error {worst:.2e}"


def pin_stream_equals_batch(O):
    """Streaming (Algorithm 4, any p) equals batch (Algorithm 1) bit for bit
    (Section 3.1)."""
    X = _noisy_small(n=500, N=30)
    ref = O.foa_batch(X)
    for p in (1, 4, 30):
        st = O.foa_stream_init(X.shape[0], X.shape[1])
        for c0 in range(0, X.shape[1], p):
            O.foa_stream_update(st, X[:, c0:c0 + p])
        same = (st.q == ref.q and np.array_equal(st.V, ref.V) and np.array_equal(st.H, ref.H)
                and np.array_equal(st.beta, ref.beta))
        if not same:
            return False, f"p={p} differs from batch"
    return True, "p in (1, 4, 30) bitwise equal"


def pin_vandermonde_slope(O):
    """Error in the computed projection grows like kappa (not kappa^2) for
    A = vander(linspace(0, 1, 50)) (Section 3.2.2 figure)."""
    A = np.vander(np.linspace(0, 1, 50))
    psi1 = np.random.default_rng(5).standard_normal(50)
    ks, es = [], []
    for N in range(5, 12):
        X = _krylov(A, psi1, N)
        st = O.foa_batch(X, tol=0.0)
        m = N - 1
        V = st.V[:, :m]
        es.append(np.linalg.norm(V.T @ A @ V - st.H[:m, :m]))
        ks.append(np.linalg.cond(X[:, :m]))
    slope = np.polyfit(np.log(ks), np.log(es), 1)[0]
    return 0.8 <= slope <= 1.2, f"log-log slope {slope:.2f}"


class _FlopArray(np.ndarray):
    """ndarray that counts the arithmetic of the operations applied to it:
    a matrix-vector or inner product with contracted length k costs 2k - 1
    per output entry, an elementwise add/subtract/multiply/divide/sqrt one
    per output entry."""

    counter = [0]
    _ARITH = (np.add, np.subtract, np.multiply, np.divide, np.true_divide, np.sqrt, np.negative)

    def __array_ufunc__(self, ufunc, method, *inputs, **kw):
        args = [np.asarray(x) if isinstance(x, _FlopArray) else x for x in inputs]
        out = getattr(ufunc, method)(*args, **kw)
        if method == "__call__":
            if ufunc is np.matmul:
                k = np.shape(args[0])[-1]
                _FlopArray.counter[0] += int(np.size(out)) * (2 * k - 1)
            elif ufunc in _FlopArray._ARITH:
                _FlopArray.counter[0] += int(np.size(out))
        return out.view(_FlopArray) if isinstance(out, np.ndarray) else out


def pin_cost_model(O):
    """Arithmetic of one iteration's length-n work (forming w through the
    normalisation), counted on the operations the oracle actually performs:
    the paper's per-stage cost (Appendix A.1: 2nj + n for forming w, 8nj + j
    for the CGS2 sweeps, 3n for the normalisation) plus 2n for ||psi||^2 of
    the breakdown reading, up to the O(j) terms whose convention the paper
    leaves open."""
    X = _noisy_small(n=300, N=12)
    ok, msgs = True, []
    for j in (3, 7, 11):
        st = O.foa_batch(X[:, :j])
        st.V = st.V.view(_FlopArray)
        psi = np.ascontiguousarray(X[:, j]).view(_FlopArray)
        cap = X.shape[1]
        for name in ("V", "H", "beta"):
            a = getattr(st, name)
            big = np.zeros((a.shape[0], cap)) if name == "V" else np.zeros((cap, cap))
            big[:a.shape[0], :a.shape[1]] = a
            setattr(st, name, big.view(_FlopArray) if name == "V" else big)
        _FlopArray.counter[0] = 0
        O.foa._iteration(st, psi, j)
        n = X.shape[0]
        expect = 10 * n * j + 4 * n + 2 * n
        got = _FlopArray.counter[0]
        ok = ok and abs(got - expect) <= 4 * j + 4
        msgs.append(f"j={j}: {got} vs {expect}")
    return ok, "; ".join(msgs)


def pin_state_rules(O):
    """Non-finite snapshot: nothing of it is kept; zero first snapshot: q = 0."""
    X = _noisy_small(n=200, N=10)
    Xb = X.copy()
    Xb[17, 6] = np.nan
    a = O.foa_batch(Xb)
    b = O.foa_batch(X[:, :6], capacity=10)
    ok = (a.status == "nonfinite" and a.q == 6 and np.array_equal(a.H, b.H)
          and np.array_equal(a.beta, b.beta) and np.array_equal(a.V, b.V))
    z = O.foa_batch(np.zeros((5, 3)))
    ok = ok and z.q == 0 and z.status == "zero_first"
    return ok, f"nonfinite q={a.q} status={a.status}; zero-first q={z.q} status={z.status}"


ALL = [
    pin_golden_diag2,
    pin_exact_rank_recovery,
    pin_householder_qr,
    pin_orthogonality,
    pin_factorisation,
    pin_shift_relation,
    pin_known_A,
    pin_indicator_residual,
    pin_reconstruction,
    pin_truncation_rank,
    pin_truncated_indicator_residual,
    pin_truncated_coefficients_lstsq,
    pin_truncation_rank_rule,
    pin_packed_reconstruction,
    pin_stream_equals_batch,
    pin_vandermonde_slope,
    pin_cost_model,
    pin_state_rules,
]


def run_all(O):
    """{pin name: (ok, detail, raised)}; raised is True when the pin did not
    get to compare values because the oracle raised."""
    out = {}
    for f in ALL:
        try:
            ok, detail = f(O)
            out[f.__name__] = (bool(ok), detail, False)
        except Exception as e:  # a broken oracle may raise instead of mismatching
            out[f.__name__] = (False, f"raised {type(e).__name__}: {e}", True)
    return out
