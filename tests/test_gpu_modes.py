"""Eigenvalues, modes, indicators, coefficients and truncation through the C
ABI, against the CPU oracle."""

import numpy as np
import pytest

import datagen
import oracle
from gpu_helpers import EPS32, announce, run_gpu
from oracle.dmd import packed_modes
from pins import _known_A, _krylov, match_eigs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    announce(request.node.nodeid)
    yield


def _modes(g, n, phi_dtype="f64"):
    import torch

    from paper_1805_05821_amd import foa as F

    s = g["stream"]
    m = g["m"]
    cols = m
    tdt = torch.float64 if phi_dtype == "f64" else torch.float32
    phi = torch.zeros((cols, n), dtype=tdt, device="cuda")
    lam, kind, amp, err = F.foa_modes(s.ctx, m, phi, n, cols, F.FOA_F64 if phi_dtype == "f64" else F.FOA_F32)
    ncols = int(np.sum(np.where(kind == 1, 2, 1)))
    Phi = phi[:ncols].double().cpu().numpy().T
    return lam, kind, amp, err, Phi


def _oracle_entries(res):
    """Oracle entries in mode order: (lam, |c|, indicator) for Im >= 0."""
    out = []
    for i in res["order"]:
        lam = res["lam"][i]
        if lam.imag < 0:
            continue
        out.append((lam, abs(res["coef"][i]), res["indicators"][i]))
    return out


def _match_columns(Phi, Phi_ref, kind):
    """Max column error, allowing the sign ambiguity of a real eigenvector."""
    worst = 0.0
    for c in range(Phi.shape[1]):
        a, b = Phi[:, c], Phi_ref[:, c]
        e = min(np.abs(a - b).max(), np.abs(a + b).max()) / max(np.abs(b).max(), 1e-300)
        worst = max(worst, e)
    return worst


def test_exact_rank_modes_and_indicators():
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam_true, _ = datagen.snapshots_numpy(w)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f64")
    lam, kind, amp, err, Phi = _modes(g, X.shape[0])
    assert len(lam) == 10 and np.all(kind == 1)
    assert match_eigs(lam, lam_true) <= 1e-9
    assert np.all(err == 0.0)  # invariant basis: exact Ritz pairs
    res = oracle.dmd_untruncated(st)
    ref = _oracle_entries(res)
    assert match_eigs(lam, [r[0] for r in ref]) <= 1e-9
    assert np.allclose(amp, [r[1] for r in ref], rtol=1e-7)
    Phi_ref, lam_ref, kind_ref = packed_modes(res, st.V)
    assert np.array_equal(kind, kind_ref)
    e = _match_columns(Phi, Phi_ref, kind)
    announce(f"mode column rel err {e:.2e}")
    assert e <= 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_known_A_indicators_are_residuals(prec):
    """|h_{m+1,m}| |e_m^T z| equals ||A phi - lambda phi|| for unit modes
    (Section 3.2.3), evaluated from the GPU's own modes."""
    A, psi1 = _known_A(n=300, seed=21)
    X = _krylov(A, psi1, 14)
    g = run_gpu(X, prec, tol=0.0)
    lam, kind, amp, err, Phi = _modes(g, X.shape[0])
    col = 0
    worst = 0.0
    for e_i, (l, k) in enumerate(zip(lam, kind)):
        phi = Phi[:, col] + (1j * Phi[:, col + 1] if k == 1 else 0.0)
        col += 2 if k == 1 else 1
        nrm = np.linalg.norm(phi)
        true = np.linalg.norm(A @ phi - l * phi) / nrm
        worst = max(worst, abs(true - err[e_i]) / max(true, 1e-12))
    announce(f"{prec}: max rel |indicator - residual| = {worst:.2e}")
    assert worst <= (1e-6 if prec == "f64" else 1e-2)


def test_untruncated_matches_oracle():
    A, psi1 = _known_A(n=500, seed=22)
    X = _krylov(A, psi1, 16)
    st = oracle.foa_batch(X, tol=0.0)
    g = run_gpu(X, "f64", tol=0.0)
    lam, kind, amp, err, Phi = _modes(g, X.shape[0])
    res = oracle.dmd_untruncated(st)
    ref = _oracle_entries(res)
    assert len(lam) == len(ref)
    assert match_eigs(lam, [r[0] for r in ref]) <= 1e-9
    assert np.allclose(amp, [r[1] for r in ref], rtol=1e-6)
    assert np.allclose(err, [r[2] for r in ref], rtol=1e-5, atol=1e-12)
    Phi_ref, _, kind_ref = packed_modes(res, st.V)
    assert np.array_equal(kind, kind_ref)
    assert _match_columns(Phi, Phi_ref, kind) <= 1e-7


def test_truncation_recovers_rank_and_eigenvalues():
    """Exact-rank data without the breakdown stop: the numerical-rank rule
    picks r = 2M and the truncated eigenvalues are the generating ones."""
    from paper_1805_05821_amd import foa as F

    w = datagen.get_workload("exact_rank_4096x64")
    X, lam_true, _ = datagen.snapshots_numpy(w)
    X = np.asfortranarray(X[:, :40])
    st = oracle.foa_batch(X, tol=0.0)
    g = run_gpu(X, "f64", tol=0.0)
    assert g["q"] == 40
    r, sig = F.foa_truncate(g["stream"].ctx)
    announce(f"truncation rank {r}")
    assert r == 20
    m = oracle.projected_size(st)
    s_ref = np.linalg.svd(st.beta[:m, :m], compute_uv=False)
    assert np.abs(sig[:20] - s_ref[:20]).max() <= 1e-10 * s_ref[0]
    lam, kind, amp, err, Phi = _modes(g, X.shape[0])
    assert len(lam) == 10
    assert match_eigs(lam, lam_true) <= 1e-8
    res = oracle.dmd_truncated(st, 20)
    ref = _oracle_entries(res)
    assert np.allclose(amp, [x[1] for x in ref], rtol=1e-6)
    assert np.allclose(err, [x[2] for x in ref], rtol=1e-3, atol=1e-9)
    lam2, err2 = F.foa_indicators(g["stream"].ctx, 64)
    assert np.array_equal(lam2, lam) and np.array_equal(err2, err)
    # clearing the truncation returns to the full projected matrix
    F.foa_truncate(g["stream"].ctx, r_force=-1)
    lam3, _ = F.foa_indicators(g["stream"].ctx, 64)
    assert len(lam3) > 10


def test_f32_modes_close_to_f64():
    A, psi1 = _known_A(n=2000, seed=23)
    X = _krylov(A, psi1, 12)
    a = run_gpu(X, "f64", tol=0.0)
    b = run_gpu(X, "f32", tol=0.0)
    la, ka, _, _, Pa = _modes(a, X.shape[0])
    lb, kb, _, _, Pb = _modes(b, X.shape[0], phi_dtype="f32")
    assert np.array_equal(ka, kb)
    assert match_eigs(la, lb) <= 1e-4
    assert _match_columns(Pb, Pa, ka) <= 1e-3


@pytest.mark.parametrize("n,N,r_force", [(100037, 101, -1), (100037, 101, 37), (5000, 300, -1)])
def test_mfma_modes_match_fp64_accumulation(n, N, r_force):
    """FP32 basis: the FP32-output reconstruction (FP32 MFMA, FP32 accumulation)
    against the FP64-output one (FP64 accumulation) from the same stored basis
    and coefficients.  Shapes span several 128-row tiles with a ragged tail,
    several 32-deep k chunks with a ragged last one, ragged mode blocks and,
    for N = 300, a second 256-mode tile.  With an orthonormal basis a column's
    2-norm error is at most gamma_{k+1} sqrt(k) times its norm (FP32 rounding
    of the coefficients and k FP32 multiply-adds); a wrong fragment layout
    gives O(1) errors."""
    import torch

    from paper_1805_05821_amd import foa as F

    rng = np.random.default_rng(n + N)
    X = rng.standard_normal((n, N))
    g = run_gpu(X, "f32", tol=0.0)
    s = g["stream"]
    assert g["q"] == N
    if r_force > 0:
        r, _ = s.truncate(r_force=r_force)
        assert r == r_force
    outs = {}
    for dt, code, tdt in (("f64", F.FOA_F64, torch.float64), ("f32", F.FOA_F32, torch.float32)):
        phi = torch.full((N, n), float("nan"), dtype=tdt, device="cuda")
        lam, kind, amp, err = F.foa_modes(s.ctx, N, phi, n, N, code)
        ncols = int(np.sum(np.where(kind == 1, 2, 1)))
        outs[dt] = (lam, kind, ncols, phi[:ncols].double().cpu().numpy())
        # columns past the packed ones are left untouched
        assert torch.isnan(phi[ncols:]).all()
    l64, k64, c64, P64 = outs["f64"]
    l32, k32, c32, P32 = outs["f32"]
    assert np.array_equal(k64, k32) and c64 == c32 and np.array_equal(l64, l32)
    k = g["m"]
    tol = (k + 2) * np.sqrt(k) * 2.0 ** -24
    err = np.linalg.norm(P32 - P64, axis=1) / np.linalg.norm(P64, axis=1)
    announce(f"n={n} N={N} r_force={r_force}: {c64} columns, k={k}, max column rel err {err.max():.2e} "
             f"(bound {tol:.1e})")
    assert np.isfinite(P32).all()
    assert err.max() <= tol
    s.close()


@pytest.mark.parametrize("n,N,r_force", [(100037, 101, -1), (100037, 101, 37), (5000, 300, -1),
                                         (70001, 260, 97)])
def test_mfma_modes_match_oracle(n, N, r_force):
    """The FP32 MFMA mode reconstruction (FP32 basis, FP32 mode matrix) against
    the oracle's modes V_{1:m} U_r z_i (Algorithm 1, both branches), column by
    column after matching eigenvalues, up to the unit factor an eigenvector
    is defined with.  Ragged rows (128-row tiles), ragged 32-deep k chunks,
    ragged 32-mode blocks and, for N = 260/300, a second 256-mode tile.
    Gaussian snapshots: kappa_2 ~ 3, so the bound is tight: 10 eps32
    (sqrt(k) + kappa_r gap_r) for the basis and subspace, plus the
    first-order eigenvector change ||dT|| s_i, plus the FP32 accumulation of
    the reconstruction, (k + 2) sqrt(k) 2^-24."""
    import torch

    import parity_bounds as PB
    from paper_1805_05821_amd import foa as F

    rng = np.random.default_rng(n + N + max(r_force, 0))
    X = rng.standard_normal((n, N)).astype(np.float32)
    st = oracle.foa_batch(X.astype(np.float64), tol=0.0)
    g = run_gpu(X, "f32", tol=0.0)
    s = g["stream"]
    m = g["m"]
    assert g["q"] == st.q == N
    r = m if r_force < 0 else r_force
    if r_force > 0:
        assert s.truncate(r_force=r_force)[0] == r_force
        res = oracle.dmd_truncated(st, r)
        T = res["Ur"].T @ st.H[:m, :m] @ res["Ur"]
    else:
        res = oracle.dmd_untruncated(st)
        T = st.H[:m, :m]
    sig = PB.svals(st.beta[:m, :m])
    kr, gr = PB.kappa_r(sig, r), PB.gap_factor(sig, r)
    lam_c, Z, Yn, cond = PB.eig_condition(T)
    sens = PB.eigvec_sensitivity(lam_c, Z, Yn)
    Hn = np.linalg.norm(st.H[:m + 1, :m], 2)
    dT = PB.C * EPS32 * kr * (1.0 + 2.0 * gr) * Hn
    Phi_o, lam_o, kind_o = packed_modes(res, st.V)
    cols = Phi_o.shape[1]
    phi = torch.full((cols + 3, n), float("nan"), dtype=torch.float32, device="cuda")
    lam_g, kind, amp, err = F.foa_modes(s.ctx, m, phi, n, cols + 3, F.FOA_F32)
    ncols = int(np.sum(np.where(kind == 1, 2, 1)))
    assert ncols == cols and torch.isnan(phi[ncols:]).all()
    Pg = PB.unpack(phi[:ncols].double().cpu().numpy().T, kind)
    Po = PB.unpack(Phi_o, kind_o)
    ja, jb = PB.match(lam_g, lam_o)
    io, ic = PB.match(lam_o, lam_c)
    sens_o = np.empty(len(lam_o))
    sens_o[io] = sens[ic]
    k = m
    worst, worst_err = 0.0, 0.0
    for a, b in zip(ja, jb):
        e = PB.phase_aligned_error(Pg[a], Po[b])
        tol = PB.C * EPS32 * (np.sqrt(k) + kr * gr) + dT * sens_o[b] + (k + 2) * np.sqrt(k) * 2.0 ** -24
        worst, worst_err = max(worst, e / tol), max(worst_err, e)
    announce(f"n={n} N={N} r={r}: {len(ja)} entries / {ncols} columns, kappa_r={kr:.2e}, "
             f"max phase-aligned column error {worst_err:.2e}, max err/bound {worst:.2e}")
    assert worst <= 1.0
    s.close()
