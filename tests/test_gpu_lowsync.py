"""The one-reduction form (foa_set_form(FOA_FORM_ONE_REDUCTION)) through the C
ABI, against the sequential oracle of Algorithm 1 (the same factors in exact
arithmetic) with the gates of the FP32-CGS2 form, and against the oracle of
the one-reduction form itself (oracle/lowsync.py: the same operations, so
FP64 agreement within a few ulps scaled by kappa)."""

import numpy as np
import pytest

import datagen
import oracle
import oracle.lowsync as LS
import parity_bounds as PB
from gpu_helpers import EPS32, EPS64, announce, kappa_of, rel, run_gpu
from pins import _known_A, _krylov, match_eigs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()
    announce(request.node.nodeid)
    yield
    torch.cuda.empty_cache()


def _noisy(n, N, name="noisy_2p20x200"):
    w = datagen.get_workload(name).with_n(n).with_N(N)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    return X


def _vs_ls_oracle_f64(g, X, c=10.0, tol=None):
    """FP64 basis against the one-reduction oracle: same operations, summation
    order aside: H_bar, beta, V within c q eps64 kappa_2 (Frobenius-relative)
    and column by column against the prefix condition number."""
    ref = LS.run(X, tol=tol)
    q, m = g["q"], g["m"]
    assert q == ref.q and g["status"] == (1 if ref.status == "invariant" else 0)
    kap = kappa_of(ref.beta[:max(m, 1), :max(m, 1)]) if m > 0 else 1.0
    tol = c * q * EPS64 * max(kap, 1.0)
    rows = min(q + 1, ref.H.shape[0])
    eH = rel(g["H"][:rows, :m], ref.H[:rows, :m])
    bc = q + 1 if ref.status == "invariant" else q
    eB = rel(g["beta"][:q, :bc], ref.beta[:q, :bc])
    eV = np.abs(g["V"] - LS.basis(ref)).max()
    announce(f"vs one-reduction oracle: q={q} kappa={kap:.1e} relH={eH:.1e} relB={eB:.1e} maxV={eV:.1e} tol={tol:.1e}")
    assert eH <= tol and eB <= tol and eV <= tol
    return ref


@pytest.mark.parametrize("n,N", [(1, 1), (37, 9), (64, 33), (65, 60), (1000, 130), (4133, 257), (12293, 200)])
def test_f64_vs_oracles_ragged(n, N):
    """FP64 basis, FP64 snapshots, every tile width (1..16 groups) and ragged
    rows: against the one-reduction oracle (same operations) and against the
    sequential oracle (the same factorisation)."""
    if n < N:
        X = np.random.default_rng(n + N).standard_normal((n, N))
    else:
        X = _noisy(n, N)
    g = run_gpu(X, "f64", tol=0.0, form="one_reduction")
    _vs_ls_oracle_f64(g, X, tol=0.0)
    st = oracle.foa_batch(X, tol=0.0)
    q, m = g["q"], g["m"]
    assert q == st.q
    if m > 0:
        kap = kappa_of(st.beta[:m, :m])
        eH = rel(g["H"][:q, :m], st.H[:q, :m])
        announce(f"vs sequential oracle: relH={eH:.1e} (bound {100 * q * EPS64 * kap:.1e})")
        assert eH <= 100 * q * EPS64 * kap
    g["stream"].close()


@pytest.mark.parametrize("n,N", [(777, 40), (20000, 129), (100037, 300), (4097, 500)])
def test_f32_basis_gates(n, N):
    """FP32 basis with FP64 accumulation against the sequential FP64 oracle:
    ||H32 - H||_2 / ||H||_2 <= 10 eps32 kappa_2, ||I - V^T V||_2 <= 10 sqrt(q)
    eps32, factorisation on every row <= 10 sqrt(q) eps32, and the truncated
    eigenvalues at the FP32 rank rule within 10 eps32 kappa_r cond_i.  The
    widths cover every tile shape of the FP32 sweep (4 and 8 wavefronts,
    1..16 groups)."""
    import torch

    X = _noisy(n, N)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f32", form="one_reduction")
    q, m = g["q"], g["m"]
    assert q == st.q == N and m == N - 1
    sig = PB.svals(st.beta[:m, :m])
    kap = sig[0] / sig[-1]
    eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
    V = g["V"]
    orth = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    fact = np.linalg.norm(X - V @ g["beta"][:q, :q]) / np.linalg.norm(X)
    announce(f"f32 n={n} N={N}: kappa_2={kap:.1e} relH2={eH:.1e} (bound {10 * EPS32 * kap:.1e}) "
             f"orth={orth:.1e} fact={fact:.1e} (bound {10 * np.sqrt(q) * EPS32:.1e})")
    assert eH <= 10 * EPS32 * kap
    assert orth <= 10 * np.sqrt(q) * EPS32
    assert fact <= 10 * np.sqrt(q) * EPS32
    r = oracle.truncation_rank(sig, st.q, "f32")
    g["stream"].truncate(r_force=r)
    lam_g, _ = g["stream"].indicators()
    res = oracle.dmd_truncated(st, r)
    keep = res["lam"].imag >= 0
    P_o, T_o, _ = PB.truncated_projection(st.H[:m, :m], st.beta[:m, :m], r)
    lam_c, Z, Yn, cond = PB.eig_condition(T_o)
    io, ic = PB.match(res["lam"][keep], lam_c)
    cond_o = np.empty(int(keep.sum()))
    cond_o[io] = cond[ic]
    kr = PB.kappa_r(sig, r)
    ratio, err, _ = PB.eig_gate(lam_g, res["lam"][keep], cond_o, EPS32, kr)
    announce(f"  truncated r={r} kappa_r={kr:.1e}: eigenvalues max err {err:.1e}, err/bound {ratio:.1e}")
    assert 10 * EPS32 * kr < 1.0 and ratio <= 1.0
    g["stream"].close()


@pytest.mark.timeout(600)
def test_headline_recipe_reduced_n():
    """noisy_2p24x500's recipe at n = 2^18 + 37 (kappa_2 ~ 2e9, FP32
    snapshots, FP32 basis): orthogonality, the FP32 rank rule equal to the
    oracle's, and the truncated gates (eigenvalues, basis-free projection,
    indicators) against the sequential oracle."""
    from test_gpu_recipes import HEADLINE_ROWS, _gram_gpu, _truncated_checks

    w = datagen.get_workload("noisy_2p24x500").with_n(HEADLINE_ROWS)
    X32, _, _ = datagen.snapshots_numpy(w)
    st = oracle.foa_batch(X32.astype(np.float64))
    g = run_gpu(X32, "f32", form="one_reduction")
    q, m = g["q"], g["m"]
    assert q == st.q == w.N
    orth = np.linalg.norm(np.eye(q) - _gram_gpu(g["stream"], q), 2)
    sig = PB.svals(st.beta[:m, :m])
    eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
    announce(f"one-reduction f32: kappa_2={sig[0] / sig[-1]:.2e} relH2={eH:.2e} ||I-V^TV||={orth:.2e} "
             f"(bound {10 * np.sqrt(q) * EPS32:.1e})")
    assert orth <= 10 * np.sqrt(q) * EPS32
    r_g, _ = g["stream"].truncate()
    r_o = oracle.truncation_rank(sig, st.q, "f32")
    assert r_g == r_o, (r_g, r_o)
    _truncated_checks(g, st, r_o, EPS32, "one-reduction f32 truncated (default rank)")
    g["stream"].close()


def test_exact_rank_breakdown():
    """exact_rank_4096x64, FP64 basis: the dependent snapshot 21 is found when
    its column finishes; the stream is invariant with q = 20 and the 20
    generating eigenvalues to 1e-9."""
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, _ = datagen.snapshots_numpy(w)
    g = run_gpu(X, "f64", form="one_reduction")
    assert g["status"] == 1 and g["q"] == 20, (g["status"], g["q"])
    _vs_ls_oracle_f64(g, X)
    m = g["m"]
    err = match_eigs(np.linalg.eigvals(g["H"][:m, :m]), np.concatenate([lam, lam.conj()]))
    announce(f"max |d lambda| = {err:.1e}")
    assert err <= 1e-9
    g["stream"].close()


def test_nonfinite_snapshot_and_zero_first():
    """A NaN in snapshot 8: not committed, the stream stops (FOA_E_NONFINITE)
    and the first 7 snapshots are completed, as in the oracle; a zero first
    snapshot leaves q = 0 (FOA_E_ZERO)."""
    from paper_1805_05821_amd import foa as F

    X = _noisy(5000, 12)
    Xb = X.copy()
    Xb[123, 7] = np.nan
    g = run_gpu(Xb, "f64", form="one_reduction")
    assert g["status"] == F.FOA_E_NONFINITE and g["q"] == 7
    ref = LS.run(X[:, :7], capacity=12)
    assert rel(g["H"][:7, :6], ref.H[:7, :6]) <= 1e-12 and rel(g["beta"][:7, :7], ref.beta[:7, :7]) <= 1e-12
    g["stream"].close()
    z = run_gpu(np.zeros((300, 4)), "f64", form="one_reduction")
    assert z["status"] == F.FOA_E_ZERO and z["q"] == 0
    z["stream"].close()


def test_sync_midway_and_determinism():
    """Synchronising in the middle finishes the pending columns and the stream
    goes on (the same factorisation to rounding); two runs with the same
    pushes and syncs are bitwise equal; an FP32-basis run with FP32
    snapshots matches the oracle's FP32-storage form."""
    import torch

    from paper_1805_05821_amd.stream import FOAStream

    X = _noisy(30011, 60)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    outs = []
    for rep in range(2):
        s = FOAStream(X.shape[0], 60, prec="f64", form="one_reduction", ws_fill=0xFF)
        for k in range(60):
            s.push(Xd[k])
            if k in (0, 1, 9, 30):
                s.sync()
        s.sync()
        outs.append(s.state())
        s.close()
    assert all(np.array_equal(a, b) for a, b in zip(outs[0][:2], outs[1][:2]))
    ref = LS.init(X.shape[0], 60)
    for k in range(60):
        LS.push(ref, X[:, k])
        if k in (0, 1, 9, 30):
            LS.flush(ref)
    LS.flush(ref)
    H = outs[0][0]
    kap = kappa_of(ref.beta[:59, :59])
    e = rel(H[:60, :59], ref.H[:60, :59])
    announce(f"sync midway vs oracle with the same flushes: relH={e:.1e} kappa={kap:.1e}")
    assert e <= 10 * 60 * EPS64 * kap
    X32 = X.astype(np.float32)
    g = run_gpu(X32, "f32", form="one_reduction")
    r32 = LS.run(X32.astype(np.float64), storage="f32")
    q = g["q"]
    kap = kappa_of(r32.beta[:q - 1, :q - 1])
    eH = np.linalg.norm(g["H"][:q, :q - 1] - r32.H[:q, :q - 1], 2) / np.linalg.norm(r32.H[:q, :q - 1], 2)
    announce(f"f32 vs the oracle's FP32-storage form: relH2={eH:.1e} (bound {10 * EPS32 * kap:.1e})")
    assert eH <= 10 * EPS32 * kap
    g["stream"].close()


def test_modes_and_indicators_known_A():
    """Modes and indicators of the one-reduction form: indicator equals the
    true residual ||A phi - lambda phi|| for unit modes (Section 3.2.3)."""
    from test_gpu_modes import _modes

    A, psi1 = _known_A(n=300, seed=21)
    X = _krylov(A, psi1, 14)
    g = run_gpu(X, "f64", tol=0.0, form="one_reduction")
    lam, kind, amp, err, Phi = _modes(g, X.shape[0])
    worst, col = 0.0, 0
    for e_i, (l, k) in enumerate(zip(lam, kind)):
        phi = Phi[:, col] + (1j * Phi[:, col + 1] if k == 1 else 0.0)
        col += 2 if k == 1 else 1
        true = np.linalg.norm(A @ phi - l * phi) / np.linalg.norm(phi)
        worst = max(worst, abs(true - err[e_i]) / max(true, 1e-12))
    announce(f"max rel |indicator - residual| = {worst:.2e}")
    assert worst <= 1e-6
    g["stream"].close()


def test_form_rules():
    """The form is chosen before the first push; an FP64 basis holds at most
    257 snapshots in this form; the blocked form and the in-place snapshot
    buffer are not available on a one-reduction stream."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOAStream

    s = FOAStream(1000, 20, prec="f32")
    s.push(torch.ones(1000, device="cuda"))
    with pytest.raises(F.FOAError) as e:
        F.foa_set_form(s.ctx, F.FOA_FORM_ONE_REDUCTION)
    assert e.value.code == F.FOA_E_STATE
    s.reset()
    F.foa_set_form(s.ctx, F.FOA_FORM_ONE_REDUCTION)
    with pytest.raises(F.FOAError) as e:
        F.foa_next_column(s.ctx)
    assert e.value.code == F.FOA_E_STATE
    with pytest.raises(F.FOAError) as e:
        s.push_blocked(torch.ones((4, 1000), device="cuda"))
    assert e.value.code == F.FOA_E_STATE
    s.close()
    with pytest.raises(F.FOAError) as e:
        FOAStream(1000, 300, prec="f64", form="one_reduction")
    assert e.value.code == F.FOA_E_ARG


@pytest.mark.parametrize("n,N", [(5000, 384), (5000, 500), (20000, 500)])
def test_f32_noise_floor_gram_correction(n, N):
    """FP32 basis where new snapshots sit at the data's noise floor and the
    stored basis is orthonormal only to E = Q^T Q - I of a few 1e-8 (the
    noisy_2p24x500 recipe at small n): with the Gram-corrected second
    projection, orthogonality and factorisation stay within 10 sqrt(q) eps32
    and H_bar within 10 eps32 kappa_2 of the sequential oracle; the single
    stream and a batch of the same stream agree to that bound."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    w = datagen.get_workload("noisy_2p24x500").with_n(n).with_N(N)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f32", form="one_reduction")
    q, m = g["q"], g["m"]
    assert q == st.q == N
    V = g["V"]
    orth = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    fact = np.linalg.norm(X - V @ g["beta"][:q, :q]) / np.linalg.norm(X)
    sig = PB.svals(st.beta[:m, :m])
    kap = sig[0] / sig[-1]
    eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
    b = 10 * np.sqrt(q) * EPS32
    announce(f"n={n} N={N}: ||I-V^TV||={orth:.2e} factorisation {fact:.2e} (bound {b:.1e}) "
             f"relH2={eH:.2e} (bound {10 * EPS32 * kap:.1e})")
    assert orth <= b and fact <= b
    assert eH <= 10 * EPS32 * kap
    g["stream"].close()
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    bt = FOABatch([n], [N], prec="f32", form="one_reduction")
    for k in range(N):
        bt.push_ptrs(torch.tensor([Xd[k].data_ptr()], dtype=torch.int64, device="cuda"), F.FOA_F64)
        torch.cuda.synchronize()
    qb, sb = bt.sync()
    view = bt.view(0)
    Vb = torch.empty((N, n), dtype=torch.float64, device="cuda")
    F.foa_copy_basis(view, Vb, n, F.FOA_F64, N)
    Vb = Vb.cpu().numpy().T
    orth_b = np.linalg.norm(np.eye(N) - Vb.T @ Vb, 2)
    announce(f"  batched: q={qb[0]} status={sb[0]} ||I-V^TV||={orth_b:.2e}")
    assert qb[0] == N and sb[0] == 0 and orth_b <= b
    bt.close()
