"""Parity of the HIP push path (through the C ABI) with the CPU oracle."""

import numpy as np
import pytest

import datagen
import oracle
import parity_bounds as PB
from gpu_helpers import EPS32, EPS64, announce, kappa_of, rel, run_gpu
from pins import match_eigs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    announce(request.node.nodeid)
    yield


def _noisy(n, N, seed_name="noisy_2p20x200"):
    w = datagen.get_workload(seed_name).with_n(n).with_N(N)
    X, lam, b = datagen.snapshots_numpy(w, dtype="float64")
    return X


def _compare_f64(g, st, c=100.0):
    """FP64 GPU vs FP64 oracle: rounding-order differences scaled by kappa."""
    q = st.q
    assert g["q"] == q, (g["q"], q)
    m = oracle.projected_size(st)
    assert g["m"] == m
    kap = kappa_of(st.beta[:max(m, 1), :max(m, 1)]) if m > 0 else 1.0
    tol = c * EPS64 * max(kap, 1.0) * q
    rows = min(q + 1, st.H.shape[0])
    eH = rel(g["H"][:rows, :m], st.H[:rows, :m])
    bc = q + 1 if st.status == "invariant" else q
    eB = rel(g["beta"][:q, :bc], st.beta[:q, :bc])
    eV = np.abs(g["V"] - st.V[:, :q]).max()
    col = PB.column_gate_f64(g, st)
    announce(f"q={q} kappa={kap:.2e} relH={eH:.2e} relB={eB:.2e} maxV={eV:.2e} tol={tol:.2e} "
             f"column err/bound {col:.2e}")
    assert eH <= tol and eB <= tol and eV <= tol
    assert col <= 1.0
    return kap


@pytest.mark.parametrize("n", [777, 2048, 20000, 100037])
def test_f64_tight_well_conditioned(n):
    """kappa_2(X) <= ~3: GPU and oracle agree to a few ulps scaled by q.
    Krylov sequence of a known map for small n, Gaussian snapshots for large n."""
    from pins import _known_A, _krylov

    if n <= 2048:
        A, psi1 = _known_A(n=n, seed=31)
        X = _krylov(A, psi1, 30)
    else:
        X = np.random.default_rng(n).standard_normal((n, 30))
    st = oracle.foa_batch(X, tol=0.0)
    g = run_gpu(X, "f64", tol=0.0)
    q, m = g["q"], g["m"]
    assert q == st.q == 30
    eH = np.abs(g["H"][:q, :m] - st.H[:q, :m]).max() / np.abs(st.H[:q, :m]).max()
    eB = np.abs(g["beta"][:q, :q] - st.beta[:q, :q]).max() / np.abs(st.beta[:q, :q]).max()
    eV = np.abs(g["V"] - st.V[:, :q]).max()
    announce(f"relH={eH:.2e} relB={eB:.2e} maxV={eV:.2e}")
    tol = 10 * q * EPS64
    assert eH <= tol and eB <= tol and eV <= tol


def test_exact_rank_recovers_eigenvalues():
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, _ = datagen.snapshots_numpy(w)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f64")
    assert g["status"] == 1 and g["q"] == 20, (g["status"], g["q"])  # FOA_INVARIANT
    _compare_f64(g, st)
    m = g["m"]
    ev = np.linalg.eigvals(g["H"][:m, :m])
    true = np.concatenate([lam, lam.conj()])
    err = match_eigs(ev, true)
    err_or = match_eigs(ev, oracle.dmd_untruncated(st)["lam"])
    announce(f"eig err vs generating {err:.2e} vs oracle {err_or:.2e}")
    assert err <= 1e-9 and err_or <= 1e-9


@pytest.mark.parametrize("n", [1, 37, 64, 65, 1000, 4096 + 37, 3 * 64 * 64 + 5])
def test_f64_ragged_rows(n):
    N = 12 if n < 12 else 24
    X = _noisy(max(n, 1), N)
    st = oracle.foa_batch(X, tol=0.0 if n < N else None)
    g = run_gpu(X, "f64", tol=0.0 if n < N else -1.0)
    if n < N:
        # at most n independent directions: both sides stop or keep going together
        assert g["q"] == st.q
    _compare_f64(g, st)


@pytest.mark.parametrize("N", [2, 33, 65, 130, 300])
def test_f64_column_buckets(N):
    """Spans every register-tile bucket (32, 64, 128, 256, 512 columns)."""
    X = _noisy(5000, N)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f64")
    _compare_f64(g, st)


def test_f64_f32_snapshots():
    X = _noisy(4000, 40).astype(np.float32)
    st = oracle.foa_batch(X.astype(np.float64))
    g = run_gpu(X, "f64")
    _compare_f64(g, st)


@pytest.mark.parametrize("n,N", [(5000, 500), (20000, 500)])
def test_f32_cgs2_noise_floor(n, N):
    """The throughput recipe at small n (noise-floor snapshots, new directions
    about 1e-8 of their norm, FP32 basis orthonormal only to about that): the
    three projections per push (the Arnoldi recurrence's and CGS2's two) keep
    the basis orthogonal to 10 sqrt(q) eps32 and H within 10 eps32 kappa_2,
    without the corrections the one-reduction and blocked forms need there
    (two projections that take the rounded basis as orthonormal lose it)."""
    w = datagen.get_workload("noisy_2p24x500").with_n(n).with_N(N)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f32", snap_dtype=None)
    q, m = g["q"], g["m"]
    kap = kappa_of(st.beta[:m, :m])
    eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
    orth = np.linalg.norm(np.eye(q) - g["V"].T @ g["V"], 2)
    announce(f"n={n} N={N}: q={q} kappa={kap:.2e} relH2={eH:.2e} (bound {10 * EPS32 * kap:.2e}) orth={orth:.2e}")
    assert q == st.q
    assert eH <= 10 * EPS32 * kap
    assert orth <= 10 * np.sqrt(q) * EPS32


@pytest.mark.parametrize("N", [40, 140])
def test_f32_cgs2_within_bound(N):
    """FP32-stored basis, FP64 accumulation: ||H32 - H64||_2 / ||H64||_2 and
    per-eigenvalue errors within 10 eps32 kappa_2, orthogonality within
    10 sqrt(k) eps32."""
    X = _noisy(6000, N)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f32", snap_dtype=None)
    q, m = g["q"], g["m"]
    assert q == st.q
    kap = kappa_of(st.beta[:m, :m])
    bound = 10 * EPS32 * kap
    H64 = st.H[:m, :m]
    eH = np.linalg.norm(g["H"][:m, :m] - H64, 2) / np.linalg.norm(H64, 2)
    V = g["V"]
    orth = np.linalg.norm(np.eye(q) - V.T @ V, 2)
    ev32 = np.linalg.eigvals(g["H"][:m, :m])
    ev64 = np.linalg.eigvals(H64)
    eE = match_eigs(ev32, ev64)
    announce(f"kappa={kap:.2e} bound={bound:.2e} relH2={eH:.2e} orth={orth:.2e} eig={eE:.2e}")
    assert eH <= bound
    assert orth <= 10 * np.sqrt(q) * EPS32
    assert eE <= bound


def test_deterministic_and_prefetch_invariant():
    X = _noisy(9000, 70)
    a = run_gpu(X, "f32")
    b = run_gpu(X, "f32")
    c = run_gpu(X, "f32", options={"prefetch": 0})
    d = run_gpu(X, "f64", options={"prefetch": 1})
    e = run_gpu(X, "f64", options={"prefetch": 0})
    for u, v in ((a, b), (a, c), (d, e)):
        assert np.array_equal(u["H"], v["H"]) and np.array_equal(u["beta"], v["beta"])
        assert np.array_equal(u["V"], v["V"])


def test_grid_sizes_agree():
    X = _noisy(20000, 50)
    st = oracle.foa_batch(X)
    for grid in (1, 7, 64, 0):
        g = run_gpu(X, "f64", options={"grid": grid})
        _compare_f64(g, st)


@pytest.mark.parametrize("nw", [0, 4, 8, 16])
def test_f32_workgroup_shapes_agree(nw):
    """FP32 basis, every workgroup shape of the row passes (0 = automatic: 4
    wavefronts up to 128 columns, 8 beyond; 4 falls back to 8 above 256
    columns), N = 300 spanning all column tiles: within the FP32 bound of the
    oracle."""
    X = _noisy(9000, 300)
    st = oracle.foa_batch(X)
    g = run_gpu(X, "f32", options={"nw": nw})
    m = st.q - 1
    kap = kappa_of(st.beta[:m, :m])
    eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
    orth = np.linalg.norm(np.eye(g["q"]) - g["V"].T @ g["V"], 2)
    announce(f"nw={nw}: kappa={kap:.2e} relH2={eH:.2e} orth={orth:.2e}")
    assert g["q"] == st.q and eH <= 10 * EPS32 * kap and orth <= 10 * np.sqrt(g["q"]) * EPS32


def test_block_push_equals_single_pushes():
    X = _noisy(3000, 30)
    a = run_gpu(X, "f64")
    b = run_gpu(X, "f64", block=True)
    assert np.array_equal(a["H"], b["H"]) and np.array_equal(a["beta"], b["beta"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_next_column_in_place(prec):
    """Snapshots written into the in-place buffer give bitwise the same state
    as pushes from a separate FP64 array (ragged n, several panels)."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOAStream

    X = _noisy(5000 + 37, 24)
    ref = run_gpu(X, prec)
    s = FOAStream(X.shape[0], X.shape[1], prec=prec, ws_fill=0xFF)
    addr = F.foa_next_column(s.ctx)
    assert addr % 8 == 0
    # a tensor view of the buffer, through the workspace tensor that holds it
    off = addr - s.ws.data_ptr()
    assert 0 <= off and off + 8 * X.shape[0] <= s.ws.numel()
    col = s.ws[off:off + 8 * X.shape[0]].view(torch.float64)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    for k in range(X.shape[1]):
        col.copy_(Xd[k])
        F.foa_push_snapshot(s.ctx, addr, F.FOA_F64)
    st, q = s.sync()
    H, B, q2, m = s.state()
    assert q == ref["q"]
    assert np.array_equal(H, ref["H"]) and np.array_equal(B, ref["beta"])
    s.close()


def test_zero_first_snapshot():
    X = _noisy(500, 5)
    X[:, 0] = 0.0
    g = run_gpu(X, "f64")
    assert g["status"] == -8 and g["q"] == 0  # FOA_E_ZERO


def test_nonfinite_snapshot_not_committed():
    X = _noisy(700, 10)
    Xb = X.copy()
    Xb[123, 6] = np.nan
    g = run_gpu(Xb, "f64")
    ref = oracle.foa_batch(Xb)
    assert g["status"] == -4 and g["q"] == 6 == ref.q  # FOA_E_NONFINITE
    _compare_f64(g, ref)


def test_capacity_and_state_errors():
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOAStream

    X = torch.from_numpy(np.ascontiguousarray(_noisy(300, 4).T)).cuda()
    s = FOAStream(300, 3, "f64")
    s.push_all(X[:3])
    with pytest.raises(F.FOAError) as ei:
        s.push(X[3])
    assert ei.value.code == F.FOA_E_CAPACITY
    # invariant stream refuses further pushes once the host knows
    w = datagen.get_workload("exact_rank_4096x64")
    Xe, _, _ = datagen.snapshots_numpy(w)
    Xt = torch.from_numpy(np.ascontiguousarray(Xe.T)).cuda()
    s2 = FOAStream(4096, 64, "f64")
    s2.push_all(Xt[:25])
    st, q = s2.sync()
    assert st == F.FOA_INVARIANT and q == 20
    with pytest.raises(F.FOAError) as ei:
        s2.push(Xt[25])
    assert ei.value.code == F.FOA_E_STATE
    s2.reset()
    s2.push_all(Xt[:5])
    assert s2.sync() == (F.FOA_OK, 5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_max_capacity(prec):
    """n_max = FOA_MAX_CAPACITY: all 512 snapshots (the widest column tile
    full), Gaussian snapshots of n = 1500 rows (kappa_2 small)."""
    from paper_1805_05821_amd import foa as F

    N = F.FOA_MAX_CAPACITY
    X = np.random.default_rng(512).standard_normal((1500, N))
    st = oracle.foa_batch(X)
    g = run_gpu(X, prec)
    if prec == "f64":
        _compare_f64(g, st)
    else:
        m = st.q - 1
        kap = kappa_of(st.beta[:m, :m])
        eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
        orth = np.linalg.norm(np.eye(g["q"]) - g["V"].T @ g["V"], 2)
        announce(f"f32 N={N}: kappa={kap:.2e} relH2={eH:.2e} orth={orth:.2e}")
        assert g["q"] == N and eH <= 10 * EPS32 * kap and orth <= 10 * np.sqrt(N) * EPS32
    g["stream"].close()
