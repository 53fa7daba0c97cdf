"""Batched form (many independent streams, one graph launch per step)
through the C ABI, stream by stream against the oracle."""

import numpy as np
import pytest

import datagen
import oracle
from gpu_helpers import EPS32, EPS64, announce, kappa_of
from pins import match_eigs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    announce(request.node.nodeid)
    yield


def _streams(S=7, seed=3):
    bw = datagen.get_workload("batched_256")
    ws = datagen.batched_streams(bw, streams=S)
    rng = np.random.default_rng(seed)
    out = []
    for k, w in enumerate(ws):
        # smaller sizes keep the oracle fast; ragged n on purpose
        n = int(rng.integers(100, 30000)) if k else 64 * 37 + 5
        N = int(rng.integers(8, 60))
        X, lam, b = datagen.snapshots_numpy(w.with_n(n).with_N(N), dtype="float64")
        out.append(X)
    return out


def _run_batch(Xs, prec, steps=None, nmax=None, tune=None, mutate=None):
    import torch

    from paper_1805_05821_amd.stream import FOABatch

    S = len(Xs)
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    nmax = nmax or N
    dev = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    bt = FOABatch(n, nmax, prec=prec, tune_table=tune, ws_fill=0xFF)
    T = steps or max(N)
    for k in range(T):
        xs = [dev[s][k] if k < N[s] else None for s in range(S)]
        bt.push(xs)
    q, st = bt.sync()
    return bt, q, st


def _view_state(bt, s):
    from paper_1805_05821_amd import foa as F

    v = bt.view(s)
    H, B, q, m = F.foa_get_state(v)
    V = np.zeros((bt.n[s], q))
    if q:
        import torch

        out = torch.empty((q, bt.n[s]), dtype=torch.float64, device="cuda")
        F.foa_copy_basis(v, out, bt.n[s], F.FOA_F64, q)
        V = out.cpu().numpy().T
    return H, B, q, m, V


def test_batch_f64_matches_oracle_per_stream():
    Xs = _streams()
    bt, q, st = _run_batch(Xs, "f64")
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        H, B, qq, m, V = _view_state(bt, s)
        assert qq == q[s] == ref.q, (s, qq, q[s], ref.q)
        kap = kappa_of(ref.beta[:m, :m])
        tol = 100 * EPS64 * kap * qq
        eH = np.abs(H[:qq, :m] - ref.H[:qq, :m]).max() / np.abs(ref.H[:qq, :m]).max()
        eB = np.abs(B[:qq, :qq] - ref.beta[:qq, :qq]).max() / np.abs(ref.beta[:qq, :qq]).max()
        eV = np.abs(V - ref.V[:, :qq]).max()
        announce(f"stream {s}: n={X.shape[0]} q={qq} kappa={kap:.1e} relH={eH:.1e} relB={eB:.1e} V={eV:.1e}")
        assert eH <= tol and eB <= tol and eV <= tol
    bt.close()


def test_batch_f32_within_bound():
    Xs = _streams(seed=4)
    bt, q, st = _run_batch(Xs, "f32")
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        H, B, qq, m, V = _view_state(bt, s)
        assert qq == ref.q
        kap = kappa_of(ref.beta[:m, :m])
        eH = np.linalg.norm(H[:m, :m] - ref.H[:m, :m], 2) / np.linalg.norm(ref.H[:m, :m], 2)
        orth = np.linalg.norm(np.eye(qq) - V.T @ V, 2)
        announce(f"stream {s}: kappa={kap:.1e} relH2={eH:.1e} orth={orth:.1e}")
        assert eH <= 10 * EPS32 * kap
        assert orth <= 10 * np.sqrt(qq) * EPS32
    bt.close()


def test_batch_f32_noise_floor():
    """Batched three-sweep form on the throughput recipe at small n (noise-
    floor snapshots): every stream orthogonal to 10 sqrt(q) eps32 and within
    10 eps32 kappa_2 of the FP64 oracle."""
    w = datagen.get_workload("noisy_2p24x500")
    Xs = [datagen.snapshots_numpy(w.with_n(n).with_N(N), dtype="float64")[0]
          for n, N in ((5000, 500), (20000, 500), (3000, 77))]
    bt, q, st = _run_batch(Xs, "f32")
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        H, B, qq, m, V = _view_state(bt, s)
        assert qq == ref.q
        kap = kappa_of(ref.beta[:m, :m])
        eH = np.linalg.norm(H[:m, :m] - ref.H[:m, :m], 2) / np.linalg.norm(ref.H[:m, :m], 2)
        orth = np.linalg.norm(np.eye(qq) - V.T @ V, 2)
        announce(f"stream {s}: n={X.shape[0]} q={qq} kappa={kap:.1e} relH2={eH:.1e} orth={orth:.1e}")
        assert eH <= 10 * EPS32 * kap
        assert orth <= 10 * np.sqrt(qq) * EPS32
    bt.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_late_starting_streams(prec):
    """Streams that start several pushes after the reset (idle before), next
    to one long stream whose basis grows past 128 columns: each push's graph
    leaves out only the buckets that no stream can have reached by then, so
    the lagging streams still find their narrower buckets launched.  Every
    stream against the oracle on its own snapshots."""
    import torch

    from paper_1805_05821_amd.stream import FOABatch

    Xs = _streams(S=4, seed=7)
    bw = datagen.get_workload("batched_256")
    w = datagen.batched_streams(bw, streams=1)[0]
    Xl, _, _ = datagen.snapshots_numpy(w.with_n(64 * 31 + 9).with_N(150), dtype="float64")
    Xs.append(Xl)
    off = [0, 9, 33, 70, 0]
    S = len(Xs)
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    dev = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    bt = FOABatch(n, N, prec=prec, ws_fill=0xFF)
    T = max(o + m for o, m in zip(off, N))
    for k in range(T):
        bt.push([dev[s][k - off[s]] if off[s] <= k < off[s] + N[s] else None for s in range(S)])
    q, st = bt.sync()
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        H, B, qq, m, V = _view_state(bt, s)
        assert qq == q[s] == ref.q, (s, qq, q[s], ref.q)
        kap = kappa_of(ref.beta[:m, :m])
        eH = np.linalg.norm(H[:m, :m] - ref.H[:m, :m], 2) / np.linalg.norm(ref.H[:m, :m], 2)
        announce(f"{prec} stream {s}: start {off[s]} n={n[s]} q={qq} kappa={kap:.1e} relH2={eH:.1e}")
        eps = EPS64 if prec == "f64" else EPS32
        assert eH <= (100 * qq if prec == "f64" else 10) * eps * kap
    bt.close()


def test_batch_equals_single_streams_and_replays(tmp_path):
    """Same results as single streams (to rounding), and bitwise-equal results
    from two batches with the same launch configuration (the second reads the
    first's entry in the tune table; the row-pass decomposition, and so the
    summation order, depends on the grid and the smallest range)."""
    from gpu_helpers import run_gpu

    Xs = _streams(S=4, seed=5)
    table = str(tmp_path / "tune.json")
    a, qa, _ = _run_batch(Xs, "f64", tune=table)
    b, qb, _ = _run_batch(Xs, "f64", tune=table)
    for s, X in enumerate(Xs):
        Ha, Ba, _, _, _ = _view_state(a, s)
        Hb, Bb, _, _, _ = _view_state(b, s)
        assert np.array_equal(Ha, Hb) and np.array_equal(Ba, Bb)
        g = run_gpu(X, "f64")
        m = g["m"]
        assert np.abs(Ha[:, :m] - g["H"][:, :m]).max() <= 1e-9 * np.abs(g["H"]).max()
    a.close()
    b.close()


def test_batch_capacity_idle_and_nonfinite():
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    Xs = _streams(S=3, seed=6)
    Xs[1] = Xs[1].copy()
    Xs[1][17, 4] = np.nan
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    nmax = [5, N[1], N[2]]  # stream 0 gets more snapshots than its capacity
    dev = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    bt = FOABatch(n, nmax, prec="f64")
    for k in range(max(N)):
        xs = [dev[s][k] if k < N[s] else None for s in range(3)]
        if k % 3 == 1:
            xs[2] = None  # idle steps do not advance stream 2
        bt.push(xs)
    q, st = bt.sync()
    assert q[0] == 5 and st[0] == F.FOA_E_CAPACITY
    assert q[1] == 4 and st[1] == F.FOA_E_NONFINITE
    fed = [k for k in range(N[2]) if k % 3 != 1]
    ref = oracle.foa_batch(Xs[2][:, fed])
    H, B, qq, m, V = _view_state(bt, 2)
    assert qq == ref.q and st[2] == 0
    assert np.abs(H[:qq, :m] - ref.H[:qq, :m]).max() <= 1e-8 * np.abs(ref.H[:qq, :m]).max()
    bt.close()


def test_batch_views_modes_and_tune_table(tmp_path):
    from paper_1805_05821_amd import foa as F

    Xs = _streams(S=3, seed=8)
    path = str(tmp_path / "tune.json")
    bt, q, st = _run_batch(Xs, "f64", tune=path)
    import json

    table = json.load(open(path))
    assert len(table["entries"]) == 1 and table["entries"][0]["unit_panels"] in (4, 16, 64)
    bt2, q2, st2 = _run_batch(Xs, "f64", tune=path)  # reuses the entry
    assert len(json.load(open(path))["entries"]) == 1
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        res = oracle.dmd_untruncated(ref)
        lam, kind, amp, err = F.foa_modes(bt.view(s), 64)
        assert match_eigs(lam, res["lam"][res["lam"].imag >= 0]) <= 1e-6
    import torch

    with pytest.raises(F.FOAError) as ei:  # pushes go through foa_batch_push only
        F.foa_push_snapshot(bt.view(0), torch.zeros(Xs[0].shape[0], dtype=torch.float64, device="cuda"))
    assert ei.value.code == F.FOA_E_STATE
    bt.close()
    bt2.close()


def _forced_table(Xs, prec, tmp_path, persist, unit, name):
    """A tune table whose entry for this batch forces one configuration
    (the key comes from a first, tuned batch of the same shape)."""
    import json

    path = str(tmp_path / f"{name}.json")
    bt, _, _ = _run_batch(Xs, prec, steps=2, nmax=[X.shape[1] for X in Xs], tune=path)  # same key
    bt.close()
    table = json.load(open(path))
    e = table["entries"][0]
    e.update(persist=int(persist), unit_panels=int(unit))
    json.dump({"entries": [e]}, open(path, "w"))
    return path


def _streams_wide(seed=11):
    """Mixed widths for the persistent step: most streams at most 256
    columns, one beyond (taken by the bucket launches in persistent mode),
    ragged n, one stream longer than one work item."""
    Xs = _streams(S=6, seed=seed)
    w = datagen.get_workload("noisy_2p20x200")
    Xw, _, _ = datagen.snapshots_numpy(w.with_n(1500).with_N(290), dtype="float64")
    Xl, _, _ = datagen.snapshots_numpy(w.with_n(64 * 300 + 17).with_N(40), dtype="float64")
    return Xs + [Xw, Xl]


@pytest.mark.parametrize("unit", [8, 64])
def test_batch_persistent_f32_within_bound(tmp_path, unit):
    """Persistent step (one launch for the streams of up to 256 columns):
    every stream within the FP32 bound of the oracle; the run leaves the
    wait-error flag clear (sync returns without error)."""
    Xs = _streams_wide()
    nmax = [X.shape[1] for X in Xs]
    table = _forced_table(Xs, "f32", tmp_path, True, unit, "p")
    bt, q, st = _run_batch(Xs, "f32", tune=table)
    for s, X in enumerate(Xs):
        ref = oracle.foa_batch(X)
        H, B, qq, m, V = _view_state(bt, s)
        assert qq == ref.q == nmax[s]
        kap = kappa_of(ref.beta[:m, :m])
        eH = np.linalg.norm(H[:m, :m] - ref.H[:m, :m], 2) / np.linalg.norm(ref.H[:m, :m], 2)
        orth = np.linalg.norm(np.eye(qq) - V.T @ V, 2)
        announce(f"persistent unit {unit} stream {s}: n={X.shape[0]} q={qq} kappa={kap:.1e} relH2={eH:.1e} orth={orth:.1e}")
        assert eH <= 10 * EPS32 * kap
        assert orth <= 10 * np.sqrt(qq) * EPS32
    bt.close()


def test_batch_persistent_replays_and_matches_buckets(tmp_path):
    """Two persistent batches with the same configuration give bitwise-equal
    results (partial sums go to slot = work item, whichever workgroup ran
    it); the bucket launches give the same results to rounding."""
    Xs = _streams_wide(seed=12)
    tp = _forced_table(Xs, "f32", tmp_path, True, 16, "p")
    tb = _forced_table(Xs, "f32", tmp_path, False, 16, "b")
    a, qa, _ = _run_batch(Xs, "f32", tune=tp)
    b, qb, _ = _run_batch(Xs, "f32", tune=tp)
    c, qc, _ = _run_batch(Xs, "f32", tune=tb)
    assert np.array_equal(qa, qb) and np.array_equal(qa, qc)
    for s in range(len(Xs)):
        Ha, Ba, _, m, _ = _view_state(a, s)
        Hb, Bb, _, _, _ = _view_state(b, s)
        Hc, Bc, _, _, _ = _view_state(c, s)
        assert np.array_equal(Ha, Hb) and np.array_equal(Ba, Bb)
        assert np.abs(Ha[:, :m] - Hc[:, :m]).max() <= 1e-5 * np.abs(Hc[:, :m]).max()
    a.close()
    b.close()
    c.close()


def test_batch_persistent_capacity_idle_and_nonfinite(tmp_path):
    """Persistent step with a stream past its capacity, idle steps and a
    non-finite snapshot: the same outcomes as the bucket launches."""
    import json

    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    Xs = _streams(S=3, seed=6)
    Xs[1] = Xs[1].copy()
    Xs[1][17, 4] = np.nan
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    nmax = [5, N[1], N[2]]
    path = str(tmp_path / "t.json")
    FOABatch(n, nmax, prec="f32", tune_table=path).close()
    table = json.load(open(path))
    table["entries"][0].update(persist=1, unit_panels=8)
    json.dump(table, open(path, "w"))
    dev = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    bt = FOABatch(n, nmax, prec="f32", tune_table=path)
    for k in range(max(N)):
        xs = [dev[s][k] if k < N[s] else None for s in range(3)]
        if k % 3 == 1:
            xs[2] = None
        bt.push(xs)
    q, st = bt.sync()
    assert q[0] == 5 and st[0] == F.FOA_E_CAPACITY
    assert q[1] == 4 and st[1] == F.FOA_E_NONFINITE
    fed = [k for k in range(N[2]) if k % 3 != 1]
    ref = oracle.foa_batch(Xs[2][:, fed])
    H, B, qq, m, V = _view_state(bt, 2)
    kap = kappa_of(ref.beta[:m, :m])
    eH = np.linalg.norm(H[:m, :m] - ref.H[:m, :m], 2) / np.linalg.norm(ref.H[:m, :m], 2)
    assert qq == ref.q and st[2] == 0 and eH <= 10 * EPS32 * kap
    bt.close()


def test_batch_persistent_wait_bound_reports_error(tmp_path, monkeypatch):
    """A persistent-step barrier wait that gives up sets the error flag, and
    foa_batch_sync reports it as a device error.  The host forces it by
    bounding every wait to zero polls (FOA_PERSIST_SPIN=0), so every kernel
    still ends normally.  A batch made without the bound then runs to
    completion."""
    from paper_1805_05821_amd import foa as F

    Xs = _streams(S=3, seed=13)
    table = _forced_table(Xs, "f32", tmp_path, True, 8, "spin")
    monkeypatch.setenv("FOA_PERSIST_SPIN", "0")
    with pytest.raises(F.FOAError) as err:
        _run_batch(Xs, "f32", tune=table)
    assert err.value.code == F.FOA_E_DEVICE
    monkeypatch.delenv("FOA_PERSIST_SPIN")
    bt, q, st = _run_batch(Xs, "f32", tune=table)
    assert list(q) == [X.shape[1] for X in Xs] and not any(st)
    bt.close()
