"""The batched form with the one-reduction sweep (foa_batch_set_form with
FOA_FORM_ONE_REDUCTION) through the C ABI: every stream against the oracles
(the one-reduction oracle for an FP64 basis: same operations; the sequential
oracle with the FP32 gates for an FP32 basis), streams that are idle on some
steps or start late, a non-finite snapshot, the capacity rule, and the
benchmark's batched_256 shape."""

import numpy as np
import pytest

import datagen
import oracle
import oracle.lowsync as LS
import parity_bounds as PB
from gpu_helpers import EPS32, EPS64, announce, kappa_of, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()
    announce(request.node.nodeid)
    yield
    torch.cuda.empty_cache()


def _run_batch(Xs, prec, n_max=None, start=None, offers=None, stride=None, form="one_reduction", ws_fill=0xFF):
    """Push snapshot k of stream s at step start[s] + k stride[s] (NULL on the
    other steps); offers[s] snapshots are offered (default: all its
    columns)."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    S = len(Xs)
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    n_max = n_max or N
    start = start or [0] * S
    offers = offers or N
    stride = stride or [1] * S
    dt = torch.float64 if Xs[0].dtype == np.float64 else torch.float32
    Xd = [torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dt) for X in Xs]
    T = max(start[s] + (offers[s] - 1) * stride[s] + 1 for s in range(S))
    ptr = np.zeros((T, S), dtype=np.int64)
    for s in range(S):
        for k in range(offers[s]):
            ptr[start[s] + k * stride[s], s] = Xd[s].data_ptr() + Xd[s].stride(0) * Xd[s].element_size() * min(k, N[s] - 1)
    bt = FOABatch(n, n_max, prec=prec, form=form, ws_fill=ws_fill)
    dptr = torch.from_numpy(ptr).cuda()
    code = F.FOA_F64 if dt == torch.float64 else F.FOA_F32
    for t in range(T):
        bt.push_ptrs(dptr[t], code)
    q, st = bt.sync()
    out = []
    for s in range(S):
        v = bt.view(s)
        H, B, qv, m = F.foa_get_state(v)
        V = torch.empty((max(qv, 1), n[s]), dtype=torch.float64, device="cuda")
        if qv:
            F.foa_copy_basis(v, V, n[s], F.FOA_F64, qv)
        out.append(dict(q=int(q[s]), status=int(st[s]), H=H, beta=B, m=m, V=V[:qv].cpu().numpy().T, view=v))
    return bt, out


def _mixed():
    shapes = [(1, 1), (37, 20), (5000, 60), (30011, 129), (65, 40), (100037, 200), (4133, 257)]
    w = datagen.get_workload("noisy_2p20x200")
    return [np.asfortranarray(datagen.snapshots_numpy(w.with_n(n).with_N(N), dtype="float64")[0])
            for n, N in shapes]


def test_f64_every_stream_vs_oracle():
    """FP64 basis: every stream of a mixed batch (rows 1 .. 100037, 3 .. 257
    snapshots, so every tile bucket) against the one-reduction oracle (same
    operations: 10 q eps64 kappa_2); two streams start late and one is idle
    every other step."""
    Xs = _mixed()
    bt, out = _run_batch(Xs, "f64", start=[0, 5, 0, 0, 17, 0, 0], stride=[1, 1, 2, 1, 1, 1, 1])
    for s, (X, g) in enumerate(zip(Xs, out)):
        ref = LS.run(X)
        q, m = g["q"], g["m"]
        assert q == ref.q, (s, q, ref.q)
        kap = kappa_of(ref.beta[:max(m, 1), :max(m, 1)]) if m > 0 else 1.0
        rows = min(q + 1, ref.H.shape[0])
        eH = rel(g["H"][:rows, :m], ref.H[:rows, :m])
        eB = rel(g["beta"][:q, :q], ref.beta[:q, :q])
        eV = np.abs(g["V"] - LS.basis(ref)).max() if q else 0.0
        tol = 10 * q * EPS64 * max(kap, 1.0)
        announce(f"stream {s}: n={X.shape[0]} q={q} kappa={kap:.1e} relH={eH:.1e} relB={eB:.1e} maxV={eV:.1e} "
                 f"tol={tol:.1e}")
        assert eH <= tol and eB <= tol and eV <= tol
    bt.close()


def test_f32_gates_and_batch_equals_single():
    """FP32 basis: every stream within the FP32 gates against the sequential
    oracle (||H32 - H||_2 / ||H||_2 <= 10 eps32 kappa_2, ||I - V^T V||_2 <= 10
    sqrt(q) eps32); and each stream of the batch equals the same stream pushed
    alone in the one-reduction form to rounding (the two sum their partials in
    different workgroup ranges)."""
    import torch

    from gpu_helpers import run_gpu

    Xs = [X.astype(np.float32) for X in _mixed()]
    bt, out = _run_batch(Xs, "f32")
    for s, (X, g) in enumerate(zip(Xs, out)):
        st = oracle.foa_batch(X.astype(np.float64))
        q, m = g["q"], g["m"]
        assert q == st.q
        if m < 2:
            continue
        kap = kappa_of(st.beta[:m, :m])
        eH = np.linalg.norm(g["H"][:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2)
        orth = np.linalg.norm(np.eye(q) - g["V"].T @ g["V"], 2)
        single = run_gpu(X, "f32", form="one_reduction")
        eS = rel(g["H"][:q, :m], single["H"][:q, :m])
        single["stream"].close()
        announce(f"stream {s}: n={X.shape[0]} q={q} kappa={kap:.1e} relH2={eH:.1e} (bound {10 * EPS32 * kap:.1e}) "
                 f"orth={orth:.1e} batch vs single {eS:.1e}")
        assert eH <= 10 * EPS32 * kap
        assert orth <= 10 * np.sqrt(q) * EPS32
        assert eS <= 10 * EPS32 * kap
    bt.close()


def test_nonfinite_capacity_idle():
    """A NaN snapshot stops its stream only (FOA_E_NONFINITE, the snapshots
    before it completed as in the oracle); offering more snapshots than the
    capacity reports FOA_E_CAPACITY with the first n_max taken; the other
    streams are unaffected."""
    from paper_1805_05821_amd import foa as F

    w = datagen.get_workload("noisy_2p20x200")
    Xs = [np.asfortranarray(datagen.snapshots_numpy(w.with_n(n).with_N(N), dtype="float64")[0])
          for n, N in ((3000, 30), (7001, 30), (513, 30))]
    Xs[1][77, 11] = np.nan
    bt, out = _run_batch(Xs, "f64", n_max=[30, 30, 20], offers=[30, 30, 26])
    assert out[0]["status"] == 0 and out[0]["q"] == 30
    assert out[1]["status"] == F.FOA_E_NONFINITE and out[1]["q"] == 11
    ref = LS.run(Xs[1][:, :11], capacity=30)
    assert rel(out[1]["H"][:11, :10], ref.H[:11, :10]) <= 1e-12
    assert out[2]["status"] == F.FOA_E_CAPACITY and out[2]["q"] == 20
    ref2 = LS.run(Xs[2][:, :20])
    assert rel(out[2]["H"][:20, :19], ref2.H[:20, :19]) <= 1e-12
    bt.close()


def _bucket(j):
    return 0 if j <= 32 else 1 if j <= 64 else 2 if j <= 128 else 3 if j <= 256 else 4


@pytest.mark.timeout(900)
def test_batched_256_full_shape_vs_oracle():
    """All 256 streams of batched_256 in the one-reduction form (the
    configuration its autotuner picks), every tile bucket checked against the
    sequential oracle on the streams that end in it: orthogonality,
    untruncated G14 relation, truncated eigenvalues at the FP32 rank rule."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    bw = datagen.get_workload("batched_256")
    ws = datagen.batched_streams(bw)
    S = len(ws)
    n = [x.n for x in ws]
    N = [x.N for x in ws]
    T = max(N)
    Xd = [datagen.snapshots_torch(x, "cuda")[0] for x in ws]
    ptr = np.zeros((T, S), dtype=np.int64)
    for s, X in enumerate(Xd):
        ptr[:N[s], s] = X.data_ptr() + X.stride(0) * X.element_size() * np.arange(N[s], dtype=np.int64)
    dptr = torch.from_numpy(ptr).cuda()
    bt = FOABatch(n, N, prec="f32", form="one_reduction")
    for k in range(T):
        bt.push_ptrs(dptr[k], F.FOA_F32)
    q, status = bt.sync()
    assert np.all(q == np.array(N)) and np.all(status == 0)
    pick = set()
    for bkt in range(5):
        idx = [s for s in range(S) if _bucket(N[s] - 1) == bkt]
        if idx:
            pick.update({min(idx, key=lambda s: N[s]), max(idx, key=lambda s: N[s]),
                         max(idx, key=lambda s: n[s]), min(idx, key=lambda s: n[s])})
    pick.update({int(np.argmax(n)), int(np.argmin(n))})
    worst = dict(orth=0.0, eH=0.0, eig=0.0)
    for s in sorted(pick):
        st = oracle.foa_batch(np.asfortranarray(Xd[s].double().cpu().numpy().T))
        view = bt.view(s)
        H, B, qv, m = F.foa_get_state(view)
        assert qv == st.q == N[s]
        V = torch.empty((qv, n[s]), dtype=torch.float64, device="cuda")
        F.foa_copy_basis(view, V, n[s], F.FOA_F64, qv)
        orth = np.linalg.norm(np.eye(qv) - (V @ V.T).cpu().numpy(), 2) / (10 * np.sqrt(qv) * EPS32)
        sig = PB.svals(st.beta[:m, :m])
        kap = sig[0] / sig[-1]
        eH = np.linalg.norm(H[:m, :m] - st.H[:m, :m], 2) / np.linalg.norm(st.H[:m, :m], 2) / (10 * EPS32 * kap)
        r = oracle.truncation_rank(sig, st.q, "f32")
        kr = PB.kappa_r(sig, r)
        _, T_o, _ = PB.truncated_projection(st.H[:m, :m], st.beta[:m, :m], r)
        F.foa_truncate(view, -1.0, r)
        lam_g, _ = F.foa_indicators(view, m)
        lam_o, Z, Yn, cond = PB.eig_condition(T_o)
        full = np.concatenate([lam_g, lam_g[lam_g.imag > 0].conj()])
        ratio, err, _ = PB.eig_gate(full, lam_o, cond, EPS32, kr)
        announce(f"stream {s}: n={n[s]} N={N[s]} bucket={_bucket(N[s] - 1)} orth/bound={orth:.2e} "
                 f"relH/bound={eH:.2e} r={r} kappa_r={kr:.1e} eig/bound={ratio:.2e}")
        assert PB.C * EPS32 * kr < 1.0
        for k, v in (("orth", orth), ("eH", eH), ("eig", ratio)):
            worst[k] = max(worst[k], v)
        del V
    announce(f"{len(pick)} streams checked; worst err/bound: {worst}")
    assert max(worst.values()) <= 1.0
    bt.close()


def test_flush_midway_then_continue():
    """foa_batch_flush after 13 steps finishes every stream's pending columns
    without waiting; the pushes after it continue the streams: against the
    one-reduction oracle that flushes at the same point (FP64 basis)."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    w = datagen.get_workload("noisy_2p20x200")
    Xs = [np.asfortranarray(datagen.snapshots_numpy(w.with_n(n).with_N(N), dtype="float64")[0])
          for n, N in ((2000, 40), (9001, 25), (70, 33))]
    S = len(Xs)
    Xd = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    T = max(X.shape[1] for X in Xs)
    bt = FOABatch([X.shape[0] for X in Xs], [X.shape[1] for X in Xs], prec="f64", form="one_reduction")
    ptr = np.zeros((T, S), dtype=np.int64)
    for s in range(S):
        for t in range(Xs[s].shape[1]):
            ptr[t, s] = Xd[s][t].data_ptr()
    dptr = torch.from_numpy(ptr).cuda()
    for t in range(T):
        if t == 13:
            bt.flush()
        bt.push_ptrs(dptr[t], F.FOA_F64)
    q, st = bt.sync()
    for s, X in enumerate(Xs):
        ref = LS.init(X.shape[0], X.shape[1])
        for t in range(X.shape[1]):
            if t == 13:
                LS.flush(ref)
            LS.push(ref, np.ascontiguousarray(X[:, t]))
        LS.flush(ref)
        H, B, qv, m = F.foa_get_state(bt.view(s))
        assert qv == ref.q == X.shape[1] and st[s] == 0
        kap = kappa_of(ref.beta[:m, :m])
        eH, eB = rel(H[:qv, :m], ref.H[:qv, :m]), rel(B[:qv, :qv], ref.beta[:qv, :qv])
        announce(f"stream {s}: q={qv} kappa={kap:.1e} relH={eH:.1e} relB={eB:.1e}")
        assert max(eH, eB) <= 10 * qv * EPS64 * kap
    bt.close()


def test_shared_table_bitwise_and_reset_replay(tmp_path):
    """Two one-reduction batches with the same launch configuration (the second
    reads the first's entry in the tuning table, key with "/form1") give
    bitwise-equal H_bar, beta and basis; a reset followed by the same pushes
    replays the captured step graphs and reproduces the first run bitwise."""
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOABatch

    Xs = [X.astype(np.float32) for X in _mixed()[1:5]]
    S = len(Xs)
    n = [X.shape[0] for X in Xs]
    N = [X.shape[1] for X in Xs]
    Xd = [torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in Xs]
    T = max(N)
    ptr = np.zeros((T, S), dtype=np.int64)
    for s in range(S):
        for t in range(N[s]):
            ptr[t, s] = Xd[s][t].data_ptr()
    dptr = torch.from_numpy(ptr).cuda()
    table = str(tmp_path / "tune.json")

    def run(bt):
        for t in range(T):
            bt.push_ptrs(dptr[t], F.FOA_F32)
        q, st = bt.sync()
        out = []
        for s in range(S):
            v = bt.view(s)
            H, B, qv, m = F.foa_get_state(v)
            V = torch.empty((qv, n[s]), dtype=torch.float64, device="cuda")
            F.foa_copy_basis(v, V, n[s], F.FOA_F64, qv)
            out.append((qv, H, B, V.cpu().numpy()))
        return q, st, out

    a = FOABatch(n, N, prec="f32", form="one_reduction", tune_table=table)
    qa, sa, ra = run(a)
    b = FOABatch(n, N, prec="f32", form="one_reduction", tune_table=table)
    qb, sb, rb = run(b)
    a.reset()
    qc, sc, rc = run(a)
    assert np.array_equal(qa, np.array(N)) and np.all(sa == 0)
    for s in range(S):
        for other in (rb[s], rc[s]):
            assert other[0] == ra[s][0]
            for x, y in zip(ra[s][1:], other[1:]):
                assert np.array_equal(x, y), s
    announce(f"{S} streams: shared table and reset replay bitwise equal")
    a.close()
    b.close()
