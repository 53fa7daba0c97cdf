"""The seeded input generator: determinism, shapes, layouts and the
statistics each workload promises."""

import numpy as np

import datagen


def test_same_seed_same_bytes():
    w = datagen.get_workload("noisy_2p20x200").with_n(5000).with_N(17)
    a, la, ba = datagen.snapshots_numpy(w)
    b, lb, bb = datagen.snapshots_numpy(w)
    assert a.tobytes() == b.tobytes()
    assert np.array_equal(la, lb) and np.array_equal(ba, bb)


def test_layout_and_dtype():
    w = datagen.get_workload("noisy_2p24x500").with_n(3000).with_N(7)
    X, lam, b = datagen.snapshots_numpy(w)
    assert X.shape == (3000, 7) and X.dtype == np.float32 and X.flags["F_CONTIGUOUS"]
    assert lam.shape == (120,) and np.all(np.abs(lam) <= 1.0 + 1e-15)
    assert np.isclose(b[0], 1.0) and np.isclose(b[-1], 1e-7)


def test_exact_rank_properties():
    w = datagen.get_workload("exact_rank_4096x64")
    X, lam, b = datagen.snapshots_numpy(w)
    s = np.linalg.svd(X, compute_uv=False)
    assert s[19] / s[0] > 1e-6 and s[20] / s[0] < 1e-13
    s20 = np.linalg.svd(X[:, :20], compute_uv=False)
    assert s20[0] / s20[-1] <= 1e3
    full = np.concatenate([lam, lam.conj()])
    d = np.abs(full[:, None] - full[None, :]) + np.eye(20) * 9
    assert d.min() >= 1e-3


def test_noise_level():
    w = datagen.get_workload("noisy_2p20x200").with_n(1 << 16).with_N(5)
    lam, b, sub = datagen.mode_parameters(w)
    X, _, _ = datagen.snapshots_numpy(w)
    w0 = w.__class__(**{**w.__dict__, "noise": 0.0})
    X0, _, _ = datagen.snapshots_numpy(w0)
    rms = datagen.expected_rms(lam, b, w.n, w.N)
    meas = np.sqrt(((X - X0) ** 2).mean(axis=0))
    assert np.allclose(meas / (w.noise * rms), 1.0, atol=0.05)
    clean = np.sqrt((X0 ** 2).mean(axis=0))
    assert np.allclose(clean / rms, 1.0, atol=0.1)


def test_batched_streams_ranges():
    bw = datagen.get_workload("batched_256")
    ss = datagen.batched_streams(bw)
    assert len(ss) == 256
    for s in ss:
        assert bw.n_lo <= s.n <= bw.n_hi and bw.N_lo <= s.N <= bw.N_hi
        assert bw.pairs_lo <= s.pairs <= bw.pairs_hi
    assert ss[3] == datagen.batched_streams(bw)[3]
