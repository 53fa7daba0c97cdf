"""The truncated FP32-vs-FP64 gate that bench.py reports (truncated_gate):
it passes on a run whose truncated eigenvalues are those of the reference
run, and fails once one eigenvalue moves past its bound, so the figure in the
benchmark line is a gate that can fail (Section 3.2.2, the truncated
backward-error bound).  CPU only: both runs are the oracle's."""

import numpy as np

import bench
import datagen
import oracle
import parity_bounds as PB


def _runs():
    w = datagen.get_workload("noisy_2p24x500").with_n(4096).with_N(80)
    X, _, _ = datagen.snapshots_numpy(w, dtype="float64")
    st = oracle.foa_batch(X)
    m = oracle.projected_size(st)
    sig = PB.svals(st.beta[:m, :m])
    r = oracle.truncation_rank(sig, st.q, "f32")
    lam = oracle.dmd_truncated(st, r)["lam"]
    ref = dict(beta=st.beta, H=st.H, m=m, r_trunc=r)
    run = dict(r_trunc=r, lam_trunc=lam[lam.imag >= 0])
    return run, ref, sig


def test_gate_passes_on_the_reference_eigenvalues_and_binds():
    run, ref, sig = _runs()
    g = bench.truncated_gate(run, ref)
    r = run["r_trunc"]
    assert 1 <= r < ref["m"]
    assert g["rank"] == g["rank_f64_run"] == r
    assert abs(g["kappa_r"] - sig[0] / sig[r - 1]) <= 1e-12 * g["kappa_r"]
    assert g["bound_10_eps32_kappa_r"] < 1.0          # the gate binds at this rank
    assert g["within_bound"] and g["max_err_over_bound"] < 1e-3
    assert g["eigenvalues"] == r


def test_gate_fails_when_one_eigenvalue_moves_past_its_bound():
    """A move of a tenth of the smallest per-eigenvalue bound passes; a move
    of twice the largest one fails."""
    run, ref, _ = _runs()
    g = bench.truncated_gate(run, ref)
    m, r = ref["m"], run["r_trunc"]
    _, T, _ = PB.truncated_projection(ref["H"][:m, :m], ref["beta"][:m, :m], r)
    cond = PB.eig_condition(T)[3]
    unit = g["bound_10_eps32_kappa_r"]                  # 10 eps32 kappa_r; bound_i = unit * max(1, cond_i)
    lam = run["lam_trunc"]
    k = int(np.argmin(np.abs(lam.imag)))
    small = lam.copy()
    small[k] += 0.1 * unit
    ok = bench.truncated_gate(dict(run, lam_trunc=small), ref)
    assert ok["within_bound"] and 0.05 < ok["max_err_over_bound"] <= 0.1 + 1e-6
    big = lam.copy()
    big[k] += 2.0 * unit * max(1.0, float(np.max(cond)))
    bad = bench.truncated_gate(dict(run, lam_trunc=big), ref)
    assert not bad["within_bound"]
    assert bad["max_err_over_bound"] > 1.0
