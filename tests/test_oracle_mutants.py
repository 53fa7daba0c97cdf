"""Plant plausible mistakes in the oracle (on the CPU) and require that at
least one pin fails for each, by comparing values (a pin that fails only
because the mutated oracle raised does not count): evidence that the pins
would catch a dropped term, a wrong sign or index, or a transposed operand.

Not listed: dropping the coefficients of the second Gram-Schmidt pass from
the Hessenberg column.  After one classical pass those coefficients are of
rounding size (||s|| ~ eps ||w||), so that mutant changes H only at the level
of ordinary rounding, which no mathematical pin can separate from a correct
run (an equivalent mutant)."""

import types

import numpy as np
import pytest

import oracle
import oracle.dmd as odmd
import oracle.foa as ofoa
import pins


def _failed_by_value(res):
    return [k for k, (ok, _, raised) in res.items() if not ok and not raised]


# ---- mistakes in the FOA iteration (module oracle.foa) ----------------------

def _cgs_single_pass(V, w, j):
    Vj = V[:, :j]
    h = Vj.T @ w
    return h, w - Vj @ h


def _cgs_sign(V, w, j):
    Vj = V[:, :j]
    h = np.zeros(j)
    for p in range(2):
        s = Vj.T @ w
        w = w + Vj @ s if p == 0 else w - Vj @ s
        h = h + s
    return h, w


def _cgs_keeps_last_pass_only(V, w, j):
    Vj = V[:, :j]
    for _ in range(2):
        s = Vj.T @ w
        w = w - Vj @ s
    return s, w


def _partial_beta_row_shift(H, beta, j):
    return H[1:j + 1, :j - 1] @ beta[:j - 1, j - 1]


def _partial_beta_transposed(H, beta, j):
    return H[:j - 1, :j].T @ beta[:j - 1, j - 1]


def _partial_beta_wrong_column(H, beta, j):
    return H[:j, :j - 1] @ beta[:j - 1, j - 2]


def _arnoldi_vector_sign(V, b, bjj, psi, j):
    return (psi + V[:, :j] @ b) / bjj


def _arnoldi_vector_unscaled(V, b, bjj, psi, j):
    return psi - V[:, :j] @ b


def _arnoldi_vector_drops_last(V, b, bjj, psi, j):
    return (psi - V[:, :j - 1] @ b[:j - 1]) / bjj


def _completed_beta_no_diag(b, hcol, bjj):
    col = np.zeros(hcol.shape[0])
    col[:b.shape[0]] = b
    col[:-1] += hcol[:-1] * bjj
    return col


def _completed_beta_unscaled(b, hcol, bjj):
    col = np.zeros(hcol.shape[0])
    col[:b.shape[0]] = b
    return col + hcol


FOA_MUTANTS = {
    "cgs_without_reorthogonalisation": ("_cgs2", _cgs_single_pass),
    "cgs_sign_error_first_pass": ("_cgs2", _cgs_sign),
    "cgs_keeps_second_pass_coefficients_only": ("_cgs2", _cgs_keeps_last_pass_only),
    "partial_beta_row_shift": ("_partial_beta_column", _partial_beta_row_shift),
    "partial_beta_transposed_H": ("_partial_beta_column", _partial_beta_transposed),
    "partial_beta_wrong_beta_column": ("_partial_beta_column", _partial_beta_wrong_column),
    "arnoldi_vector_sign": ("_arnoldi_vector", _arnoldi_vector_sign),
    "arnoldi_vector_not_divided_by_beta_jj": ("_arnoldi_vector", _arnoldi_vector_unscaled),
    "arnoldi_vector_drops_last_basis_vector": ("_arnoldi_vector", _arnoldi_vector_drops_last),
    "completed_beta_drops_diagonal": ("_completed_beta_column", _completed_beta_no_diag),
    "completed_beta_not_scaled_by_beta_jj": ("_completed_beta_column", _completed_beta_unscaled),
}


@pytest.mark.parametrize("name", sorted(FOA_MUTANTS))
def test_foa_mutant_is_caught(name, monkeypatch):
    attr, fn = FOA_MUTANTS[name]
    assert hasattr(ofoa, attr), attr
    monkeypatch.setattr(ofoa, attr, fn)
    failed = _failed_by_value(pins.run_all(oracle))
    assert failed, f"mutant {name} passed every pin"


# ---- mistakes in the post-processing (replaced in a namespace) ---------------

def _ns(**over):
    ns = types.SimpleNamespace(**{k: getattr(oracle, k) for k in oracle.__all__})
    for k, v in over.items():
        assert hasattr(ns, k), k
        setattr(ns, k, v)
    return ns


def test_unmutated_oracle_passes_every_pin():
    """Control: without a mutation every pin passes, both on the package and
    on the namespace the post-processing mutants are planted in, so a caught
    mutant is caught by its mistake."""
    for O in (oracle, _ns()):
        res = pins.run_all(O)
        bad = {k: d for k, (ok, d, _) in res.items() if not ok}
        assert not bad, bad


def _dmd_wrong_indicator_row(st):
    res = odmd.dmd_untruncated(st)
    m = res["m"]
    hlast = 0.0 if st.status == "invariant" else float(st.H[m, m - 1])
    res["indicators"] = abs(hlast) * np.abs(res["Z"][0, :])
    return res


def _dmd_wrong_coef_rhs(st):
    res = odmd.dmd_untruncated(st)
    m = res["m"]
    rhs = np.zeros(m, dtype=np.complex128)
    rhs[0] = st.beta[1, 1]
    res["coef"] = np.linalg.solve(res["Z"], rhs)
    res["order"] = odmd._order(res["lam"], res["coef"])
    return res


def _dmd_trunc_right_vectors(st, r):
    m = odmd.projected_size(st)
    Hm = st.H[:m, :m]
    U, S, Wt = np.linalg.svd(st.beta[:m, :m])
    Wr = Wt.T[:, :r]
    lam, Z = np.linalg.eig(Wr.T @ Hm @ Wr)
    return {"m": m, "r": r, "lam": lam, "Z": Z, "B": Wr @ Z, "indicators": np.zeros(r),
            "coef": np.ones(r), "order": np.arange(r)}


def _dmd_transposed_H(st):
    class S:
        pass
    s2 = S()
    s2.__dict__.update(st.__dict__)
    s2.H = st.H.T.copy()
    return odmd.dmd_untruncated(s2)


def _trunc_indicators(st, res, projector=True, h_row=True):
    m, r = res["m"], res["r"]
    Hm = st.H[:m, :m]
    Ur = res["Ur"]
    hlast = float(st.H[m, m - 1])
    out = np.empty(r)
    for i in range(r):
        y = Ur @ res["Z"][:, i]
        inside = Hm @ y
        if projector:
            inside = inside - Ur @ (Ur.T @ inside)
        along = hlast * y[m - 1] if h_row else 0.0
        out[i] = np.sqrt(np.linalg.norm(inside) ** 2 + abs(along) ** 2)
    return out


def _trunc_no_projector(st, r):
    res = odmd.dmd_truncated(st, r)
    res["indicators"] = _trunc_indicators(st, res, projector=False)
    return res


def _trunc_no_h_row(st, r):
    res = odmd.dmd_truncated(st, r)
    res["indicators"] = _trunc_indicators(st, res, h_row=False)
    return res


def _trunc_coef_doubled(st, r):
    res = odmd.dmd_truncated(st, r)
    res["coef"] = 2.0 * res["coef"]
    return res


def _trunc_coef_exrecon_rhs(st, r):
    res = odmd.dmd_truncated(st, r)
    rhs = np.zeros(r, dtype=np.complex128)
    rhs[0] = st.beta[0, 0]
    res["coef"] = np.linalg.solve(res["Z"], rhs)
    res["order"] = odmd._order(res["lam"], res["coef"])
    return res


def _rank_unit_spacing(sigma, nsnap, storage="f64"):
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.size == 0:
        return 0
    eps = 2.0 ** -23 if storage == "f32" else 2.0 ** -52
    return int(np.count_nonzero(sigma > nsnap * eps))


def _rank_ignores_storage(sigma, nsnap, storage="f64"):
    return odmd.truncation_rank(sigma, nsnap, "f64")


def _rank_off_by_one(sigma, nsnap, storage="f64"):
    return odmd.truncation_rank(sigma, nsnap - 1, storage)


def _packed_swap_re_im(res, V):
    Phi, lams, kinds = odmd.packed_modes(res, V)
    Phi = Phi.copy()
    col = 0
    for k in kinds:
        if k == 1:
            Phi[:, [col, col + 1]] = Phi[:, [col + 1, col]]
            col += 2
        else:
            col += 1
    return Phi, lams, kinds


def _packed_lower_member(res, V):
    flipped = dict(res)
    flipped["lam"] = res["lam"].conj()
    return odmd.packed_modes(flipped, V)


def _packed_coef_conjugated(res):
    return odmd.packed_coefficients(res).conj()


DMD_MUTANTS = {
    "indicator_uses_first_row": dict(dmd_untruncated=_dmd_wrong_indicator_row),
    "coefficients_wrong_rhs": dict(dmd_untruncated=_dmd_wrong_coef_rhs),
    "truncation_right_singular_vectors": dict(dmd_truncated=_dmd_trunc_right_vectors),
    "eig_of_transposed_projection": dict(dmd_untruncated=_dmd_transposed_H),
    "truncated_indicator_without_projector": dict(dmd_truncated=_trunc_no_projector),
    "truncated_indicator_without_h_row": dict(dmd_truncated=_trunc_no_h_row),
    "truncated_coefficients_doubled": dict(dmd_truncated=_trunc_coef_doubled),
    "truncated_coefficients_untruncated_rhs": dict(dmd_truncated=_trunc_coef_exrecon_rhs),
    "rank_rule_spacing_at_one": dict(truncation_rank=_rank_unit_spacing),
    "rank_rule_ignores_storage_precision": dict(truncation_rank=_rank_ignores_storage),
    "rank_rule_off_by_one_snapshot_count": dict(truncation_rank=_rank_off_by_one),
    "packed_modes_re_im_swapped": dict(packed_modes=_packed_swap_re_im),
    "packed_modes_lower_pair_member": dict(packed_modes=_packed_lower_member),
    "packed_coefficients_conjugated": dict(packed_coefficients=_packed_coef_conjugated),
}


@pytest.mark.parametrize("name", sorted(DMD_MUTANTS))
def test_dmd_mutant_is_caught(name):
    failed = _failed_by_value(pins.run_all(_ns(**DMD_MUTANTS[name])))
    assert failed, f"mutant {name} passed every pin"
