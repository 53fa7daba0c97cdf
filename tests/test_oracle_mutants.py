"""Plant plausible mistakes in the oracle (on the CPU) and require that at
least one pin fails for each: evidence that the pins would catch a dropped
term, a wrong sign or index, or a transposed operand.

Not listed: dropping the Hessenberg correction h += s.  After one classical Gram-Schmidt
pass the correction s = V^T w is of rounding size (||s|| ~ eps ||w||), so that
mutant changes H only at the level of ordinary rounding, which no
mathematical pin can separate from a correct run (an equivalent mutant)."""

import types

import numpy as np
import pytest

import oracle
import oracle.dmd as odmd
import oracle.foa as ofoa
import pins


def _cgs_no_reorth(V, w, j):
    h = V[:, :j].T @ w
    w = w - V[:, :j] @ h
    return h, w


def _cgs_sign(V, w, j):
    h = V[:, :j].T @ w
    w = w + V[:, :j] @ h
    s = V[:, :j].T @ w
    h = h + s
    w = w - V[:, :j] @ s
    return h, w


def _beta_partial_shifted(H, beta, j):
    beta[0, j] = H[0, 0:j - 1] @ beta[0:j - 1, j - 1]
    for i in range(2, j + 1):
        beta[i - 1, j] = H[i - 1, i - 1:j - 1] @ beta[i - 1:j - 1, j - 1]


def _beta_partial_transposed(H, beta, j):
    beta[0, j] = H[0:j - 1, 0] @ beta[0:j - 1, j - 1]
    for i in range(2, j + 1):
        beta[i - 1, j] = H[i - 2:j - 1, i - 1] @ beta[i - 2:j - 1, j - 1]


def _beta_complete_short(H, beta, j):
    for i in range(1, j + 1):
        beta[i - 1, j] = beta[i - 1, j] + H[i - 1, j - 1] * beta[j - 1, j - 1]


def _form_w_wrong_diag(V, beta, psi, j):
    return (psi - V[:, :j] @ beta[:j, j]) / beta[0, 0]


def _form_w_wrong_col(V, beta, psi, j):
    return (psi - V[:, :j] @ beta[:j, j - 1]) / beta[j - 1, j - 1]


FOA_MUTANTS = {
    "cgs_without_reorthogonalisation": ("_cgs2", _cgs_no_reorth),
    "cgs_sign_error_step11": ("_cgs2", _cgs_sign),
    "beta_partial_index_shift": ("_beta_partial", _beta_partial_shifted),
    "beta_partial_transposed_H": ("_beta_partial", _beta_partial_transposed),
    "beta_complete_drops_diag": ("_beta_complete", _beta_complete_short),
    "form_w_wrong_diagonal": ("_form_w", _form_w_wrong_diag),
    "form_w_wrong_beta_column": ("_form_w", _form_w_wrong_col),
}


@pytest.mark.parametrize("name", sorted(FOA_MUTANTS))
def test_foa_mutant_is_caught(name, monkeypatch):
    attr, fn = FOA_MUTANTS[name]
    monkeypatch.setattr(ofoa, attr, fn)
    res = pins.run_all(oracle)
    failed = [k for k, (ok, _) in res.items() if not ok]
    assert failed, f"mutant {name} passed every pin"


def _ns(**over):
    ns = types.SimpleNamespace(**{k: getattr(oracle, k) for k in oracle.__all__})
    for k, v in over.items():
        setattr(ns, k, v)
    return ns


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


DMD_MUTANTS = {
    "indicator_uses_first_row": dict(dmd_untruncated=_dmd_wrong_indicator_row),
    "coefficients_wrong_rhs": dict(dmd_untruncated=_dmd_wrong_coef_rhs),
    "truncation_right_singular_vectors": dict(dmd_truncated=_dmd_trunc_right_vectors),
    "eig_of_transposed_projection": dict(dmd_untruncated=_dmd_transposed_H),
}


@pytest.mark.parametrize("name", sorted(DMD_MUTANTS))
def test_dmd_mutant_is_caught(name):
    res = pins.run_all(_ns(**DMD_MUTANTS[name]))
    failed = [k for k, (ok, _) in res.items() if not ok]
    assert failed, f"mutant {name} passed every pin"
