"""Helpers for the GPU tests: run the HIP path through the C ABI and compare
with the CPU oracle on the same seeded inputs."""

import sys

import numpy as np

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23


def announce(*parts):
    """Name the case on stderr before a GPU step (survives a lost box)."""
    sys.stderr.write("[gpu case] " + " ".join(str(p) for p in parts) + "\n")
    sys.stderr.flush()


def run_gpu(X, prec="f64", tol=-1.0, snap_dtype=None, options=None, n_max=None, block=False, ws_fill=0xFF,
            form="cgs2", blocked=False):
    """Push the columns of X (n x N NumPy) through the library; returns dict.
    block: one foa_push_block call (the snapshots taken one at a time);
    blocked: the blocked form (foa_push_blocked, blocks of 4 snapshots)."""
    import torch

    from paper_1805_05821_amd.stream import FOAStream

    n, N = X.shape
    dt = snap_dtype or (torch.float64 if X.dtype == np.float64 else torch.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to(device="cuda", dtype=dt)
    # the workspace starts as NaN bytes: nothing may depend on its initial content
    s = FOAStream(n, n_max or N, prec=prec, breakdown_tol=tol, ws_fill=ws_fill, form=form)
    for k, v in (options or {}).items():
        s.set_option(k, v)
    if blocked:
        s.push_blocked(Xd)
    elif block:
        s.push_block(Xd)
    else:
        s.push_all(Xd)
    status, q = s.sync()
    H, B, q, m = s.state()
    V = s.basis(q).cpu().numpy().T if q > 0 else np.zeros((n, 0))
    out = dict(status=status, q=q, m=m, H=H, beta=B, V=V, stream=s)
    return out


def kappa_of(beta_m):
    s = np.linalg.svd(beta_m, compute_uv=False)
    return float(s[0] / s[-1])


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
