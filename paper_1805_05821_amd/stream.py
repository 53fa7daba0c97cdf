"""Convenience wrapper over the C ABI for one FOA stream: allocates the
workspace as a torch uint8 tensor on the device and forwards every call to
the functions of ``foa.py`` (argument marshalling only)."""

import numpy as np

from . import foa as F


class FOAStream:
    def __init__(self, n, n_max, prec="f64", device="cuda", stream=None, breakdown_tol=-1.0, ws_fill=None,
                 form="cgs2"):
        import torch

        self.n = int(n)
        self.n_max = int(n_max)
        self.prec = F.FOA_PREC_F64 if prec in ("f64", F.FOA_PREC_F64) else F.FOA_PREC_F32
        nbytes = F.foa_workspace_bytes(self.n, self.n_max, self.prec)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        if ws_fill is not None:  # tests: start from a workspace full of a given byte
            self.ws.fill_(int(ws_fill))
        self.stream = stream
        self.ctx = F.foa_init(self.n, self.n_max, self.prec, self.ws, nbytes, stream, breakdown_tol)
        if form != "cgs2":
            F.foa_set_form(self.ctx, F.FOA_FORM_ONE_REDUCTION if form == "one_reduction" else form)

    # pushes ---------------------------------------------------------------
    def push(self, x):
        return F.foa_push_snapshot(self.ctx, x)

    def push_all(self, X):
        """X: (N, n) tensor, one snapshot per row."""
        for k in range(X.shape[0]):
            F.foa_push_snapshot(self.ctx, X[k])

    def push_blocked(self, X):
        """X: (p, n) tensor; blocked form (foa_push_blocked), blocks of 4
        snapshots.  The block workspace is allocated on first use."""
        import torch

        if getattr(self, "bws", None) is None:
            nb = F.foa_block_workspace_bytes(self.n, self.n_max, self.prec)
            self.bws = torch.empty(nb, dtype=torch.uint8, device=self.ws.device)
        dt = F.FOA_F64 if str(X.dtype) == "torch.float64" else F.FOA_F32
        return F.foa_push_blocked(self.ctx, X, X.stride(0), X.shape[0], dt, self.bws, self.bws.numel())

    def push_blocked_static(self, X):
        """As push_blocked, with the library's static block workspace
        (foa_push_blocked_static: nothing is allocated)."""
        dt = F.FOA_F64 if str(X.dtype) == "torch.float64" else F.FOA_F32
        return F.foa_push_blocked_static(self.ctx, X, X.stride(0), X.shape[0], dt)

    def push_block(self, X):
        dt = F.FOA_F64 if str(X.dtype) == "torch.float64" else F.FOA_F32
        return F.foa_push_block(self.ctx, X, X.stride(0), X.shape[0], dt)

    def flush(self):
        """One-reduction form: finish the pending columns (stream-ordered)."""
        return F.foa_flush(self.ctx)

    # queries --------------------------------------------------------------
    def sync(self):
        return F.foa_sync(self.ctx)

    def state(self):
        return F.foa_get_state(self.ctx)

    def basis(self, ncols=None, dtype=None):
        """First ncols Arnoldi vectors as an (ncols, n) tensor (row k = v_{k+1})."""
        import torch

        if ncols is None:
            _, ncols = self.sync()
        dtype = dtype or torch.float64
        out = torch.empty((max(ncols, 1), self.n), dtype=dtype, device=self.ws.device)
        F.foa_copy_basis(self.ctx, out, self.n, F.FOA_F64 if dtype == torch.float64 else F.FOA_F32, ncols)
        return out[:ncols]

    def basis_rows(self, r0, nrows, ncols, dtype=None):
        """Rows [r0, r0+nrows) of v_1..v_ncols as an (ncols, nrows) tensor."""
        import torch

        dtype = dtype or torch.float64
        out = torch.empty((max(ncols, 1), max(nrows, 1)), dtype=dtype, device=self.ws.device)
        F.foa_copy_basis_rows(self.ctx, r0, nrows, out, max(nrows, 1),
                              F.FOA_F64 if dtype == torch.float64 else F.FOA_F32, ncols)
        return out[:ncols, :nrows]

    def truncate(self, rel_tol=-1.0, r_force=0):
        return F.foa_truncate(self.ctx, rel_tol, r_force)

    def modes(self, m_max=None, phi=None, phi_cols=0, phi_dtype=F.FOA_F32):
        m_max = m_max or self.n_max
        ld = self.n if phi is not None else 0
        return F.foa_modes(self.ctx, m_max, phi, ld, phi_cols, phi_dtype)

    def indicators(self, m_max=None):
        return F.foa_indicators(self.ctx, m_max or self.n_max)

    def set_option(self, key, value):
        return F.foa_set_option(self.ctx, key, value)

    def reset(self):
        return F.foa_reset(self.ctx)

    def close(self):
        if self.ctx is not None:
            F.foa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hbar_beta_numpy(stream):
    H, B, q, m = stream.state()
    return np.asarray(H), np.asarray(B), q, m


class FOABatch:
    """Many independent streams in one workspace, advanced together
    (foa_batch_* of the C ABI)."""

    def __init__(self, n_list, nmax_list, prec="f32", device="cuda", stream=None, breakdown_tol=-1.0,
                 tune_table=None, ws_fill=None, form="cgs2"):
        import torch

        self.n = [int(v) for v in n_list]
        self.n_max = [int(v) for v in nmax_list]
        self.S = len(self.n)
        self.prec = F.FOA_PREC_F64 if prec in ("f64", F.FOA_PREC_F64) else F.FOA_PREC_F32
        nbytes = F.foa_batch_workspace_bytes(self.n, self.n_max, self.prec)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        if ws_fill is not None:
            self.ws.fill_(int(ws_fill))
        self.device = device
        self.b = F.foa_batch_init(self.n, self.n_max, self.prec, self.ws, stream, breakdown_tol, tune_table)
        if form != "cgs2":
            F.foa_batch_set_form(self.b, F.FOA_FORM_ONE_REDUCTION if form == "one_reduction" else form)
        self._ptrs = torch.zeros(self.S, dtype=torch.int64, device=device)

    def push(self, xs, x_dtype=None):
        """xs: list of S device tensors (or None for an idle stream)."""
        import torch

        host = [0 if x is None else x.data_ptr() for x in xs]
        if x_dtype is None:
            x0 = next((x for x in xs if x is not None), None)
            x_dtype = F.FOA_F64 if x0 is not None and x0.dtype == torch.float64 else F.FOA_F32
        self._ptrs.copy_(torch.tensor(host, dtype=torch.int64), non_blocking=False)
        return F.foa_batch_push(self.b, self._ptrs, x_dtype)

    def push_ptrs(self, d_ptrs, x_dtype):
        """d_ptrs: device int64 tensor of S snapshot addresses (0 = idle)."""
        return F.foa_batch_push(self.b, d_ptrs, x_dtype)

    def reset(self):
        return F.foa_batch_reset(self.b)

    def flush(self):
        """One-reduction form: enqueue the steps that finish the pending columns."""
        return F.foa_batch_flush(self.b)

    def sync(self):
        return F.foa_batch_sync(self.b, self.S)

    def view(self, s):
        return F.foa_batch_view(self.b, s)

    def close(self):
        if self.b is not None:
            F.foa_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
