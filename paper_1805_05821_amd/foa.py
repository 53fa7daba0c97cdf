"""Thin ctypes binding of libfoa.so (include/foa.h).

Functions keep the C names and only marshal arguments: device buffers are
torch tensors (or raw integer device addresses), host buffers are NumPy
arrays.  All computation happens in the HIP library; importing this module
fails loudly if the library has not been built.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfoa.so")

FOA_OK = 0
FOA_INVARIANT = 1
FOA_E_ARG = -1
FOA_E_CAPACITY = -2
FOA_E_STATE = -3
FOA_E_NONFINITE = -4
FOA_E_DEVICE = -5
FOA_E_NOMEM = -6
FOA_E_NUMERIC = -7
FOA_E_ZERO = -8

FOA_PREC_F64 = 0
FOA_PREC_F32 = 1
FOA_F32 = 0
FOA_F64 = 1
FOA_MAX_CAPACITY = 512
FOA_FORM_CGS2 = 0
FOA_FORM_ONE_REDUCTION = 1

EXPORTED = [
    "foa_workspace_bytes", "foa_init", "foa_push_snapshot", "foa_push_block", "foa_sync",
    "foa_get_state", "foa_copy_basis", "foa_copy_basis_rows", "foa_truncate", "foa_modes", "foa_indicators",
    "foa_reset", "foa_destroy", "foa_status_str", "foa_last_error", "foa_set_option", "foa_profile",
    "foa_profile_modes", "foa_next_column", "foa_block_workspace_bytes", "foa_push_blocked",
    "foa_push_blocked_static", "foa_set_form", "foa_flush", "foa_batch_set_form",
    "foa_batch_flush",
    "foa_batch_workspace_bytes", "foa_batch_init", "foa_batch_push", "foa_batch_sync",
    "foa_batch_view", "foa_batch_reset", "foa_batch_destroy",
]


class FOAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def _load():
    # torch ships its own HIP runtime under the same soname as the system one
    # (libamdhip64.so.7).  Load torch first so the library binds to that one
    # runtime: the streams and allocations it receives come from torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1805_05821_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P = c.c_void_p
    i32, i64, f64, sz = c.c_int32, c.c_int64, c.c_double, c.c_size_t
    sig = {
        "foa_workspace_bytes": [i64, i32, c.c_int, c.POINTER(sz)],
        "foa_init": [c.POINTER(P), i64, i32, c.c_int, P, sz, P, f64],
        "foa_push_snapshot": [P, P, c.c_int],
        "foa_push_block": [P, P, i64, i32, c.c_int],
        "foa_sync": [P, c.POINTER(i32)],
        "foa_get_state": [P, P, P, i32, c.POINTER(i32), c.POINTER(i32)],
        "foa_copy_basis": [P, P, i64, c.c_int, i32],
        "foa_copy_basis_rows": [P, i64, i64, P, i64, c.c_int, i32],
        "foa_truncate": [P, f64, i32, c.POINTER(i32), P],
        "foa_modes": [P, i32, P, P, P, P, P, i64, i32, c.c_int, c.POINTER(i32)],
        "foa_indicators": [P, i32, P, P, c.POINTER(i32)],
        "foa_reset": [P],
        "foa_destroy": [P],
        "foa_set_option": [P, c.c_char_p, i64],
        "foa_profile": [P, P],
        "foa_profile_modes": [P, P],
        "foa_next_column": [P, P],
        "foa_block_workspace_bytes": [ctypes.c_int64, ctypes.c_int32, ctypes.c_int, P],
        "foa_push_blocked": [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, P, ctypes.c_size_t],
        "foa_push_blocked_static": [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int],
        "foa_set_form": [P, c.c_int],
        "foa_batch_set_form": [P, c.c_int],
        "foa_flush": [P],
        "foa_batch_flush": [P],
        "foa_batch_workspace_bytes": [i32, P, P, c.c_int, c.POINTER(sz)],
        "foa_batch_init": [c.POINTER(P), i32, P, P, c.c_int, P, sz, P, f64, c.c_char_p],
        "foa_batch_push": [P, P, c.c_int],
        "foa_batch_sync": [P, P, P],
        "foa_batch_view": [P, i32, c.POINTER(P)],
        "foa_batch_reset": [P],
        "foa_batch_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c.c_int
    lib.foa_status_str.argtypes = [c.c_int]
    lib.foa_status_str.restype = c.c_char_p
    lib.foa_last_error.argtypes = [P]
    lib.foa_last_error.restype = c.c_char_p
    return lib


lib = _load()


def _addr(buf):
    """Device address of a torch tensor, or an int address, or None."""
    if buf is None:
        return None
    if isinstance(buf, int):
        return buf
    return buf.data_ptr()


def _host(arr):
    return None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def status_str(code):
    return lib.foa_status_str(code).decode()


def _check(code, ctx=None, ok=(FOA_OK,)):
    if code in ok:
        return code
    msg = status_str(code)
    if ctx is not None:
        detail = lib.foa_last_error(ctx).decode()
        if detail:
            msg = f"{msg}: {detail}"
    raise FOAError(code, msg)


# ---- functions with the C names --------------------------------------------

def foa_workspace_bytes(n, n_max, prec):
    out = ctypes.c_size_t()
    _check(lib.foa_workspace_bytes(int(n), int(n_max), int(prec), ctypes.byref(out)))
    return out.value


def foa_init(n, n_max, prec, workspace, ws_bytes=None, stream=None, breakdown_tol=-1.0):
    ctx = ctypes.c_void_p()
    nb = ws_bytes if ws_bytes is not None else workspace.numel() * workspace.element_size()
    _check(lib.foa_init(ctypes.byref(ctx), int(n), int(n_max), int(prec), _addr(workspace), int(nb),
                        _stream_handle(stream), float(breakdown_tol)))
    return ctx


def foa_push_snapshot(ctx, x, x_dtype=None):
    if x_dtype is None:
        x_dtype = FOA_F64 if str(x.dtype) == "torch.float64" else FOA_F32
    return _check(lib.foa_push_snapshot(ctx, _addr(x), int(x_dtype)), ctx)


def foa_push_block(ctx, X, ld, p, x_dtype):
    return _check(lib.foa_push_block(ctx, _addr(X), int(ld), int(p), int(x_dtype)), ctx)


def foa_sync(ctx):
    """Returns (status, q); status is FOA_OK, FOA_INVARIANT or raises."""
    q = ctypes.c_int32()
    st = lib.foa_sync(ctx, ctypes.byref(q))
    if st < 0 and st not in (FOA_E_NONFINITE, FOA_E_ZERO):
        _check(st, ctx)
    return st, q.value


def foa_get_state(ctx, ld=None):
    """Returns (Hbar (q+1) x m, beta, q, m) as NumPy float64 arrays."""
    q = ctypes.c_int32()
    m = ctypes.c_int32()
    _check(lib.foa_get_state(ctx, None, None, 1, ctypes.byref(q), ctypes.byref(m)), ctx)
    qq, mm = q.value, m.value
    ld = max(qq + 1, 1) if ld is None else ld
    H = np.zeros((max(mm, 1), ld), dtype=np.float64)      # column-major: H[col, row]
    B = np.zeros((qq + 1, ld), dtype=np.float64)
    _check(lib.foa_get_state(ctx, _host(H), _host(B), int(ld), ctypes.byref(q), ctypes.byref(m)), ctx)
    Hbar = H.T[: qq + 1, :mm].copy()
    beta = B.T[: qq + 1, : qq + 1].copy()
    return Hbar, beta, qq, mm


def foa_copy_basis(ctx, out, ld, dtype, ncols):
    return _check(lib.foa_copy_basis(ctx, _addr(out), int(ld), int(dtype), int(ncols)), ctx)


def foa_copy_basis_rows(ctx, r0, nrows, out, ld, dtype, ncols):
    return _check(lib.foa_copy_basis_rows(ctx, int(r0), int(nrows), _addr(out), int(ld), int(dtype), int(ncols)), ctx)


def foa_truncate(ctx, rel_tol=-1.0, r_force=0, m_hint=None):
    r = ctypes.c_int32()
    sig = np.zeros(FOA_MAX_CAPACITY + 1, dtype=np.float64)
    _check(lib.foa_truncate(ctx, float(rel_tol), int(r_force), ctypes.byref(r), _host(sig)), ctx)
    return r.value, sig


def foa_modes(ctx, m_max, phi=None, ld_phi=0, phi_cols=0, phi_dtype=FOA_F32):
    lam = np.zeros(2 * m_max, dtype=np.float64)
    kind = np.zeros(m_max, dtype=np.int8)
    amp = np.zeros(m_max, dtype=np.float64)
    err = np.zeros(m_max, dtype=np.float64)
    m = ctypes.c_int32()
    _check(lib.foa_modes(ctx, int(m_max), _host(lam), _host(kind), _host(amp), _host(err), _addr(phi),
                         int(ld_phi), int(phi_cols), int(phi_dtype), ctypes.byref(m)), ctx)
    k = m.value
    lam_c = lam[0:2 * k:2] + 1j * lam[1:2 * k:2]
    return lam_c, kind[:k].copy(), amp[:k].copy(), err[:k].copy()


def foa_indicators(ctx, m_max):
    lam = np.zeros(2 * m_max, dtype=np.float64)
    err = np.zeros(m_max, dtype=np.float64)
    m = ctypes.c_int32()
    _check(lib.foa_indicators(ctx, int(m_max), _host(lam), _host(err), ctypes.byref(m)), ctx)
    k = m.value
    return lam[0:2 * k:2] + 1j * lam[1:2 * k:2], err[:k].copy()


def foa_reset(ctx):
    return _check(lib.foa_reset(ctx), ctx)


def foa_destroy(ctx):
    return _check(lib.foa_destroy(ctx))


def foa_set_option(ctx, key, value):
    return _check(lib.foa_set_option(ctx, key.encode(), int(value)), ctx)


def foa_profile(ctx):
    """(launches, total_ms, algorithmic_bytes) of the row passes since the last call."""
    out = np.zeros(3, dtype=np.float64)
    _check(lib.foa_profile(ctx, _host(out)), ctx)
    return int(out[0]), float(out[1]), float(out[2])


def foa_profile_modes(ctx):
    """(launches, total_ms, algorithmic_flops) of the mode reconstruction since the last call."""
    out = np.zeros(3, dtype=np.float64)
    _check(lib.foa_profile_modes(ctx, _host(out)), ctx)
    return int(out[0]), float(out[1]), float(out[2])


def foa_block_workspace_bytes(n, n_max, prec):
    out = ctypes.c_size_t()
    _check(lib.foa_block_workspace_bytes(int(n), int(n_max), int(prec), ctypes.byref(out)))
    return int(out.value)


def foa_push_blocked(ctx, X, ld, p, x_dtype, bws, bws_bytes):
    return _check(lib.foa_push_blocked(ctx, _addr(X), int(ld), int(p), int(x_dtype), _addr(bws),
                                       int(bws_bytes)), ctx)


def foa_set_form(ctx, form):
    return _check(lib.foa_set_form(ctx, int(form)), ctx)


def foa_batch_set_form(b, form):
    return _check(lib.foa_batch_set_form(b, int(form)))


def foa_flush(ctx):
    return _check(lib.foa_flush(ctx), ctx)


def foa_batch_flush(b):
    return _check(lib.foa_batch_flush(b))


def foa_push_blocked_static(ctx, X, ld, p, x_dtype):
    return _check(lib.foa_push_blocked_static(ctx, _addr(X), int(ld), int(p), int(x_dtype)), ctx)


FOA_BLOCK_STATIC_BYTES = 64 << 20


def foa_next_column(ctx):
    """Device address of the in-place snapshot buffer (n FP64 entries)."""
    out = ctypes.c_void_p()
    _check(lib.foa_next_column(ctx, ctypes.byref(out)), ctx)
    return int(out.value)


def foa_last_error(ctx):
    return lib.foa_last_error(ctx).decode()


# ---- batched form -------------------------------------------------------------

def foa_batch_workspace_bytes(n_list, nmax_list, prec):
    n = np.ascontiguousarray(n_list, dtype=np.int64)
    m = np.ascontiguousarray(nmax_list, dtype=np.int32)
    out = ctypes.c_size_t()
    _check(lib.foa_batch_workspace_bytes(len(n), _host(n), _host(m), int(prec), ctypes.byref(out)))
    return out.value


def foa_batch_init(n_list, nmax_list, prec, workspace, stream=None, breakdown_tol=-1.0, tune_table=None):
    n = np.ascontiguousarray(n_list, dtype=np.int64)
    m = np.ascontiguousarray(nmax_list, dtype=np.int32)
    b = ctypes.c_void_p()
    nb = workspace.numel() * workspace.element_size()
    _check(lib.foa_batch_init(ctypes.byref(b), len(n), _host(n), _host(m), int(prec), _addr(workspace), int(nb),
                              _stream_handle(stream), float(breakdown_tol),
                              None if tune_table is None else tune_table.encode()))
    return b


def foa_batch_push(b, d_ptrs, x_dtype):
    return _check(lib.foa_batch_push(b, _addr(d_ptrs), int(x_dtype)))


def foa_batch_sync(b, S):
    q = np.zeros(S, dtype=np.int32)
    st = np.zeros(S, dtype=np.int32)
    _check(lib.foa_batch_sync(b, _host(q), _host(st)))
    return q, st


def foa_batch_view(b, s):
    v = ctypes.c_void_p()
    _check(lib.foa_batch_view(b, int(s), ctypes.byref(v)))
    return v


def foa_batch_reset(b):
    return _check(lib.foa_batch_reset(b))


def foa_batch_destroy(b):
    return _check(lib.foa_batch_destroy(b))
