"""Seeded snapshot sequences following the snapshot model of Section 2.

Recipe (identical for the NumPy and the torch backends, only the random
streams differ):

* lambda_m = exp(sigma_m + i omega_m) with sigma_m ~ U[-0.05, 0] and
  omega_m ~ U[0.1, pi] (time step 1), m = 1..M, drawn from PCG64(seed, sub_seed).
* b_m ~ N(0, 1) when no amplitude spread is given, else the real positive
  geometric sequence |b_m| = 10^(-d (m-1)/(M-1)).
* phi_m = g_m / sqrt(2 n) with g_m a complex standard Gaussian vector, so that
  E ||phi_m||_2 = 1.
* x_j = Re(sum_m b_m phi_m lambda_m^(j-1)) + a * rms_j * e_j, j = 1..N, where
  e_j is i.i.d. N(0, 1) and rms_j = sqrt(sum_m b_m^2 |lambda_m|^(2(j-1)) / (2n))
  is the expected root-mean-square entry of the clean snapshot.

Rows are generated in blocks of ``BLOCK_ROWS`` with one random stream per
block, so large inputs never need more than one block of temporaries.

Layouts: NumPy returns an (n, N) Fortran-ordered array (each snapshot is a
contiguous column); torch returns an (N, n) row-major tensor (each snapshot is
a contiguous row).  Both hold the same logical matrix X = [x_1 ... x_N].
"""

import math

import numpy as np

BLOCK_ROWS = 1 << 16


def _param_rng(seed: int, sub_seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(sub_seed), 0]))


def _block_rng(seed: int, sub_seed: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(sub_seed), 1, int(block)]))


def _draw_modes(M: int, amp_decades, rng: np.random.Generator):
    sigma = rng.uniform(-0.05, 0.0, M)
    omega = rng.uniform(0.1, math.pi, M)
    lam = np.exp(sigma + 1j * omega)
    if amp_decades is None:
        b = rng.standard_normal(M)
    else:
        m = np.arange(M, dtype=np.float64)
        b = 10.0 ** (-float(amp_decades) * m / max(M - 1, 1))
    return lam, b


def _accept_modes(lam: np.ndarray, min_sep: float = 1e-3) -> bool:
    """Distinct, non-real eigenvalues: pairwise gaps (including conjugates) and
    distance from the real axis at least ``min_sep``."""
    full = np.concatenate([lam, lam.conj()])
    if np.min(np.abs(lam.imag)) < min_sep:
        return False
    d = np.abs(full[:, None] - full[None, :])
    d[np.diag_indices_from(d)] = np.inf
    return bool(np.min(d) >= min_sep)


def _shape_matrix(lam, b, N):
    """D[m, j] = b_m lambda_m^j, j = 0..N-1 (complex, M x N)."""
    j = np.arange(N, dtype=np.float64)
    return b[:, None] * np.power(lam[:, None], j[None, :])


def expected_rms(lam, b, n, N):
    """rms_j of the clean snapshot j (j = 1..N), see the module docstring."""
    j = np.arange(N, dtype=np.float64)
    power = (b[:, None] ** 2) * np.power(np.abs(lam)[:, None], 2.0 * j[None, :])
    return np.sqrt(power.sum(axis=0) / (2.0 * n))


def _raw_numpy(w, n, N, sub_seed, lam, b):
    D = _shape_matrix(lam, b, N)
    M = lam.shape[0]
    Dst = np.concatenate([D.real, -D.imag], axis=0)  # (2M, N)
    scale = 1.0 / math.sqrt(2.0 * n)
    rms = expected_rms(lam, b, n, N) if w.noise > 0 else None
    X = np.empty((n, N), dtype=np.float64, order="F")
    nblk = (n + BLOCK_ROWS - 1) // BLOCK_ROWS
    for k in range(nblk):
        r0 = k * BLOCK_ROWS
        r1 = min(n, r0 + BLOCK_ROWS)
        rng = _block_rng(w.seed, sub_seed, k)
        G = rng.standard_normal((r1 - r0, 2 * M))
        blk = (G @ Dst) * scale
        if rms is not None:
            blk += rng.standard_normal((r1 - r0, N)) * (w.noise * rms)[None, :]
        X[r0:r1, :] = blk
    return X


def mode_parameters(w, n=None, max_tries: int = 1000):
    """Return (lambda, b, sub_seed) for workload ``w``.

    For a workload with ``kappa_max`` set (exact-rank data) sub-seeds are
    advanced until the eigenvalues are separated (>= 1e-3, also from the real
    axis) and the independent prefix X_1^{2M} has kappa_2 <= kappa_max.
    """
    n = w.n if n is None else int(n)
    M = w.pairs
    for sub in range(max_tries):
        lam, b = _draw_modes(M, w.amp_decades, _param_rng(w.seed, sub))
        if w.kappa_max is None:
            return lam, b, sub
        if not _accept_modes(lam):
            continue
        Xp = _raw_numpy(w, n, 2 * M, sub, lam, b)
        s = np.linalg.svd(Xp, compute_uv=False)
        if s[-1] > 0 and s[0] / s[-1] <= w.kappa_max:
            return lam, b, sub
    raise RuntimeError(f"no acceptable sub-seed for {w.name} in {max_tries} tries")


def snapshots_numpy(w, n=None, N=None, dtype=None):
    """X = [x_1 .. x_N] as an (n, N) Fortran-ordered array.

    ``dtype`` defaults to the workload's snapshot precision; FP32 snapshots are
    the FP64 values rounded once to nearest.
    Returns (X, lam, b).
    """
    n = w.n if n is None else int(n)
    N = w.N if N is None else int(N)
    lam, b, sub = mode_parameters(w, n=n)
    X = _raw_numpy(w, n, N, sub, lam, b)
    dt = dtype or ("float32" if w.snap_dtype == "f32" else "float64")
    if dt in ("float32", np.float32, "f32"):
        X = np.asfortranarray(X.astype(np.float32))
    return X, lam, b


def snapshots_torch(w, device, n=None, N=None, dtype=None, out=None, chunk_rows=1 << 20):
    """Generate X on ``device`` as an (N, n) tensor (row j = snapshot j+1).

    Uses torch's generator seeded per row chunk, so the values differ from
    ``snapshots_numpy`` while the statistics (modes, amplitudes, noise) are the
    same.  Returns (X, lam, b).
    """
    import torch

    n = w.n if n is None else int(n)
    N = w.N if N is None else int(N)
    if dtype is None:
        dtype = torch.float32 if w.snap_dtype == "f32" else torch.float64
    lam, b, sub = mode_parameters(w, n=min(n, 1 << 16))
    D = _shape_matrix(lam, b, N)
    Dst = np.concatenate([D.real, -D.imag], axis=0) / math.sqrt(2.0 * n)
    M2 = Dst.shape[0]
    Dt = torch.from_numpy(Dst).to(device=device, dtype=dtype)
    rms = torch.from_numpy(w.noise * expected_rms(lam, b, n, N)).to(device=device, dtype=dtype)
    if out is None:
        out = torch.empty((N, n), device=device, dtype=dtype)
    nch = (n + chunk_rows - 1) // chunk_rows
    for k in range(nch):
        r0 = k * chunk_rows
        r1 = min(n, r0 + chunk_rows)
        g = torch.Generator(device=device)
        g.manual_seed((int(w.seed) * 1_000_003 + int(sub) * 7919 + k) % (2**63 - 1))
        G = torch.randn((r1 - r0, M2), generator=g, device=device, dtype=dtype)
        blk = G @ Dt
        if w.noise > 0:
            blk += torch.randn((r1 - r0, N), generator=g, device=device, dtype=dtype) * rms[None, :]
        out[:, r0:r1].copy_(blk.t())
        del G, blk
    return out, lam, b


def batched_streams(bw, streams=None):
    """Per-stream workloads of a batched description (n_s log-uniform, N_s and
    pair counts uniform integers), deterministic in ``bw.seed``."""
    from .workloads import Workload

    S = bw.streams if streams is None else int(streams)
    rng = np.random.Generator(np.random.PCG64([int(bw.seed), 2]))
    out = []
    for s in range(S):
        n_s = int(round(2.0 ** rng.uniform(math.log2(bw.n_lo), math.log2(bw.n_hi))))
        N_s = int(rng.integers(bw.N_lo, bw.N_hi + 1))
        p_s = int(rng.integers(bw.pairs_lo, bw.pairs_hi + 1))
        out.append(Workload(f"{bw.name}[{s}]", n=n_s, N=N_s, pairs=p_s, amp_decades=None,
                            noise=bw.noise, snap_dtype=bw.snap_dtype,
                            seed=int(bw.seed) * 1000 + s))
    return out
