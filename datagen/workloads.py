"""Workload descriptions: sizes, mode counts, amplitude spread, noise and seeds.

Each workload is named by what it is.  The five shapes are

* ``exact_rank_4096x64``  - n=4096, N=64, 10 complex modes (rank 20), b_m ~ N(0,1),
  no noise, FP64 snapshots, kappa_2 of the independent prefix kept <= 1e3 by
  rejection of sub-seeds.
* ``noisy_2p20x200``      - n=2^20, N=200, 40 pairs, |b_m| decaying geometrically
  over 1e0..1e-4, relative noise 1e-6, FP64 snapshots.
* ``noisy_2p24x500``      - n=2^24, N=500, 120 pairs over 1e0..1e-7, noise 1e-8,
  FP32 snapshots (the throughput workload).
* ``batched_256``         - 256 independent streams, n_s log-uniform in
  [2^12, 2^18], N_s ~ U[20, 300], 5..30 pairs each, noise 1e-6, FP32.
* ``large_1e8x300``       - n=1e8, N=300, 80 pairs over 1e0..1e-5, noise 1e-7, FP32,
  followed by a rank-160 mode reconstruction.

They stand in for the paper's flow datasets (linearised channel flow, cylinder
wake, jets in cross-flow), which are not available: the sizes and conditioning
follow the paper's regimes (Section 4), the values are synthetic.
"""

from dataclasses import dataclass, replace
from typing import Optional


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # snapshot length (rows)
    N: int                 # number of snapshots
    pairs: int             # number of complex-conjugate mode pairs
    amp_decades: Optional[float]  # None: b_m ~ N(0,1); else |b_m| = 10^(-d (m-1)/(M-1))
    noise: float           # relative i.i.d. Gaussian noise amplitude
    snap_dtype: str        # "f64" or "f32": precision the snapshots are held in
    seed: int
    kappa_max: Optional[float] = None  # rejection bound on kappa_2 of the independent prefix
    modes_r: int = 0       # packed mode columns reconstructed after the run (0: none)

    def with_n(self, n: int) -> "Workload":
        """Same modes, amplitudes, noise and seed at a different row count."""
        return replace(self, n=int(n))

    def with_N(self, N: int) -> "Workload":
        return replace(self, N=int(N))


@dataclass(frozen=True)
class BatchedWorkload:
    name: str
    streams: int
    n_lo: int
    n_hi: int
    N_lo: int
    N_hi: int
    pairs_lo: int
    pairs_hi: int
    noise: float
    snap_dtype: str
    seed: int


WORKLOADS = {
    "exact_rank_4096x64": Workload(
        "exact_rank_4096x64", n=4096, N=64, pairs=10, amp_decades=None, noise=0.0,
        snap_dtype="f64", seed=1805, kappa_max=1e3),
    "noisy_2p20x200": Workload(
        "noisy_2p20x200", n=1 << 20, N=200, pairs=40, amp_decades=4.0, noise=1e-6,
        snap_dtype="f64", seed=1806),
    "noisy_2p24x500": Workload(
        "noisy_2p24x500", n=1 << 24, N=500, pairs=120, amp_decades=7.0, noise=1e-8,
        snap_dtype="f32", seed=1807),
    "batched_256": BatchedWorkload(
        "batched_256", streams=256, n_lo=1 << 12, n_hi=1 << 18, N_lo=20, N_hi=300,
        pairs_lo=5, pairs_hi=30, noise=1e-6, snap_dtype="f32", seed=1808),
    "large_1e8x300": Workload(
        "large_1e8x300", n=100_000_000, N=300, pairs=80, amp_decades=5.0, noise=1e-7,
        snap_dtype="f32", seed=1809, modes_r=160),
}


def get_workload(name: str):
    try:
        return WORKLOADS[name]
    except KeyError:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}") from None
