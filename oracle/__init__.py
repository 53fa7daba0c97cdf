"""CPU FP64 oracle of FOA-based DMD (test infrastructure).

ONLY ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The
product path (the HIP library and its Python binding) never uses it, and this
package never imports the product path.

Everything here is plain NumPy in float64, written from the paper:
Algorithm 1 (batch FOA-based DMD), Algorithm 2 (Rayleigh-Ritz with Arnoldi,
used only as a known-A test reference), Algorithms 3/4 (streaming form), the
error indicators of Section 3.2.3 and the coefficients of Section 3.2.4;
``lowsync`` is the one-reduction form of the FOA step (the QR view of
Section 3.1 with the two Gram-Schmidt projections of consecutive snapshots
sharing one sweep and one reduction).
"""

from .foa import (
    EPS64,
    EPS32,
    FOAState,
    foa_batch,
    foa_stream_init,
    foa_stream_update,
    default_breakdown_tol,
    arnoldi_known_A,
)
from .dmd import (
    projected_size,
    dmd_untruncated,
    dmd_truncated,
    truncation_rank,
    kappa2,
    spacing,
    packed_modes,
    packed_coefficients,
)
from . import foa, dmd, lowsync

__all__ = [
    "EPS64",
    "EPS32",
    "FOAState",
    "foa_batch",
    "foa_stream_init",
    "foa_stream_update",
    "default_breakdown_tol",
    "arnoldi_known_A",
    "projected_size",
    "dmd_untruncated",
    "dmd_truncated",
    "truncation_rank",
    "kappa2",
    "spacing",
    "packed_modes",
    "packed_coefficients",
    "foa",
    "dmd",
    "lowsync",
]
