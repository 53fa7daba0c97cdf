"""foa_push_blocked_static (the blocked push with the library's static block
workspace, for callers that cannot allocate device memory) against
foa_push_blocked with a caller workspace, through the C ABI.

Both run the same kernels in the same launch configuration with fixed-order
reductions, so the results must be bitwise equal.  Two calls in a row, the
second on a smaller stream, so the second reads a static array that still
holds the first call's contents."""

import numpy as np
import pytest

import datagen
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name_case(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    announce(request.node.nodeid)
    yield


def _run(X, prec, static):
    import torch

    from paper_1805_05821_amd.stream import FOAStream

    N, n = X.shape
    s = FOAStream(n, N, prec=prec, ws_fill=0xFF)
    if static:
        s.push_blocked_static(X)
    else:
        s.push_blocked(X)
        s.bws.fill_(0xFF)  # the caller's block workspace is no longer needed
    status, q = s.sync()
    H, B, q, m = s.state()
    V = s.basis(q, dtype=torch.float64).cpu().numpy()
    s.close()
    return status, q, H, B, V


def test_static_block_workspace_matches_caller_workspace():
    import torch

    # each call smaller than the one before; the last one, noise-floor snapshots
    # at small n, takes the third projection in many of its blocks
    cases = [("f32", 300007, 44, "noisy_2p20x200"), ("f64", 50021, 22, "noisy_2p20x200"),
             ("f32", 5000, 400, "noisy_2p24x500")]
    for prec, n, N, name in cases:
        w = datagen.get_workload(name).with_n(n).with_N(N)
        Xh, _, _ = datagen.snapshots_numpy(w)
        X = torch.from_numpy(np.ascontiguousarray(Xh.T)).cuda()
        announce(f"blocked push, prec={prec} n={n} N={N}: caller workspace, then static workspace")
        ref = _run(X, prec, static=False)
        got = _run(X, prec, static=True)
        assert ref[0] == got[0] == 0 and ref[1] == got[1] == N
        for a, b, name in zip(ref[2:], got[2:], ("H_bar", "beta", "basis")):
            assert a.shape == b.shape and np.array_equal(a, b), f"{name} differs ({prec}, n={n})"
        announce(f"  bitwise equal: q={got[1]}")


def test_static_block_workspace_rejects_large_streams():
    import torch

    from paper_1805_05821_amd import foa as F
    from paper_1805_05821_amd.stream import FOAStream

    n, N = 2_500_000, 64
    need = F.foa_block_workspace_bytes(n, N, F.FOA_PREC_F32)
    assert need > F.FOA_BLOCK_STATIC_BYTES
    s = FOAStream(n, N, prec="f32")
    X = torch.zeros((4, n), dtype=torch.float32, device="cuda")
    with pytest.raises(F.FOAError) as e:
        s.push_blocked_static(X)
    assert e.value.code == F.FOA_E_NOMEM
    assert s.sync() == (0, 0)   # nothing was enqueued
    s.close()
