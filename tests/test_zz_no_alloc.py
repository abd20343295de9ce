"""The allocation-free TT inner product (ttiga_tt_dot_noalloc) against the allocating entry point
ttiga_tt_dot and the oracle: two calls in a row, the second with a smaller input (the shared
scratch array keeps the first call's contents), each giving the same bits as ttiga_tt_dot and
agreeing with the oracle's dot within the rounding bound; inputs too large for the fixed
scratch are refused before anything is launched."""
import numpy as np
import pytest

from oracle import tt
from tests.gpu_helpers import rand_tt, say, to_dev

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _abs_bound(x, y):
    """Forward error bound of the contraction chain: a small multiple of u times the dot of the
    absolute cores (each GEMM contributes at most its contraction length times u)."""
    ax = [np.abs(c) for c in x]
    ay = [np.abs(c) for c in y]
    length = sum(c.shape[0] * c.shape[1] for c in x) + sum(c.shape[1] for c in y)
    return 4 * length * U * tt.dot(ax, ay)


def test_noalloc_dot_matches_dot(gpu_lib):
    import torch

    from paper_2509_13224_amd import ttiga
    ctx = ttiga.Context(workspace_bytes=1 << 30)
    rng = np.random.default_rng(2025)
    # a large call first, then a smaller one on the same scratch
    cases = [((300, 256, 200), (48, 37), (33, 64)), ((17, 9, 30), (3, 5), (2, 7))]
    for shape, rx, ry in cases:
        say("noalloc dot", shape, rx, ry)
        x = rand_tt(shape, rx, rng)
        y = rand_tt(shape, ry, rng)
        xd, yd = to_dev(x), to_dev(y)
        ref = ctx.tt_dot(xd, yd)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
        ctx.tt_dot_noalloc(xd, yd, out)
        got = float(out.item())  # synchronises torch's current stream, the context's stream
        assert got == ref, (got, ref)
        exact = tt.dot(x, y)
        assert abs(got - exact) <= _abs_bound(x, y), (got, exact)


def test_noalloc_dot_refuses_oversized_inputs(gpu_lib):
    import torch

    from paper_2509_13224_amd import ttiga
    say("noalloc dot: oversized")
    ctx = ttiga.Context(workspace_bytes=1 << 30)
    shape, r = (600, 600, 600), (200, 200)
    cores = [torch.zeros((a, n, b), dtype=torch.float64, device="cuda:0")
             for a, n, b in zip((1,) + r, shape, r + (1,))]
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ttiga.TTIGAError) as e:
        ctx.tt_dot_noalloc(cores, cores, out)
    assert e.value.code == ttiga.TTIGA_E_ARG and "scratch" in str(e.value)
