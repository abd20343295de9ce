"""Mixed precision: the FP32/BF16 banded product against the FP64 product and against the
oracle's product of the rounded operands, and the iterative-refinement solve against the
FP64 path (1e-6, the mixed-precision gate) and the oracle's sparse direct solution."""
import numpy as np
import pytest

import workloads as W
from oracle import sparse_iga, tt, tt_iga
from tests.gpu_helpers import banded_to_dense_cores, rand_banded, rand_tt, say, to_dev
from workloads.problem import PREC_BF16, PREC_FP32, PREC_FP64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=8 << 30)


def _round_f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _round_bf16(a):
    """FP64 -> FP32 -> BF16, round to nearest even (finite inputs)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rel(a, b):
    return tt.norm(tt.add(a, tt.scale(b, -1.0))) / tt.norm(b)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("shape,rK,rx,p", [((13, 9, 11), (3, 2), (4, 5), 2), ((17, 16, 15), (5, 4), (7, 6), 3)])
def test_lowp_matvec(ctx, dtype, shape, rK, rx, p):
    say("lowp matvec", dtype, shape)
    rng = np.random.default_rng(sum(shape) + 10 * dtype)
    K = rand_banded(shape, rK, p, rng)
    x = rand_tt(shape, rx, rng)
    y = ctx.tt_matvec(to_dev(K), p, to_dev(x), dtype=dtype)
    assert tt.ranks(y) == [1, rK[0] * rx[0], rK[1] * rx[1], 1]
    exact = tt.matvec(banded_to_dense_cores(K, p), x)
    # FP32 operands: within 1e-6 of the FP64 product; BF16 operator: within 3e-2
    assert _rel(y, exact) <= (1e-6 if dtype == 1 else 3e-2)
    # and the product of the rounded operands, to FP32 accumulation accuracy, core by core
    Kr = [(_round_f32 if dtype == 1 else _round_bf16)(c) for c in K]
    xr = [_round_f32(c) for c in x]
    ref = tt.matvec(banded_to_dense_cores(Kr, p), xr)
    for a, b in zip(y, ref):
        assert np.max(np.abs(a - b)) <= 2e-6 * np.max(np.abs(b))


@pytest.mark.parametrize("prec", [PREC_FP32, PREC_BF16])
def test_mixed_solve_matches_fp64(ctx, prec):
    """Plain-vs-mixed family (annulus, p=3, Fourier source) at n=24: the refined solution is
    within 1e-6 of the FP64 solve at eps/10, tol/10 and of the sparse direct solution."""
    say("mixed solve", prec)
    pr = W.c2_problem(n=24, precision=prec)
    h = ctx.problem_create(pr, precond=1)
    h.assemble()
    st = h.solve()
    u = h.solution()
    assert st["refine_steps"] >= 2
    ref_pr = W.c2_problem(n=24, eps=1e-7, tol=1e-8)
    hr = ctx.problem_create(ref_pr, precond=1)
    hr.assemble()
    hr.solve()
    u_ref = hr.solution()
    assert _rel(u, u_ref) <= 1e-6
    u_h = sparse_iga.solve(pr)
    x = tt_iga.full_solution(pr, u).ravel()
    assert np.linalg.norm(x - u_h) <= 1e-6 * np.linalg.norm(u_h)


def test_bf16_refinement_stops_when_not_contracting(ctx):
    """At n=128 kappa u_bf16 exceeds one: the refinement stops with E_NOTCONV after a few
    steps (the solution and its error estimate are still returned), FP32 converges."""
    from paper_2509_13224_amd import ttiga
    say("bf16 n128")
    h = ctx.problem_create(W.c2_problem(n=128, precision=PREC_BF16), precond=1)
    h.assemble()
    st = h.solve(allow_notconv=True)
    assert st["status"] == ttiga.TTIGA_E_NOTCONV and st["refine_steps"] <= 6
    assert st["rel_pres"] > 1e-6 and h.solution() is not None
    h2 = ctx.problem_create(W.c2_problem(n=128, precision=PREC_FP32), precond=1)
    h2.assemble()
    st2 = h2.solve()
    assert st2["status"] == 0 and st2["rel_pres"] <= 1e-7


def test_mixed_batch_equals_alone(ctx):
    say("mixed batch")
    reqs = W.c4_requests(count=4, sizes=(12, 16), precision=PREC_FP32, eps=1e-6, tol=1e-7)
    out = ctx.solve_batch(reqs, lanes=2)
    for pr, (res, u) in zip(reqs, out):
        assert res["status"] == 0 and res["refine_steps"] >= 1, res
        h = ctx.problem_create(pr, precond=1)
        h.assemble()
        h.solve()
        u0 = h.solution()
        h.close()
        assert _rel(u, u0) <= 1e-12
