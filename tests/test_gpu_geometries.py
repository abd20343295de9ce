"""The paper's own geometries on the HIP path (Section 5): the L-shape with a C0 knot in its
map (Section 5.1) and the full ring with the nine-point rational circle (Section 5.2), each
against the oracle's sparse direct solution, and their TT-evaluated L2 errors against the
closed-form solutions the paper gives."""
import numpy as np
import pytest

import workloads as W
from oracle import errors, sources, sparse_iga, tt_iga
from tests.gpu_helpers import say
from workloads.problem import BC_CONSTANT, BC_NATURAL, BC_ZERO, Dirichlet

pytestmark = pytest.mark.gpu

LSHAPE_BC = Dirichlet(kind=(BC_ZERO,) * 4 + (BC_NATURAL,) * 2, value=(0.0,) * 6)
RING_BC = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=8 << 30)


def _solve(ctx, pr, precond=0):
    h = ctx.problem_create(pr, precond=precond)
    h.assemble()
    h.solve()
    return h


@pytest.mark.parametrize("p", [1, 2])
def test_lshape_matches_sparse_and_exact(ctx, p):
    """Linear (the paper's choice) and quadratic B-splines on the L-shape, f = sin(pi x) sin(pi y),
    homogeneous Dirichlet on the lateral faces, natural on z = 0, 1: the TT solution equals the
    oracle's u_h, and the device's L2 error equals the oracle's integral of the same solution."""
    from paper_2509_13224_amd import ttiga
    nb = (21, 11, 4) if p == 1 else (22, 12, 5)
    say("lshape", p, nb)
    pr = W.small_problem(W.lshape(), nb, p, W.sine_xy_source(), dirichlet=LSHAPE_BC, eps=1e-12, tol=1e-12)
    u_h = sparse_iga.solve(pr)
    h = _solve(ctx, pr)
    u = tt_iga.full_solution(pr, h.solution())
    assert np.linalg.norm(u.ravel() - u_h) <= 1e-9 * np.linalg.norm(u_h)
    got = h.l2_error(ttiga.TTIGA_EXACT_SINE_XY)
    ref = errors.rel_l2(pr, u, sources.lshape_solution)
    say("lshape", p, "L2 error device", got["rel_l2"], "oracle", ref)
    assert abs(got["rel_l2"] - ref) <= 1e-8 * ref
    h.close()


def test_lshape_linear_convergence_on_device(ctx):
    """The paper's observation for the L-shape with linear functions: slope about 2 of the L2
    error against the points per edge, here from the device's TT-evaluated errors of
    preconditioned solves up to the paper's 61 x 31 x 31 mesh."""
    from paper_2509_13224_amd import ttiga
    errs = []
    for nb in ((16, 8, 8), (31, 16, 16), (61, 31, 31)):
        say("lshape convergence", nb)
        pr = W.small_problem(W.lshape(), nb, 1, W.sine_xy_source(), dirichlet=LSHAPE_BC, eps=1e-9, tol=1e-9)
        h = _solve(ctx, pr, precond=1)
        errs.append(h.l2_error(ttiga.TTIGA_EXACT_SINE_XY)["rel_l2"])
        h.close()
    say("lshape errors", errs)
    slope = np.log(errs[1] / errs[2]) / np.log(30.0 / 15.0)
    assert 1.7 <= slope <= 2.3, (errs, slope)


def test_full_ring_matches_sparse_and_exact(ctx):
    """The full ring (r 0.5..1, height 1) with u = 1 and 2 on the cylinders: the TT solution equals
    the oracle's u_h and its L2 error the oracle's integral; the log solution is reached to the
    discretisation error."""
    from paper_2509_13224_amd import ttiga
    say("full ring")
    pr = W.small_problem(W.ring(), (8, 13, 4), 2, W.zero_source(), dirichlet=RING_BC, eps=1e-12, tol=1e-12)
    u_h = sparse_iga.solve(pr)
    h = _solve(ctx, pr)
    u = tt_iga.full_solution(pr, h.solution())
    assert np.linalg.norm(u.ravel() - u_h) <= 1e-9 * np.linalg.norm(u_h)
    prm = (0.5, 1.0, 1.0, 2.0)
    got = h.l2_error(ttiga.TTIGA_EXACT_RADIAL_LOG, params=prm)
    ref = errors.rel_l2(pr, u, lambda x: sources.ring_log_solution(x, *prm))
    say("full ring L2 error device", got["rel_l2"], "oracle", ref)
    assert abs(got["rel_l2"] - ref) <= 1e-8 * ref and got["rel_l2"] < 1e-4
    h.close()
