"""GPU end-to-end TT solve against the oracle's sparse direct solution."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import errors, sources, sparse_iga, tt, tt_iga
from tests.gpu_helpers import say
from workloads.problem import BC_CONSTANT, BC_NATURAL, Dirichlet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context()


def _full(pr, x):
    return tt_iga.full_solution(pr, x)


def test_c1_parity_mode(ctx):
    """Quarter annulus p=2 n=16, eps 1e-13, tol 1e-13: ||u_gpu - u_h|| <= 1e-10 ||u_h||."""
    say("c1 parity")
    pr = W.c1_problem(eps=1e-13, tol=1e-13)
    u_h = sparse_iga.solve(pr)
    h = ctx.problem_create(pr)
    h.assemble()
    st = h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-10 * np.linalg.norm(u_h), st
    assert st["rel_res"] <= 1e-13


def test_c1_config_mode(ctx):
    """The plain FP64 workload itself (eps 1e-10, rel-res 1e-10): error within eps + kappa tol."""
    say("c1 config")
    pr = W.c1_problem()
    u_h, sysd = sparse_iga.solve(pr, return_system=True)
    kappa = sparse_iga.condition_estimate(sysd["KII"])
    h = ctx.problem_create(pr)
    h.assemble()
    st = h.solve()
    u = _full(pr, h.solution())
    err = np.linalg.norm(u.ravel() - u_h) / np.linalg.norm(u_h)
    assert err <= 1e-10 + kappa * 1e-10, (err, kappa, st)
    l2 = errors.rel_l2(pr, u, sources.manufactured_annulus_solution)
    l2h = errors.rel_l2(pr, u_h.reshape(16, 16, 16), sources.manufactured_annulus_solution)
    assert abs(l2 - l2h) <= 1e-8


def test_twisted_box_solve(ctx):
    say("twisted solve")
    geo = W.twisted_box(1.0)
    pr = W.small_problem(geo, 10, 3, W.fourier_source(geo, 21), eps=1e-12, tol=1e-12)
    u_h = sparse_iga.solve(pr)
    h = ctx.problem_create(pr)
    h.assemble()
    st = h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-9 * np.linalg.norm(u_h), st


def test_ring_constant_dirichlet_solve(ctx):
    say("ring solve")
    geo = W.annulus_sector(0.5, 1.0, math.pi / 2, 1.0)
    bc = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    pr = W.small_problem(geo, 9, 2, W.zero_source(), dirichlet=bc, eps=1e-12, tol=1e-12)
    u_h = sparse_iga.solve(pr)
    h = ctx.problem_create(pr)
    h.assemble()
    h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-9 * np.linalg.norm(u_h)


def test_max_iter_reports_notconv(ctx):
    from paper_2509_13224_amd import ttiga
    say("notconv")
    pr = W.c1_problem(n=10)
    pr.options.max_iter = 1
    h = ctx.problem_create(pr)
    h.assemble()
    st = h.solve(allow_notconv=True)
    assert st["status"] == ttiga.TTIGA_E_NOTCONV and st["iterations"] == 1
    assert h.solution() is not None


@pytest.mark.parametrize("name", ["annulus_c1", "twisted_p3_n10", "bumpy_p3_n9"])
def test_preconditioned_solve_matches_sparse(ctx, name):
    """Flexible PCG with the separable preconditioner reaches the same discrete solution."""
    say("pcg", name)
    if name == "annulus_c1":
        pr = W.c1_problem(eps=1e-12, tol=1e-12)
    elif name == "twisted_p3_n10":
        geo = W.twisted_box(1.0)
        pr = W.small_problem(geo, 10, 3, W.fourier_source(geo, 21), eps=1e-11, tol=1e-11)
    else:
        geo = W.bumpy_cube()
        pr = W.small_problem(geo, 9, 3, W.fourier_source(geo, 4), eps=1e-11, tol=1e-11)
    u_h = sparse_iga.solve(pr)
    h = ctx.problem_create(pr, precond=1)
    h.assemble()
    st = h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-8 * np.linalg.norm(u_h), st
    assert st["iterations"] <= 40, st


def test_rank_cap_reports_rankcap(ctx):
    """A rank cap below what a TT needs fails the call with E_RANKCAP instead of truncating
    silently: at assembly when the operator itself needs more (annulus K^TT has ranks (3, 2)),
    at the solve when only the iterates do."""
    from paper_2509_13224_amd import ttiga
    say("rankcap")
    pr = W.c1_problem(n=12, eps=1e-10, tol=1e-10)
    pr.options.max_rank = 2
    h = ctx.problem_create(pr)
    with pytest.raises(ttiga.TTIGAError) as e:
        h.assemble()
    assert e.value.code == ttiga.TTIGA_E_RANKCAP
    h.close()
    pr.options.max_rank = 4
    h = ctx.problem_create(pr)
    st = h.assemble()
    assert max(st["rank_K"]) <= 4
    with pytest.raises(ttiga.TTIGAError) as e:
        h.solve()
    assert e.value.code == ttiga.TTIGA_E_RANKCAP
    h.close()
