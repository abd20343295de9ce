"""GPU end-to-end TT solve against the oracle's sparse direct solution."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import errors, sources, sparse_iga, tt, tt_iga
from tests.gpu_helpers import say
from workloads.problem import BC_CONSTANT, BC_NATURAL, BC_TRACTION, BC_ZERO, Dirichlet

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


def test_constant_dirichlet_on_faces_of_three_directions(ctx):
    """Constant data on faces of all three directions, with different values meeting at edges and
    corners, a homogeneous face and a natural one (Section 3.1 boundary split; the later face in
    face order wins where faces meet): the lifted right-hand side and the solution equal the
    oracle's reduction and sparse direct solve."""
    say("dirichlet three directions")
    geo = W.twisted_box(0.6)
    bc = Dirichlet(kind=(BC_CONSTANT, BC_ZERO, BC_CONSTANT, BC_NATURAL, BC_CONSTANT, BC_CONSTANT),
                   value=(1.0, 0.0, -2.0, 0.0, 0.5, 3.0))
    pr = W.small_problem(geo, 9, 2, W.fourier_source(geo, 7), dirichlet=bc, eps=1e-12, tol=1e-12)
    u_h, sysd = sparse_iga.solve(pr, return_system=True)
    h = ctx.problem_create(pr)
    h.assemble()
    rhs = tt.full(h.tt(3)).ravel()
    assert np.linalg.norm(rhs - sysd["rhs"]) <= 1e-11 * np.linalg.norm(sysd["rhs"])
    h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-9 * np.linalg.norm(u_h)


def test_traction_faces_match_sparse(ctx):
    """Flux (traction) data on three faces of a twisted box, whose face tangents are not
    orthogonal, beside homogeneous, constant and natural faces (Section 3.1 boundary split): the
    load vector with the face integrals and the solution equal the oracle's."""
    say("traction")
    geo = W.twisted_box(0.8)
    bc = Dirichlet(kind=(BC_ZERO, BC_TRACTION, BC_NATURAL, BC_TRACTION, BC_CONSTANT, BC_TRACTION),
                   value=(0.0, 0.7, 0.0, -1.3, 0.4, 2.0))
    pr = W.small_problem(geo, 9, 2, W.fourier_source(geo, 3), dirichlet=bc, eps=1e-12, tol=1e-12)
    _, F_sp = sparse_iga.assemble(pr)
    u_h = sparse_iga.solve(pr)
    h = ctx.problem_create(pr)
    h.assemble()
    F = tt.full(h.tt(1)).ravel()
    assert np.linalg.norm(F - F_sp) <= 1e-11 * np.linalg.norm(F_sp)
    h.solve()
    u = _full(pr, h.solution()).ravel()
    assert np.linalg.norm(u - u_h) <= 1e-9 * np.linalg.norm(u_h)


def test_ring_traction_reaches_the_log_solution(ctx):
    """Section 5.2's radial solution with the outer condition as a flux: u = 1 at r = 1 and
    du/dr = 1 / (2 ln 2) at r = 2 give u = 1 + ln(r) / ln 2; the device's TT-evaluated L2 error
    equals the oracle's integral of the same solution and is at the discretisation level."""
    from paper_2509_13224_amd import ttiga
    say("ring traction")
    g = 1.0 / (2.0 * math.log(2.0))
    bc = Dirichlet(kind=(BC_CONSTANT, BC_TRACTION) + (BC_NATURAL,) * 4, value=(1.0, g, 0, 0, 0, 0))
    pr = W.small_problem(W.annulus_sector(), (10, 5, 4), 3, W.zero_source(), dirichlet=bc, eps=1e-12, tol=1e-12)
    h = ctx.problem_create(pr)
    h.assemble()
    h.solve()
    prm = (1.0, 2.0, 1.0, 2.0)
    got = h.l2_error(ttiga.TTIGA_EXACT_RADIAL_LOG, params=prm)["rel_l2"]
    ref = errors.rel_l2(pr, _full(pr, h.solution()), lambda x: sources.ring_log_solution(x, *prm))
    assert abs(got - ref) <= 1e-8 * ref and got < 1e-5, (got, ref)


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
