"""TT-evaluated accuracy and compression reporting (Section 5) against the oracle.

ttiga_l2_error evaluates the relative L2 error of a solution entirely in TT format on the
device; the oracle integrates the same quantity on the dense Gauss grid (errors.rel_l2, p + 3
points per span, the same rule).  Compression ratios are checked against their definitions
from the oracle's own objects (sparse K non-zeros, the TT ranks)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import errors, sources, sparse_iga, tt_iga
from tests.gpu_helpers import say
from workloads.problem import BC_CONSTANT, BC_NATURAL, Dirichlet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=8 << 30)


def test_l2_error_manufactured_annulus(ctx):
    """The plain FP64 workload (quarter annulus, p = 2, n = 16): the device's TT-evaluated relative
    L2 error of its own solution equals the oracle's dense-grid integral of the same solution."""
    from paper_2509_13224_amd import ttiga
    say("accuracy: manufactured annulus")
    pr = W.c1_problem()
    h = ctx.problem_create(pr)
    h.assemble()
    h.solve()
    got = h.l2_error(ttiga.TTIGA_EXACT_MANUFACTURED_ANNULUS)
    u = tt_iga.full_solution(pr, h.solution())
    ref = errors.rel_l2(pr, u, sources.manufactured_annulus_solution)
    say("accuracy: device", got, "oracle", ref)
    assert abs(got["rel_l2"] - ref) <= 1e-8 * ref
    assert got["rel_l2"] < 1e-2  # the discretisation error of a degree-2 space at n = 16
    h.close()


def test_l2_error_ring_laplace(ctx):
    """The ring experiment's exact solution (Section 5.2): Laplace between radii 1 and 2 with
    u = 1 and u = 2 on the curved faces, natural elsewhere, degree 3, n = 12."""
    from paper_2509_13224_amd import ttiga
    say("accuracy: ring")
    geo = W.annulus_sector(1.0, 2.0, math.pi / 2, 1.0)
    bc = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    pr = W.small_problem(geo, 12, 3, W.zero_source(), dirichlet=bc, eps=1e-12, tol=1e-12)
    h = ctx.problem_create(pr)
    h.assemble()
    h.solve()
    prm = (1.0, 2.0, 1.0, 2.0)
    got = h.l2_error(ttiga.TTIGA_EXACT_RADIAL_LOG, params=prm)
    u = tt_iga.full_solution(pr, h.solution())
    ref = errors.rel_l2(pr, u, lambda x: sources.ring_log_solution(x, *prm))
    say("accuracy: ring device", got, "oracle", ref)
    assert abs(got["rel_l2"] - ref) <= 1e-8 * ref
    h.close()


def test_l2_error_at_full_size_and_convergence(ctx):
    """The manufactured field on the benchmark's discretisation (degree 3, n = 256, 16.7M DOF),
    where no dense grid is formed anywhere: the error is far below the solve's tolerance, and
    coarser meshes show the O(h^(p+1)) decay (slope about 4 between n = 16 and n = 32)."""
    from paper_2509_13224_amd import ttiga
    say("accuracy: full size")
    errs = {}
    for n in (16, 32, 256):
        pr = W.c2_problem(n=n)
        pr.source = W.manufactured_annulus_source()
        h = ctx.problem_create(pr, precond=1)
        h.assemble()
        h.solve()
        errs[n] = h.l2_error(ttiga.TTIGA_EXACT_MANUFACTURED_ANNULUS)["rel_l2"]
        h.close()
    say("accuracy: errors", errs)
    slope = math.log(errs[16] / errs[32]) / math.log((32 - 3) / (16 - 3))
    assert 3.3 <= slope <= 4.7, slope
    assert errs[256] <= 1e-6


def test_compression_ratios(ctx):
    """Ratios against their definitions: the sparse K of the oracle (its stored non-zeros), the
    dense N^2, N values of F, N_I of the solution, over the entries of the returned TT cores."""
    say("compression ratios")
    pr = W.c1_problem(n=14)
    h = ctx.problem_create(pr)
    h.assemble()
    h.solve()
    got = h.compression_ratios()
    K_sp, _ = sparse_iga.assemble(pr)
    p = pr.disc.degree
    Kc, Fc, uc = h.tt(0), h.tt(1), h.solution()
    k_entries = sum(c.size for c in Kc)  # banded cores [r][n][2p+1][r']
    N = np.prod(pr.disc.n_basis)
    band_count = np.prod([(n * (2 * p + 1) - p * (p + 1)) for n in pr.disc.n_basis])
    assert abs(got["K_sparse"] - band_count / k_entries) <= 1e-12 * got["K_sparse"]
    dense_entries = sum(c.shape[0] * c.shape[1] ** 2 * c.shape[-1] for c in Kc)
    assert abs(got["K_dense"] - N * N / dense_entries) <= 1e-12 * got["K_dense"]
    assert abs(got["F"] - N / sum(c.size for c in Fc)) <= 1e-12 * got["F"]
    n_int = np.prod([c.shape[1] for c in uc])
    assert abs(got["u"] - n_int / sum(c.size for c in uc)) <= 1e-12 * got["u"]
    # the sparse pattern is the Kronecker product of the 1-D bands (entries that cancel exactly
    # may be dropped by the sparse sum, never added)
    band_nnz = np.prod([(n * (2 * p + 1) - p * (p + 1)) for n in pr.disc.n_basis])
    assert 0.99 * band_nnz <= K_sp.nnz <= band_nnz
    h.close()
