"""GPU parity of the standalone TT kernels (matvec, dot, rounding, compression) against the oracle."""
import numpy as np
import pytest

from oracle import tt
from tests.gpu_helpers import banded_to_dense_cores, rand_banded, rand_tt, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context()


@pytest.mark.parametrize("shape,rK,rx,p", [
    ((5, 6, 7), (2, 3), (3, 2), 1),
    ((13, 9, 11), (3, 2), (4, 5), 2),
    ((17, 16, 15), (5, 4), (7, 6), 3),  # several 64-wide tiles and a ragged tail in the output
])
def test_matvec_matches_dense(ctx, shape, rK, rx, p):
    say("matvec", shape, rK, rx, p)
    rng = np.random.default_rng(sum(shape) + p)
    K = rand_banded(shape, rK, p, rng)
    x = rand_tt(shape, rx, rng)
    y = ctx.tt_matvec(to_dev(K), p, to_dev(x))
    assert tt.ranks(y) == [1, rK[0] * rx[0], rK[1] * rx[1], 1]
    ref = tt.mat_full(banded_to_dense_cores(K, p)) @ tt.full(x).ravel()
    got = tt.full(y).ravel()
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # the TT product itself agrees with the oracle's TT-matvec core by core
    yo = tt.matvec(banded_to_dense_cores(K, p), x)
    for a, b in zip(y, yo):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("shape,rK,rx,p", [
    ((600, 20, 9), (12, 84), (30, 7), 3),  # many row tiles with a ragged tail; LDS-limited tiles of 9 rows
    ((257, 31, 40), (5, 3), (64, 65), 2),  # vector ranks above one wave
    ((40, 30, 20), (3, 4), (5, 6), 5),     # the widest compiled band
    ((40, 30, 20), (3, 4), (5, 6), 6),     # a band width without its own kernel (generic path)
])
def test_matvec_cores_match_oracle(ctx, shape, rK, rx, p):
    """Every product core against the oracle's TT-matvec core (elementwise, within the rounding
    of a (2p+1)-term sum)."""
    say("matvec cores", shape, rK, rx, p)
    rng = np.random.default_rng(sum(shape) * 3 + p)
    K = rand_banded(shape, rK, p, rng)
    x = rand_tt(shape, rx, rng)
    y = ctx.tt_matvec(to_dev(K), p, to_dev(x))
    yo = tt.matvec(banded_to_dense_cores(K, p), x)
    for a, b in zip(y, yo):
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) <= 1e-14 * (2 * p + 1) * np.max(np.abs(b))


@pytest.mark.parametrize("shape,ra,rb", [((4, 5, 6), (2, 3), (3, 2)), ((40, 33, 70), (9, 7), (12, 5))])
def test_dot_matches_dense(ctx, shape, ra, rb):
    say("dot", shape, ra, rb)
    rng = np.random.default_rng(7)
    a, b = rand_tt(shape, ra, rng), rand_tt(shape, rb, rng)
    got = ctx.tt_dot(to_dev(a), to_dev(b))
    ref = float(np.sum(tt.full(a) * tt.full(b)))
    scale = np.linalg.norm(tt.full(a)) * np.linalg.norm(tt.full(b))
    assert abs(got - ref) <= 1e-13 * scale


def test_round_exact_low_rank_sum(ctx):
    """round(x + x) has rank(x) and equals 2x (TT-rounding of a structurally doubled train)."""
    say("round doubled")
    rng = np.random.default_rng(11)
    x = rand_tt((9, 12, 10), (3, 4), rng)
    xx = tt.add(x, x)
    y = ctx.tt_round(to_dev(xx), 1e-12)
    assert tt.ranks(y) == [1, 3, 4, 1]
    assert np.linalg.norm(tt.full(y) - 2 * tt.full(x)) <= 1e-12 * np.linalg.norm(tt.full(x))


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8, 1e-12])
def test_round_error_bound_and_ranks(ctx, eps):
    say("round eps", eps)
    rng = np.random.default_rng(12)
    # graded spectrum: sum of trains with geometrically decreasing weights
    x = None
    for s, w in enumerate((1.0, 1e-3, 1e-6, 1e-9)):
        x = tt.add(x, tt.scale(rand_tt((14, 15, 13), (3, 3), rng), w))
    y = ctx.tt_round(to_dev(x), eps)
    X = tt.full(x)
    err = np.linalg.norm(tt.full(y) - X)
    assert err <= eps * np.linalg.norm(X) * (1 + 1e-8)
    yo = tt.round_(x, eps=eps)
    assert tt.ranks(y) == tt.ranks(yo)


def test_round_large_ranks_multilevel_tsqr(ctx):
    """Ranks (40, 110) on a 40 x 60 x 120 grid: the 2400 x 110 unfolding takes the TSQR factor
    in global memory (c > 96), a tree of three levels and a last panel of two columns; the
    doubled train (ranks (80, 220)) rounds back to (40, 110) and equals 2x."""
    say("round large ranks")
    rng = np.random.default_rng(17)
    x = rand_tt((40, 60, 120), (40, 110), rng)
    X = tt.full(x)
    y = ctx.tt_round(to_dev(x), 1e-12)
    assert tt.ranks(y) == [1, 40, 110, 1]
    assert np.linalg.norm(tt.full(y) - X) <= 1e-11 * np.linalg.norm(X)
    z = ctx.tt_round(to_dev(tt.add(x, x)), 1e-12)
    assert tt.ranks(z) == [1, 40, 110, 1]
    assert np.linalg.norm(tt.full(z) - 2 * X) <= 1e-11 * np.linalg.norm(X)


def test_round_wide_unfoldings(ctx):
    """Ranks above the mode sizes (wide unfoldings) reduce to the true ranks."""
    say("round wide")
    rng = np.random.default_rng(13)
    x = rand_tt((3, 4, 3), (7, 9), rng)
    y = ctx.tt_round(to_dev(x), 1e-13)
    X = tt.full(x)
    assert tt.ranks(y)[1] <= 3 and tt.ranks(y)[2] <= 3
    assert np.linalg.norm(tt.full(y) - X) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("shape", [(12, 13, 14), (70, 40, 90)])
def test_compress_matches_ttsvd_bound(ctx, shape):
    """TT-SVD of a dense tensor (exact below 64 points per mode, randomised above)."""
    say("compress", shape)
    import torch
    rng = np.random.default_rng(14)
    A = tt.full(rand_tt(shape, (4, 5), rng)) + 1e-7 * rng.normal(size=shape)
    nrm = np.linalg.norm(A)
    for eps in (1e-3, 1e-5):
        delta = eps * nrm / np.sqrt(2)
        cores = ctx.tt_compress(torch.from_numpy(A).cuda(), delta)
        err = np.linalg.norm(tt.full(cores) - A)
        assert err <= 1.5 * eps * nrm
        ref = tt.tt_svd(A, delta=delta)
        assert tt.ranks(cores) == tt.ranks(ref)


def test_compress_zero_tensor(ctx):
    import torch
    say("compress zero")
    A = torch.zeros((5, 6, 7), dtype=torch.float64, device="cuda")
    assert ctx.tt_compress(A, 1e-12) is None


def test_compress_rank_deficient_geometry_factor(ctx):
    """f det J of the twisted box: unfoldings of numerical rank 14-16 out of 24 (regression:
    an orthogonalisation that is not exact on rank-deficient blocks returned NaN here)."""
    import torch

    import workloads as W
    from oracle import geometry
    say("compress twisted fJ")
    geo = W.twisted_box(1.2)
    pr = W.small_problem(geo, 9, 3, W.fourier_source(geo, 5), eps=1e-10)
    fac, _ = geometry.sample_factors_grid(pr)
    fj = fac[6]
    for eps in (1e-10, 1e-6):
        delta = eps * np.linalg.norm(fj) / np.sqrt(2)
        cores = ctx.tt_compress(torch.from_numpy(np.ascontiguousarray(fj)).cuda(), delta)
        assert np.linalg.norm(tt.full(cores) - fj) <= 1.5 * eps * np.linalg.norm(fj)
        assert tt.ranks(cores) == tt.ranks(tt.tt_svd(fj, delta=delta))


@pytest.mark.parametrize("block_bytes", [None, 1_000_000])
@pytest.mark.parametrize("sketch_rank", [64, 4])
@pytest.mark.parametrize("shape,rK,rx,rz,p,alpha,beta", [
    ((13, 9, 11), (3, 2), (4, 5), None, 2, 1.0, 0.0),
    ((17, 16, 15), (5, 4), (7, 6), (3, 4), 3, -1.0, 1.0),  # the residual form b - K x
    ((40, 33, 70), (6, 5), (9, 8), (4, 3), 3, 2.0, -0.5),  # several tiles and ragged tails
])
def test_matvec_round_matches_oracle(ctx, monkeypatch, shape, rK, rx, rz, p, alpha, beta, sketch_rank,
                                    block_bytes):
    """round(alpha K x + beta z, eps) without the product cores, against the oracle's exact
    alpha K x + beta z.  The random trains have no rank decay, so the rounded rank is the
    product rank: a sketch of width 64 + 10 covers it at once, one of width 4 + 10 has to be
    widened until it does; either way only the eps-rounding separates the result from the
    exact vector (<= eps ||y|| per the rounding bound; 10 eps allowed).  A 1 MB block budget
    splits the middle-mode contractions into blocks of a few rows of i with a ragged last
    block (and forms the middle sketch twice), which must not change the result."""
    say("matvec_round", shape, rK, rx, rz, p, alpha, beta, sketch_rank, block_bytes)
    if block_bytes is not None:
        monkeypatch.setenv("TTIGA_MATVEC_BLOCK_BYTES", str(block_bytes))
    rng = np.random.default_rng(sum(shape) + 7 * p + sketch_rank)
    K = rand_banded(shape, rK, p, rng)
    x = rand_tt(shape, rx, rng)
    z = rand_tt(shape, rz, rng) if rz else None
    eps = 1e-10
    y = ctx.tt_matvec_round(to_dev(K), p, to_dev(x), eps, alpha=alpha,
                            z_cores_dev=to_dev(z) if z is not None else None, beta=beta, sketch_rank=sketch_rank)
    ref = alpha * (tt.mat_full(banded_to_dense_cores(K, p)) @ tt.full(x).ravel())
    if z is not None:
        ref = ref + beta * tt.full(z).ravel()
    got = tt.full(y).ravel()
    assert np.linalg.norm(got - ref) <= 10 * eps * np.linalg.norm(ref)
    full_rank = [1, rK[0] * rx[0] + (rz[0] if rz else 0), rK[1] * rx[1] + (rz[1] if rz else 0), 1]
    assert all(a <= b for a, b in zip(tt.ranks(y), full_rank))
