"""Pins for the oracle's TT algebra (Section 4.1) and TT assembly / solve (Sections 4.2-4.3)."""
import numpy as np
import pytest

import workloads as W
from oracle import geometry, sparse_iga, tt, tt_iga


def rand_tt(shape, ranks, rng):
    r = [1] + list(ranks) + [1]
    return [rng.normal(size=(r[k], n, r[k + 1])) for k, n in enumerate(shape)]


def test_full_uses_first_index_slowest():
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(size=3), rng.normal(size=4), rng.normal(size=5)
    cores = [a.reshape(1, 3, 1), b.reshape(1, 4, 1), c.reshape(1, 5, 1)]
    assert np.allclose(tt.full(cores).ravel(), np.kron(a, np.kron(b, c)), atol=0, rtol=1e-15)


def test_ttsvd_exact_low_rank_and_bound():
    rng = np.random.default_rng(1)
    X = tt.full(rand_tt((6, 7, 8), (2, 3), rng))
    cores = tt.tt_svd(X, eps=1e-12)
    assert tt.ranks(cores) == [1, 2, 3, 1]
    assert np.linalg.norm(tt.full(cores) - X) < 1e-12 * np.linalg.norm(X)
    Y = X + 1e-3 * rng.normal(size=X.shape)
    for eps in (1e-1, 1e-2, 1e-4):
        c = tt.tt_svd(Y, eps=eps)
        assert np.linalg.norm(tt.full(c) - Y) <= eps * np.linalg.norm(Y) * (1 + 1e-12)


def test_round_of_doubled_train():
    rng = np.random.default_rng(2)
    x = rand_tt((5, 6, 7), (3, 4), rng)
    y = tt.round_(tt.add(x, x), eps=1e-13)
    assert tt.ranks(y) == [1, 3, 4, 1]
    assert np.linalg.norm(tt.full(y) - 2 * tt.full(x)) < 1e-13 * np.linalg.norm(tt.full(x))


def test_round_error_bound():
    rng = np.random.default_rng(3)
    x = tt.add(rand_tt((6, 6, 6), (3, 3), rng), tt.scale(rand_tt((6, 6, 6), (4, 4), rng), 1e-3))
    for eps in (1e-1, 1e-2, 1e-3):
        y = tt.round_(x, eps=eps)
        assert np.linalg.norm(tt.full(y) - tt.full(x)) <= eps * np.linalg.norm(tt.full(x)) * (1 + 1e-10)


def test_dot_norm_against_dense():
    rng = np.random.default_rng(4)
    a, b = rand_tt((4, 5, 6), (2, 3), rng), rand_tt((4, 5, 6), (3, 2), rng)
    assert abs(tt.dot(a, b) - np.sum(tt.full(a) * tt.full(b))) < 1e-12 * np.linalg.norm(tt.full(a)) * np.linalg.norm(tt.full(b))
    assert abs(tt.norm(a) - np.linalg.norm(tt.full(a))) < 1e-13 * np.linalg.norm(tt.full(a))


def test_matvec_equals_dense_matvec():
    rng = np.random.default_rng(5)
    r = [1, 2, 3, 1]
    M = [rng.normal(size=(r[k], n, n, r[k + 1])) for k, n in enumerate((4, 5, 3))]
    x = rand_tt((4, 5, 3), (3, 2), rng)
    y = tt.matvec(M, x)
    ref = tt.mat_full(M) @ tt.full(x).ravel()
    assert np.linalg.norm(tt.full(y).ravel() - ref) < 1e-13 * np.linalg.norm(ref)
    # rank-1 TT matrix is the Kronecker product of its cores
    A = [rng.normal(size=(n, n)) for n in (3, 4, 2)]
    K1 = [a.reshape(1, *a.shape, 1) for a in A]
    assert np.allclose(tt.mat_full(K1), np.kron(A[0], np.kron(A[1], A[2])), rtol=0, atol=1e-14)


def test_annulus_K_tt_ranks_and_dense_equality():
    pr = W.c1_problem(n=10)
    K, F = sparse_iga.assemble(pr)
    R_tts, fj = tt_iga.factor_tts(pr)
    assert [tt.ranks(r) for r in R_tts[:3]] == [[1, 1, 1, 1]] * 3
    assert all(r is None for r in R_tts[3:])
    assert tt.ranks(fj) == [1, 1, 1, 1]
    KT = tt_iga.assemble_K(pr, R_tts)
    assert tt.ranks(tt.mat_as_tt(KT)) == [1, 3, 2, 1]
    Kd = K.toarray()
    assert np.linalg.norm(tt.mat_full(KT) - Kd) < 1e-13 * np.linalg.norm(Kd)
    FT = tt_iga.assemble_F(pr, fj)
    assert np.linalg.norm(tt.full(FT).ravel() - F) < 1e-13 * np.linalg.norm(F)


def test_identity_cube_K_ranks_2_2():
    pr = W.small_problem(W.identity_cube(), 7, 3, W.zero_source(), eps=1e-12)
    R_tts, _ = tt_iga.factor_tts(pr)
    KT = tt_iga.assemble_K(pr, R_tts)
    assert tt.ranks(tt.mat_as_tt(KT)) == [1, 2, 2, 1]


@pytest.mark.parametrize("geo,eps", [(W.twisted_box(1.2), 1e-8), (W.bumpy_cube(), 1e-6)])
def test_general_geometry_K_tt_within_eps(geo, eps):
    pr = W.small_problem(geo, 7, 3, W.fourier_source(geo, 11), eps=eps)
    K, F = sparse_iga.assemble(pr)
    R_tts, fj = tt_iga.factor_tts(pr)
    KT = tt_iga.assemble_K(pr, R_tts)
    Kd = K.toarray()
    assert np.linalg.norm(tt.mat_full(KT) - Kd) <= 10 * eps * np.linalg.norm(Kd)
    FT = tt_iga.assemble_F(pr, fj)
    assert np.linalg.norm(tt.full(FT).ravel() - F) <= 10 * eps * np.linalg.norm(F)


def test_tt_cg_matches_sparse_direct_c1():
    """Plain FP64 quarter-annulus case at tight eps: TT-CG agrees with SuperLU to 1e-10."""
    pr = W.c1_problem(eps=1e-13, tol=1e-13)
    u = sparse_iga.solve(pr)
    x, info = tt_iga.solve(pr)
    assert info["stats"]["converged"]
    uf = tt_iga.full_solution(pr, x).ravel()
    assert np.linalg.norm(uf - u) <= 1e-10 * np.linalg.norm(u)


def test_tt_cg_with_lifting_ring():
    """Constant Dirichlet data through the lifting term agree with the sparse solve."""
    import math
    from workloads.problem import BC_CONSTANT, BC_NATURAL, Dirichlet
    geo = W.annulus_sector(0.5, 1.0, math.pi / 2, 1.0)
    bc = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    pr = W.small_problem(geo, 8, 2, W.zero_source(), dirichlet=bc, eps=1e-12, tol=1e-12)
    u = sparse_iga.solve(pr)
    x, info = tt_iga.solve(pr)
    uf = tt_iga.full_solution(pr, x).ravel()
    assert np.linalg.norm(uf - u) <= 1e-9 * np.linalg.norm(u)


# ---- planted mistakes: each plausible error in the oracle must fail one of the pins above ----

def _K_mismatch(pr, monkeypatch=None):
    K, _ = sparse_iga.assemble(pr)
    R_tts, _ = tt_iga.factor_tts(pr)
    KT = tt_iga.assemble_K(pr, R_tts)
    return np.linalg.norm(tt.mat_full(KT) - K.toarray()) / np.linalg.norm(K.toarray())


def test_planted_dropped_offdiagonal_term_is_caught(monkeypatch):
    pr = W.small_problem(W.twisted_box(1.2), 6, 3, W.zero_source(), eps=1e-10)
    assert _K_mismatch(pr) < 1e-9
    monkeypatch.setattr(tt_iga, "TERM_ORDER", tuple(t for t in tt_iga.TERM_ORDER if t != (0, 1)))
    assert _K_mismatch(pr) > 1e-3


def test_planted_mixed_orientation_is_caught(monkeypatch):
    pr = W.small_problem(W.twisted_box(1.2), 6, 3, W.zero_source(), eps=1e-10)
    orig = tt_iga.term_cores

    def both_on_rows(R_tt, tabs, i, j):  # derivative on the row index in both directions
        if R_tt is None:
            return None
        out = []
        for d in range(3):
            row = tabs[d]["D"] if d in (i, j) else tabs[d]["B"]
            col = tabs[d]["D"] if (d == i and d == j) else tabs[d]["B"]
            out.append(np.einsum("aqb,q,qk,ql->aklb", R_tt[d], tabs[d]["weights"], row, col))
        return out

    monkeypatch.setattr(tt_iga, "term_cores", both_on_rows)
    assert _K_mismatch(pr) > 1e-3
    monkeypatch.setattr(tt_iga, "term_cores", orig)


def test_planted_transposed_metric_is_caught(monkeypatch):
    """R = det J J^-T J^-1 instead of det J J^-1 J^-T breaks the patch test on a twisted box."""
    from tests.test_oracle_assembly import test_patch_test_twisted_box

    def wrong(J):
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        return detJ, detJ[..., None, None] * (np.swapaxes(Jinv, -1, -2) @ Jinv)

    monkeypatch.setattr(geometry, "factors_from_jacobian", wrong)
    with pytest.raises(AssertionError):
        test_patch_test_twisted_box(1.5)
