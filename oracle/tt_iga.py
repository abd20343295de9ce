"""Reference TT-IGA pipeline (Sections 4.2 and 4.3), plain FP64.

Steps, in the paper's order:

1. The geometry factors R_ij and f det J are sampled on the tensor Gauss grid
   and compressed to TT with prescribed accuracy eps.  The paper uses
   TT-cross for this; the oracle takes the deterministic TT-SVD of the full
   sample, an eps-accurate TT of the same sampled tensor.  R components are
   truncated relative to the largest ||R_ij||_F so that identically vanishing
   components become rank 0.
2. Each stiffness component K_ij becomes a TT matrix whose k-th core is the
   1-D Gauss sum of the factor core against the selector a_ij^(d)
   (Section 4.2.1): d = N'N'^T when d = i = j, m = N N^T when d differs from
   both i and j, and the mixed matrix when d equals exactly one of i, j.  The
   derivative sits on the row (test) index in direction i and on the column
   (trial) index in direction j, so K_ji is the transpose of K_ij.
3. K^TT is the sum of the nine components with TT-rounding (relative eps on
   the running sum) after each addition.
4. F^TT has cores sum_q w_q G_d(a, q, a') N_k(q) (Section 4.2.2).
5. Dirichlet conditions (Section 4.3): the rows and columns of boundary
   indices are cut from the cores, and the boundary data enter the right-hand
   side as F_I - (K u_g)_I.
6. The reduced system is solved by truncated TT-CG: conjugate gradients in
   which every new iterate, residual and direction is TT-rounded, with the
   residual replaced by the true residual b - K x every m iterations and at
   the stopping test.  (The paper solves with AMEn; CG is the TT-CG-type
   iteration used on this path, and results are compared, not iterates.)
"""
import numpy as np

from workloads.problem import BC_NATURAL, BC_TRACTION

from . import geometry, sparse_iga, tt

# Summation order of the nine components K_ij (diagonal first, then each off-diagonal pair).
TERM_ORDER = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1))


def factor_tts(problem, factors=None, eps=None):
    """TT of the six R components (global-norm truncation) and of f det J."""
    eps = problem.options.tt_eps if eps is None else eps
    if factors is None:
        factors, _ = geometry.sample_factors_grid(problem)
    d = 3
    rmax = max(np.linalg.norm(factors[i]) for i in range(6))
    delta_R = eps * rmax / np.sqrt(d - 1)
    R_tts = [tt.tt_svd(factors[i], delta=delta_R) for i in range(6)]
    fj = factors[6]
    fj_tt = tt.tt_svd(fj, delta=eps * np.linalg.norm(fj) / np.sqrt(d - 1))
    return R_tts, fj_tt


def r_index(i, j):
    """Position of R_ij (= R_ji) in geometry.R_PAIRS."""
    a, b = min(i, j), max(i, j)
    return geometry.R_PAIRS.index((a, b))


def term_cores(R_tt, tabs, i, j):
    """TT-matrix cores of K_ij: M_d[a, k, l, a'] = sum_q w_q G_d[a, q, a'] Row_d[q, k] Col_d[q, l]."""
    if R_tt is None:
        return None
    cores = []
    for d in range(3):
        row = tabs[d]["D"] if d == i else tabs[d]["B"]
        col = tabs[d]["D"] if d == j else tabs[d]["B"]
        cores.append(np.einsum("aqb,q,qk,ql->aklb", R_tt[d], tabs[d]["weights"], row, col))
    return cores


def assemble_K(problem, R_tts, tabs=None, eps=None):
    eps = problem.options.tt_eps if eps is None else eps
    if tabs is None:
        tabs = sparse_iga.one_d_tables(problem)
    K = None
    for (i, j) in TERM_ORDER:
        term = term_cores(R_tts[r_index(i, j)], tabs, i, j)
        if term is None:
            continue
        K = term if K is None else tt.mat_round(tt.mat_add(K, term), eps=eps)
    return K


def assemble_F(problem, fj_tt, tabs=None):
    """F^TT cores sum_q w_q G_d(a, q, a') N_k(q) (Section 4.2.2), plus the flux of traction
    faces (Section 3.1; the full-grid traction vector of the sparse assembly, TT-SVD at 1e-15,
    added and rounded)."""
    if tabs is None:
        tabs = sparse_iga.one_d_tables(problem)
    F = None
    if fj_tt is not None:
        F = [np.einsum("aqb,q,qk->akb", fj_tt[d], tabs[d]["weights"], tabs[d]["B"]) for d in range(3)]
    if any(k == BC_TRACTION for k in problem.dirichlet.kind):
        Fs = tt.tt_svd(sparse_iga.traction_load(problem, tabs).reshape(tuple(problem.disc.n_basis)), eps=1e-15)
        F = Fs if F is None else tt.round_(tt.add(F, Fs), eps=1e-15)
    return F


def interior_slices(problem):
    """Per direction, the index range left after removing Dirichlet end indices."""
    n = problem.disc.n_basis
    out = []
    for d in range(3):
        lo = 0 if problem.dirichlet.kind[2 * d] in (BC_NATURAL, BC_TRACTION) else 1
        hi = n[d] if problem.dirichlet.kind[2 * d + 1] in (BC_NATURAL, BC_TRACTION) else n[d] - 1
        out.append(slice(lo, hi))
    return out


def reduce_system(problem, K, F, eps=None):
    """K_II and rhs = F_I - (K u_g)_I in TT, by slicing cores and lifting the boundary data."""
    eps = problem.options.tt_eps if eps is None else eps
    sl = interior_slices(problem)
    KII = [M[:, sl[d], :, :][:, :, sl[d], :] for d, M in enumerate(K)]
    FI = None if F is None else [G[:, sl[d], :] for d, G in enumerate(F)]
    mask, vals = sparse_iga.dirichlet_values(problem)
    if np.any(vals != 0.0):
        ug = tt.tt_svd(vals.reshape(tuple(problem.disc.n_basis)), eps=1e-15)
        Kug = tt.matvec(K, ug)
        KugI = [G[:, sl[d], :] for d, G in enumerate(Kug)]
        FI = tt.round_(tt.add(FI, tt.scale(KugI, -1.0)), eps=eps * 1e-2)
    return KII, FI


def tt_cg(KII, b, eps, tol, max_iter=500, replace_every=10):
    """Truncated TT-CG with true-residual replacement; returns (x, stats).

    The iterate is rounded at min(eps, tol/10): truncating x by a relative
    delta moves the residual by up to kappa * delta, so a residual target tol
    needs the iterate kept more accurately than the search directions.
    """
    eps_x = min(eps, 0.1 * tol)
    nb = tt.norm(b)
    if nb == 0.0:
        return None, dict(iterations=0, rel_res=0.0, converged=True)
    x = None
    r = [G.copy() for G in b]
    p = [G.copy() for G in b]
    rho = tt.dot(r, r)
    hist = []
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        q = tt.round_(tt.matvec(KII, p), eps=eps)
        alpha = rho / tt.dot(p, q)
        x = tt.round_(tt.add(x, tt.scale(p, alpha)), eps=eps_x)
        r = tt.round_(tt.add(r, tt.scale(q, -alpha)), eps=eps)
        est = np.sqrt(max(tt.dot(r, r), 0.0)) / nb
        if it % replace_every == 0 or est <= tol:
            r = tt.round_(tt.add(b, tt.scale(tt.matvec(KII, x), -1.0)), eps=eps_x)
            true = tt.norm(r) / nb
            hist.append(true)
            if true <= tol:
                converged = True
                break
        rho_new = tt.dot(r, r)
        beta = rho_new / rho
        rho = rho_new
        p = tt.round_(tt.add(r, tt.scale(p, beta)), eps=eps)
    true = tt.norm(tt.add(b, tt.scale(tt.matvec(KII, x), -1.0))) / nb
    return x, dict(iterations=it, rel_res=true, converged=converged, history=hist)


def solve(problem, eps=None, tol=None, factors=None):
    """The whole reference pipeline; returns (u_I TT, dict with K, F, K_II, rhs, stats)."""
    eps = problem.options.tt_eps if eps is None else eps
    tol = problem.options.rel_res_tol if tol is None else tol
    tabs = sparse_iga.one_d_tables(problem)
    R_tts, fj_tt = factor_tts(problem, factors=factors, eps=eps)
    K = assemble_K(problem, R_tts, tabs, eps=eps)
    F = assemble_F(problem, fj_tt, tabs)
    KII, rhs = reduce_system(problem, K, F, eps=eps)
    x, stats = tt_cg(KII, rhs, eps=eps, tol=tol, max_iter=problem.options.max_iter)
    return x, dict(K=K, F=F, KII=KII, rhs=rhs, R_tts=R_tts, fj_tt=fj_tt, stats=stats)


def full_solution(problem, xI):
    """Full coefficient tensor (n0, n1, n2): interior from the TT, boundary from the data."""
    mask, vals = sparse_iga.dirichlet_values(problem)
    u = vals.reshape(tuple(problem.disc.n_basis)).copy()
    sl = interior_slices(problem)
    if xI is not None:
        u[sl[0], sl[1], sl[2]] = tt.full(xI)
    return u
