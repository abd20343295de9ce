"""Parity at the full size of the timed workload: the C2 annulus (degree 3, 256 basis functions
per direction, 16.7M DOF, 8-mode Fourier source, TT eps 1e-6), assembled by the same kernels
the batched bench runs in every lane (cross approximation of the factors, det J pass, core
assembly, sums with rounding).  The oracle cannot assemble 16.7M DOF, but it computes single
entries from their definition (Sec. 3.3, eqs. Kfinal and ffinal): a Gauss sum over the
supports of the two basis functions, with the oracle's own B-spline, NURBS and metric
routines.  Sampled entries of K^TT and F^TT, and sampled values of the factor TTs, are compared
with those."""
import numpy as np
import pytest

import workloads as W
from oracle import bspline, geometry
from oracle import tt as ott
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

N_ENTRIES = 24


@pytest.fixture(scope="module")
def ctx():
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=16 << 30)


@pytest.fixture(scope="module")
def assembled(ctx):
    from paper_2509_13224_amd import ttiga
    say("fullsize C2 assembly")
    pr = W.c2_problem(n=256)
    h = ctx.problem_create(pr, precond=1)
    st = h.assemble()
    say("fullsize C2 copy cores", st["compression_path"], st["rank_K"])
    K = h.tt(ttiga.WHICH_K)
    F = h.tt(ttiga.WHICH_F)
    fac = [h.tt(ttiga.WHICH_FACTOR0 + f) for f in range(7)]
    h.close()
    return pr, st, K, F, fac


def _tables(pr):
    """Per direction: Gauss nodes, weights, basis values B (Q x n) and derivatives D."""
    p = pr.disc.degree
    out = []
    for d, (nodes, wts) in enumerate(geometry.gauss_grid(pr)):
        kn = bspline.open_uniform_knots(pr.disc.n_basis[d], p)
        out.append((nodes, wts, bspline.basis(kn, p, nodes), bspline.basis_derivative(kn, p, nodes)))
    return out


def _reference_entries(pr, tabs, a, b):
    """K[a, b] and F[a] from their definition on the Gauss points where both supports meet."""
    sub, vals = [], []
    for d in range(3):
        nodes, wts, B, D = tabs[d]
        sa = (B[:, a[d]] != 0) | (D[:, a[d]] != 0)
        sb = (B[:, b[d]] != 0) | (D[:, b[d]] != 0)
        q = np.nonzero(sa & sb)[0]
        sub.append((nodes[q], wts[q]))
        vals.append((wts[q], B[q, a[d]], D[q, a[d]], B[q, b[d]], D[q, b[d]]))
    factors, _ = geometry.sample_factors_grid(pr, grid=sub)
    R = np.zeros((3, 3) + factors.shape[1:])
    for idx, (i, j) in enumerate(geometry.R_PAIRS):
        R[i, j] = factors[idx]
        R[j, i] = factors[idx]
    w = np.einsum("i,j,k->ijk", vals[0][0], vals[1][0], vals[2][0])

    def grad(which):
        # d phi / d xi_i on the sub-grid: the derivative in direction i only
        g = []
        for i in range(3):
            f = [vals[d][1 + 2 * which] if d != i else vals[d][2 + 2 * which] for d in range(3)]
            g.append(np.einsum("i,j,k->ijk", *f))
        return g

    ga, gb = grad(0), grad(1)
    K_ab = sum(np.sum(w * ga[i] * R[i, j] * gb[j]) for i in range(3) for j in range(3))
    # F[a] needs the full support of a alone
    sub_a, wa = [], []
    for d in range(3):
        nodes, wts, B, D = tabs[d]
        q = np.nonzero(B[:, a[d]] != 0)[0]
        sub_a.append((nodes[q], wts[q]))
        wa.append((wts[q], B[q, a[d]]))
    fa, _ = geometry.sample_factors_grid(pr, grid=sub_a)
    wb = np.einsum("i,j,k->ijk", *[wa[d][0] * wa[d][1] for d in range(3)])
    F_a = np.sum(wb * fa[6])
    # F_a is the functional sum_q w_q B_a(q) (f det J)(q) of the factor samples: by
    # Cauchy-Schwarz an error e in the f det J train moves it by at most ||w B_a||_2 ||e||_2
    return K_ab, F_a, np.sqrt(np.sum(wb * wb))


def _tt_matrix_entry(cores, a, b, p):
    v = np.ones((1,))
    for d in range(3):
        t = b[d] - a[d] + p
        v = v @ cores[d][:, a[d], t, :]
    return float(v[0])


def _tt_vector_entry(cores, a):
    v = np.ones((1,))
    for d in range(3):
        v = v @ cores[d][:, a[d], :]
    return float(v[0])


def _pairs(n, p, count, seed):
    """Random (a, b) index pairs within the band, with the faces and corners represented."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        a = rng.integers(0, n, size=3)
        if s % 4 == 0:
            a[s % 3] = 0 if s % 8 == 0 else n - 1
        off = rng.integers(-p, p + 1, size=3) if s % 3 else np.zeros(3, dtype=int)
        b = np.clip(a + off, 0, n - 1)
        out.append((tuple(int(x) for x in a), tuple(int(x) for x in b)))
    return out


def test_fullsize_entries_match_definition(assembled):
    pr, st, K, F, _ = assembled
    p, n = pr.disc.degree, pr.disc.n_basis[0]
    assert st["compression_path"] == 2  # the cross approximation, as in the bench
    assert K[0].shape[1] == n and K[0].shape[2] == 2 * p + 1
    tabs = _tables(pr)
    refK, gotK, refF, gotF, csw = [], [], [], [], []
    for a, b in _pairs(n, p, N_ENTRIES, 2025091302):
        rk, rf, cs = _reference_entries(pr, tabs, a, b)
        refK.append(rk)
        gotK.append(_tt_matrix_entry(K, a, b, p))
        refF.append(rf)
        gotF.append(_tt_vector_entry(F, a))
        csw.append(cs)
    refK, gotK, refF, gotF, csw = map(np.asarray, (refK, gotK, refF, gotF, csw))
    say("fullsize K entries: max |diff|", np.abs(gotK - refK).max(), "of max |K|", np.abs(refK).max())
    # the annulus factors are exactly separable (R rank 1, K^TT ranks (3, 2)), so the TT
    # operator reproduces every entry up to rounding in the Gauss sums
    assert np.abs(gotK - refK).max() <= 1e-9 * np.abs(refK).max()
    # F^TT is the Gauss-sum functional of the f det J train, which is within 10 eps of the
    # samples in the Frobenius norm (the bound the factor tests use); F is not rounded after
    # assembly, so each entry is within ||w B_a||_2 * 10 eps ||f det J|| of its definition
    fj_norm = ott.norm(assembled[4][6])
    bound = 10 * pr.options.tt_eps * fj_norm * csw
    say("fullsize F entries: max |diff| / bound", np.max(np.abs(gotF - refF) / bound))
    assert np.all(np.abs(gotF - refF) <= bound)
    assert np.abs(refF).max() > 0


def test_fullsize_factor_samples(assembled):
    """The seven factor TTs at 256 random Gauss points against the oracle's direct evaluation:
    the metric entries (exactly separable on the annulus) to 1e-10 of their largest sample,
    f det J within 10 eps of its norm spread over the grid (RMS per point)."""
    pr, _, _, _, fac = assembled
    nodes = [g[0] for g in geometry.gauss_grid(pr)]
    rng = np.random.default_rng(7)
    idx = [rng.integers(0, len(nodes[d]), size=256) for d in range(3)]
    pts = np.stack([nodes[d][idx[d]] for d in range(3)], axis=1)
    ref, _ = geometry.sample_factors_points(pr, pts)
    got = np.zeros_like(ref)
    for f in range(7):
        if fac[f] is None:
            continue
        for q in range(pts.shape[0]):
            v = np.ones((1,))
            for d in range(3):
                v = v @ fac[f][d][:, idx[d][q], :]
            got[f, q] = v[0]
    rmax = np.abs(ref[:6]).max()
    say("fullsize factors: metric max |diff|", np.abs(got[:6] - ref[:6]).max(), "of", rmax)
    assert np.abs(got[:6] - ref[:6]).max() <= 1e-10 * rmax
    npts = np.prod([len(x) for x in nodes])
    fnorm = ott.norm(fac[6])
    rms = np.sqrt(np.mean((got[6] - ref[6]) ** 2))
    say("fullsize factors: f det J RMS diff", rms, "allowed", 10 * pr.options.tt_eps * fnorm / np.sqrt(npts))
    assert rms <= 10 * pr.options.tt_eps * fnorm / np.sqrt(npts)


def test_fullsize_manufactured_solve(ctx):
    """The C2 discretisation (annulus, degree 3, n = 256, TT eps 1e-6, tol 1e-7) with the
    manufactured forcing of u = sin(pi r) sin(2 theta) sin(pi z) (a closed form chosen for this test: it vanishes on the six faces of the quarter annulus; its forcing is -Laplace u), solved through the
    executor beside three C2 Fourier problems as in the bench's steps: the TT solution at 300
    random points of the solid against u itself.  At this mesh the discretisation error
    (O(h^4), about 1e-9) is far below the tolerances, so what is measured is the TT solve;
    the gate is the relative accuracy the solves are held to, 1e-6 (RMS over the points,
    relative to the RMS of u)."""
    from oracle import nurbs, sources
    say("fullsize manufactured solve (4 lanes)")
    pr = W.c2_problem(n=256)
    pr.source = W.manufactured_annulus_source()
    batch = [pr] + [W.c2_problem(n=256, seed=W.configs.C2_SEED + b) for b in range(1, 4)]
    out = ctx.solve_batch(batch, lanes=4)
    res, cores = out[0]
    assert res["status"] == 0, res
    assert all(r["status"] == 0 for r, _ in out)
    rng = np.random.default_rng(11)
    pts = rng.uniform(0.0, 1.0, size=(300, 3))
    p = pr.disc.degree
    from oracle import tt_iga
    sl = tt_iga.interior_slices(pr)
    Bs = []
    for d in range(3):
        kn = bspline.open_uniform_knots(pr.disc.n_basis[d], p)
        Bs.append(bspline.basis(kn, p, pts[:, d])[:, sl[d]])
    v = Bs[0] @ cores[0][0]
    v = np.einsum("pa,anb,pn->pb", v, cores[1], Bs[1])
    uh = np.einsum("pb,bn,pn->p", v, cores[2][:, :, 0], Bs[2])
    x, _ = nurbs.solid_map_points(pr.geometry, pts)
    ue = sources.manufactured_annulus_solution(x)
    rms_err = np.sqrt(np.mean((uh - ue) ** 2))
    rms_u = np.sqrt(np.mean(ue ** 2))
    allowed = 1e-6 * rms_u
    say("fullsize manufactured: RMS error", rms_err, "max", np.abs(uh - ue).max(), "allowed RMS", allowed)
    assert rms_err <= allowed


@pytest.fixture(scope="module")
def c3_assembled():
    """The complex-geometry configuration at its full size: bumpy degree-3 NURBS cube (8^3 net,
    Gaussian bumps, weights U[0.8, 1.2]), n = 512 per direction (1.3e8 DOF, 2036 Gauss points
    per direction), TT eps 1e-6; assembled, then solved in FP64 (preconditioned TT-CG whose
    operator products are rounded as they are formed)."""
    from paper_2509_13224_amd import ttiga
    from workloads.problem import PREC_FP64
    say("fullsize C3 assembly")
    c = ttiga.Context(workspace_bytes=120 << 30)
    pr = W.c3_problem()
    pr.options.precision = PREC_FP64
    h = c.problem_create(pr, precond=1)
    st = h.assemble()
    say("fullsize C3 copy cores", st["compression_path"], st["rank_K"], st["min_detJ"])
    out = dict(pr=pr, st=st, K=h.tt(ttiga.WHICH_K), F=h.tt(ttiga.WHICH_F),
               fac=[h.tt(ttiga.WHICH_FACTOR0 + f) for f in range(7)], rhs=h.tt(ttiga.WHICH_RHS))
    say("fullsize C3 solve (about 40 s)")
    out["solve"] = h.solve()
    out["u"] = h.solution()
    say("fullsize C3 solved", out["solve"]["iterations"], out["solve"]["rank_u"], out["solve"]["rel_res"])
    h.close()
    return out


def _factor_values(fac, idx):
    got = np.zeros((7, len(idx[0])))
    for f in range(7):
        if fac[f] is None:
            continue
        for q in range(len(idx[0])):
            v = np.ones((1,))
            for d in range(3):
                v = v @ fac[f][d][:, idx[d][q], :]
            got[f, q] = v[0]
    return got


def test_c3_detj_and_factors(c3_assembled):
    """min det J over all 8.4e9 Gauss points is positive and no larger than det J at any of 512
    sampled points (oracle); the factor TTs at those points within 10 eps of their threshold
    scale spread over the grid (RMS per point), as the compression guarantees."""
    pr, st, fac = c3_assembled["pr"], c3_assembled["st"], c3_assembled["fac"]
    nodes = [g[0] for g in geometry.gauss_grid(pr)]
    rng = np.random.default_rng(13)
    idx = [rng.integers(0, len(nodes[d]), size=512) for d in range(3)]
    pts = np.stack([nodes[d][idx[d]] for d in range(3)], axis=1)
    ref, detj = geometry.sample_factors_points(pr, pts)
    assert 0.0 < st["min_detJ"] <= detj.min() * (1 + 1e-12)
    got = _factor_values(fac, idx)
    npts = float(np.prod([len(x) for x in nodes]))
    norms = [ott.norm(fac[f]) if fac[f] is not None else 0.0 for f in range(7)]
    scale = [max(norms[:6])] * 6 + [norms[6]]
    for f in range(7):
        rms = np.sqrt(np.mean((got[f] - ref[f]) ** 2))
        allowed = 10 * pr.options.tt_eps * scale[f] / np.sqrt(npts)
        say("fullsize C3 factor", f, "RMS diff", rms, "allowed", allowed)
        assert rms <= allowed


def test_c3_entries_within_bounds(c3_assembled):
    """Sampled entries of K^TT and F^TT against their definition.  K_ab is linear in the six
    metric factors and the sum of the nine terms is rounded at eps: |dK_ab| <= sum_ij
    ||w d_i phi_a d_j phi_b||_2 * 10 eps max ||R|| + eps ||K^TT||; F as for the annulus."""
    pr, K, F, fac = c3_assembled["pr"], c3_assembled["K"], c3_assembled["F"], c3_assembled["fac"]
    p, n = pr.disc.degree, pr.disc.n_basis[0]
    tabs = _tables(pr)
    eps = pr.options.tt_eps
    rnorm = max(ott.norm(fac[f]) for f in range(6) if fac[f] is not None)
    fj_norm = ott.norm(fac[6])
    k_norm = ott.norm([c.reshape(c.shape[0], -1, c.shape[-1]) for c in K])
    worst_k = worst_f = 0.0
    for a, b in _pairs(n, p, 12, 2025091303):
        sub, vals = [], []
        for d in range(3):
            nodes, wts, B, D = tabs[d]
            q = np.nonzero(((B[:, a[d]] != 0) | (D[:, a[d]] != 0)) & ((B[:, b[d]] != 0) | (D[:, b[d]] != 0)))[0]
            sub.append((nodes[q], wts[q]))
            vals.append((wts[q], B[q, a[d]], D[q, a[d]], B[q, b[d]], D[q, b[d]]))
        w = np.einsum("i,j,k->ijk", vals[0][0], vals[1][0], vals[2][0])
        g = [[np.einsum("i,j,k->ijk", *[vals[d][1 + 2 * s] if d != i else vals[d][2 + 2 * s] for d in range(3)])
              for i in range(3)] for s in range(2)]
        cs = sum(np.sqrt(np.sum((w * g[0][i] * g[1][j]) ** 2)) for i in range(3) for j in range(3))
        rk, rf, csf = _reference_entries(pr, tabs, a, b)
        dk = abs(_tt_matrix_entry(K, a, b, p) - rk)
        df = abs(_tt_vector_entry(F, a) - rf)
        bound_k = 10 * eps * rnorm * cs + eps * k_norm
        bound_f = 10 * eps * fj_norm * csf
        worst_k, worst_f = max(worst_k, dk / bound_k), max(worst_f, df / bound_f)
        assert dk <= bound_k and df <= bound_f, (a, b, dk, bound_k, df, bound_f)
    say("fullsize C3 entries: worst |dK| / bound", worst_k, "worst |dF| / bound", worst_f)


def test_c3_solution_residual_entries(c3_assembled):
    """The full-size complex-geometry solve against the oracle's discrete system, with a bound
    that uses nothing the solver reports: at 16 sampled interior rows a the oracle forms
    r_a = F_a - sum_b K_ab u_b from the definition (the 7^3 neighbouring entries of row a as
    Gauss sums over the support of a) and the GPU solution's coefficients u_b.  The RMS of these
    entries estimates ||F_I - K_II u|| / sqrt(N_I).  A solution within 10 (eps + tol) of the
    discrete one in the 2-norm has ||F_I - K_II u|| <= ||K_II|| 10 (eps + tol) ||u|| (plus what
    separates the eps-accurate K^TT and F^TT from the exact ones); ||K_II|| is estimated from the
    sampled absolute row sums (Gershgorin), ||u|| is computed from the TT.  The bound is a
    necessary condition (a smooth error of the same size leaves a smaller residual); the
    sufficient check against u_h is made at oracle size on the same path in
    test_gpu_timed_path.py."""
    pr, sol, u = c3_assembled["pr"], c3_assembled["solve"], c3_assembled["u"]
    p = pr.disc.degree
    eps, tol = pr.options.tt_eps, pr.options.rel_res_tol
    assert sol["status"] == 0 and sol["rel_pres"] <= tol
    tabs = _tables(pr)
    from oracle import tt_iga
    sl = tt_iga.interior_slices(pr)
    lo = [s.start for s in sl]
    n_interior = float(np.prod([s.stop - s.start for s in sl]))
    u_norm = ott.norm(u)
    rng = np.random.default_rng(17)
    r_rows, f_rows, row_sums = [], [], []
    for _ in range(16):
        a = tuple(int(rng.integers(s.start + p, s.stop - p)) for s in sl)
        sub, Ba, Da = [], [], []
        nb = [np.arange(a[d] - p, a[d] + p + 1) for d in range(3)]
        Bb, Db = [], []
        for d in range(3):
            nodes, wts, B, D = tabs[d]
            q = np.nonzero(B[:, a[d]] != 0)[0]
            sub.append((nodes[q], wts[q]))
            Ba.append(B[q, a[d]])
            Da.append(D[q, a[d]])
            Bb.append(B[np.ix_(q, nb[d])])
            Db.append(D[np.ix_(q, nb[d])])
        fac, _ = geometry.sample_factors_grid(pr, grid=sub)
        R = np.zeros((3, 3) + fac.shape[1:])
        for idx, (i, j) in enumerate(geometry.R_PAIRS):
            R[i, j] = fac[idx]
            R[j, i] = fac[idx]
        w = np.einsum("i,j,k->ijk", sub[0][1], sub[1][1], sub[2][1])
        ga = [np.einsum("i,j,k->ijk", *[Da[d] if d == i else Ba[d] for d in range(3)]) for i in range(3)]
        Krow = np.zeros((2 * p + 1,) * 3)
        for i in range(3):
            for j in range(3):
                g = w * ga[i] * R[i, j]
                mats = [Db[d] if d == j else Bb[d] for d in range(3)]
                Krow += np.einsum("xyz,xa,yb,zc->abc", g, *mats)
        F_a = np.sum(np.einsum("i,j,k->ijk", *[sub[d][1] * Ba[d] for d in range(3)]) * fac[6])
        ub = np.zeros((2 * p + 1,) * 3)
        for i0, b0 in enumerate(nb[0]):
            for i1, b1 in enumerate(nb[1]):
                for i2, b2 in enumerate(nb[2]):
                    v = u[0][:, b0 - lo[0], :] @ u[1][:, b1 - lo[1], :] @ u[2][:, b2 - lo[2], :]
                    ub[i0, i1, i2] = v[0, 0]
        r_rows.append(F_a - np.sum(Krow * ub))
        f_rows.append(F_a)
        row_sums.append(np.sum(np.abs(Krow)))
    res_est = np.sqrt(n_interior * np.mean(np.square(r_rows)))
    f_est = np.sqrt(n_interior * np.mean(np.square(f_rows)))
    k_est = max(row_sums)
    bound = 10 * (eps + tol) * k_est * u_norm + 10 * eps * f_est
    say("fullsize C3 residual: sampled ||r|| estimate", res_est, "bound", bound, "||F_I|| estimate", f_est,
        "||K_II|| estimate", k_est, "||u||", u_norm)
    assert res_est <= bound
