"""Pins for the oracle's geometry factors, sparse K and F, and the direct solve (Section 3)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bspline, errors, geometry, nurbs, sources, sparse_iga
from workloads.problem import BC_CONSTANT, BC_NATURAL, BC_ZERO, Dirichlet


def _annulus_closed_form(pts, r_in=1.0, r_out=2.0, sweep=math.pi / 2, H=1.0):
    """a = (rho', rho theta', H): R = diag(a2 a3/a1, a1 a3/a2, a1 a2/a3), det J = a1 a2 a3."""
    tq = math.tan(sweep / 4)
    rho = r_in + (r_out - r_in) * pts[:, 0]
    dth = 4 * tq / (1 + tq ** 2 * (2 * pts[:, 1] - 1) ** 2)
    a1, a2, a3 = (r_out - r_in) * np.ones(len(pts)), rho * dth, H * np.ones(len(pts))
    return a1 * a2 * a3, np.stack([a2 * a3 / a1, a1 * a3 / a2, a1 * a2 / a3])


def test_annulus_factors_closed_form():
    pr = W.c1_problem()
    rng = np.random.default_rng(1)
    pts = rng.uniform(0, 1, size=(200, 3))
    fac, detJ = geometry.sample_factors_points(pr, pts)
    det_cf, Rdiag = _annulus_closed_form(pts)
    assert np.max(np.abs(detJ - det_cf) / det_cf) < 1e-14
    for i in range(3):
        assert np.max(np.abs(fac[i] - Rdiag[i]) / Rdiag[i]) < 1e-13
    assert np.max(np.abs(fac[3:6])) < 1e-14


def test_identity_cube_factors():
    geo = W.identity_cube()
    pr = W.small_problem(geo, 6, 3, W.zero_source())
    pts = np.random.default_rng(2).uniform(0, 1, size=(100, 3))
    fac, detJ = geometry.sample_factors_points(pr, pts)
    assert np.max(np.abs(detJ - 1)) < 1e-14
    assert np.max(np.abs(fac[:3] - 1)) < 1e-13 and np.max(np.abs(fac[3:6])) < 1e-13


def test_manufactured_forcing_matches_laplacian():
    """-Laplace of the manufactured solution by central differences equals the coded forcing."""
    rng = np.random.default_rng(4)
    r = rng.uniform(1.1, 1.9, 30)
    th = rng.uniform(0.1, 1.4, 30)
    z = rng.uniform(0.1, 0.9, 30)
    x = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)
    h = 1e-3
    lap = -6 * sources.manufactured_annulus_solution(x)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        lap += sources.manufactured_annulus_solution(x + e) + sources.manufactured_annulus_solution(x - e)
    lap /= h * h
    f = sources.evaluate(W.manufactured_annulus_source(), x)
    assert np.max(np.abs(-lap - f)) / np.max(np.abs(f)) < 1e-5


def test_volume_from_load_vector():
    """f = 1 gives sum_I F_I = vol = (pi/4)(r_out^2 - r_in^2) H by partition of unity."""
    pr = W.c1_problem(n=10)
    fac, detJ = geometry.sample_factors_grid(pr)
    fac[6] = detJ
    _, F = sparse_iga.assemble(pr, fac)
    assert abs(F.sum() - 0.75 * math.pi) < 1e-9


def one_d_matrices(n, p):
    kn = bspline.open_uniform_knots(n, p)
    from oracle import quadrature
    x, w = quadrature.gauss_points(kn, p + 1)
    B = bspline.basis(kn, p, x)
    D = bspline.basis_derivative(kn, p, x)
    m = B.T @ (w[:, None] * B)
    d = D.T @ (w[:, None] * D)
    c = D.T @ (w[:, None] * B)
    return kn, m, d, c


@pytest.mark.parametrize("n,p", [(5, 1), (8, 2), (11, 3)])
def test_one_d_matrix_identities(n, p):
    kn, m, d, c = one_d_matrices(n, p)
    assert np.max(np.abs(d.sum(axis=1))) < 1e-12
    assert abs(m.sum() - 1) < 1e-14
    assert np.max(np.abs(m.sum(axis=1) - (kn[p + 1:] - kn[:n]) / (p + 1))) < 1e-14
    E = np.zeros((n, n))
    E[-1, -1], E[0, 0] = 1.0, -1.0
    assert np.max(np.abs(c + c.T - E)) < 1e-12
    assert np.max(np.abs(c.sum(axis=0))) < 1e-12
    band = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) > p
    assert np.all(m[band] == 0) and np.all(d[band] == 0) and np.all(c[band] == 0)


@pytest.mark.parametrize("geo", [W.annulus_sector(), W.twisted_box(1.0), W.bumpy_cube()])
def test_stiffness_symmetric_zero_rowsum_spd(geo):
    pr = W.small_problem(geo, 6, 2, W.zero_source())
    K, _ = sparse_iga.assemble(pr)
    Kd = K.toarray()
    assert np.max(np.abs(Kd - Kd.T)) < 1e-13 * np.max(np.abs(Kd))
    assert np.max(np.abs(Kd.sum(axis=1))) < 1e-12 * np.max(np.abs(Kd))
    mask, _ = sparse_iga.dirichlet_values(pr)
    KII = Kd[~mask][:, ~mask]
    assert np.linalg.eigvalsh(KII).min() > 0


def test_identity_cube_is_kronecker_sum():
    n, p = 7, 3
    pr = W.small_problem(W.identity_cube(), n, p, W.zero_source())
    K, _ = sparse_iga.assemble(pr)
    _, m, d, _ = one_d_matrices(n, p)
    ref = np.kron(d, np.kron(m, m)) + np.kron(m, np.kron(d, m)) + np.kron(m, np.kron(m, d))
    assert np.max(np.abs(K.toarray() - ref)) < 1e-13


def greville_coefficients(pr, func):
    """Coefficients c with sum_I c_I N_I(xi) = func(x(xi)) by collocation at Greville points."""
    p = pr.disc.degree
    mats, pts = [], []
    for d in range(3):
        kn = bspline.open_uniform_knots(pr.disc.n_basis[d], p)
        g = bspline.greville(kn, p)
        mats.append(bspline.basis(kn, p, g))
        pts.append(g)
    x, _ = nurbs.solid_map_grid(pr.geometry, *pts)
    vals = func(x)
    c = np.einsum("ia,abc->ibc", np.linalg.inv(mats[0]), vals)
    c = np.einsum("jb,abc->ajc", np.linalg.inv(mats[1]), c)
    c = np.einsum("kc,abc->abk", np.linalg.inv(mats[2]), c)
    return c


@pytest.mark.parametrize("twist", [0.4, 1.5])
def test_patch_test_twisted_box(twist):
    """A linear field lies in every p>=3 space on the degree-(1,1,3) box: reproduced to round-off.

    K c reduces to the Gauss sum of grad N_I^T adj(J) a, a polynomial of degree 8 in xi_2
    here, so 5 Gauss points per span integrate it exactly.
    """
    pr = W.small_problem(W.twisted_box(twist), 6, 3, W.zero_source(), g=5)
    lin = lambda x: 1.0 + 2.0 * x[..., 0] - 3.0 * x[..., 1] + 0.5 * x[..., 2]
    c = greville_coefficients(pr, lin).ravel()
    K, _ = sparse_iga.assemble(pr)
    mask, _ = sparse_iga.dirichlet_values(pr)
    I, B = np.flatnonzero(~mask), np.flatnonzero(mask)
    Kd = K.toarray()
    uI = np.linalg.solve(Kd[np.ix_(I, I)], -Kd[np.ix_(I, B)] @ c[B])
    assert np.max(np.abs(uI - c[I])) < 1e-11


@pytest.mark.slow
def test_manufactured_convergence_rate_p2():
    """O(h^(p+1)) L2 convergence on the quarter annulus (p=2: slope about 3)."""
    ns = [8, 12, 16, 24]
    errs = []
    for n in ns:
        pr = W.c1_problem(n=n)
        u = sparse_iga.solve(pr)
        errs.append(errors.rel_l2(pr, u.reshape(n, n, n), sources.manufactured_annulus_solution))
    h = 1.0 / (np.array(ns) - 2)
    slope = np.polyfit(np.log(h), np.log(errs), 1)[0]
    assert 2.6 < slope < 3.6, (errs, slope)
    assert errs[-1] < 5e-5


def test_ring_laplace_log_solution():
    """Section 5.2 problem on a quarter ring: u = 1 at r_in, 2 at r_out, natural elsewhere."""
    errs = []
    for n in (6, 10):
        geo = W.annulus_sector(0.5, 1.0, math.pi / 2, 1.0)
        bc = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4,
                       value=(1.0, 2.0, 0, 0, 0, 0))
        pr = W.small_problem(geo, n, 2, W.zero_source(), dirichlet=bc)
        u = sparse_iga.solve(pr)
        exact = lambda x: sources.ring_log_solution(x, 0.5, 1.0, 1.0, 2.0)
        errs.append(errors.rel_l2(pr, u.reshape(n, n, n), exact))
    assert errs[1] < errs[0] / 4 and errs[1] < 1e-4


def test_lshape_geometry_volume_and_orientation():
    """The L-shape of Section 5.1 as one C0 patch: det J > 0 at every Gauss point and the volume
    (3 for height 1: the 2 x 2 square minus the unit cutout) from the load vector of f = 1."""
    pr = W.small_problem(W.lshape(), (9, 5, 3), 1, W.zero_source())
    fac, detJ = geometry.sample_factors_grid(pr)
    assert detJ.min() > 0.0
    fac[6] = detJ
    _, F = sparse_iga.assemble(pr, fac)
    assert abs(F.sum() - 3.0) < 1e-12


def test_lshape_forcing_matches_laplacian():
    """-Laplace of the L-shape solution by central differences equals sin(pi x) sin(pi y), and the
    two-mode Fourier source evaluates to the same function."""
    rng = np.random.default_rng(6)
    x = np.stack([rng.uniform(-0.9, 0.9, 40), rng.uniform(-0.9, -0.1, 40), rng.uniform(0.1, 0.9, 40)], axis=1)
    h = 1e-3
    lap = -6 * sources.lshape_solution(x)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        lap += sources.lshape_solution(x + e) + sources.lshape_solution(x - e)
    lap /= h * h
    f_exact = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    assert np.max(np.abs(-lap - f_exact)) < 1e-6
    assert np.max(np.abs(sources.evaluate(W.sine_xy_source(), x) - f_exact)) < 1e-14


@pytest.mark.slow
def test_lshape_linear_convergence_rate():
    """Section 5.1 with linear B-splines, homogeneous Dirichlet on the lateral faces and natural
    faces at z = 0, 1 (reading of the garbled boundary sentence): the L2 error against
    sin(pi x) sin(pi y) / (2 pi^2) decays with slope about 2 in the points per edge."""
    bc = Dirichlet(kind=(BC_ZERO,) * 4 + (BC_NATURAL,) * 2, value=(0.0,) * 6)
    errs, ns = [], [(9, 5, 2), (17, 9, 2), (33, 17, 2)]
    for nb in ns:
        pr = W.small_problem(W.lshape(), nb, 1, W.sine_xy_source(), dirichlet=bc)
        u = sparse_iga.solve(pr)
        errs.append(errors.rel_l2(pr, u.reshape(nb), sources.lshape_solution))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log((ns[i + 1][1] - 1) / (ns[i][1] - 1)) for i in range(2)]
    assert 1.7 < slopes[-1] < 2.3, (errs, slopes)


def test_full_ring_volume_and_log_solution():
    """The full ring of Section 5.2 (r 0.5..1, height 1, nine-point circle with C0 knots): volume
    pi (r_out^2 - r_in^2) h from f = 1, and the radial Laplace solution with u = 1 / 2 on the
    cylinders (natural seam and end faces) within the discretisation error, decreasing with n."""
    pr = W.small_problem(W.ring(), (3, 10, 3), 2, W.zero_source())
    fac, detJ = geometry.sample_factors_grid(pr)
    assert detJ.min() > 0.0
    fac[6] = detJ
    _, F = sparse_iga.assemble(pr, fac)
    assert abs(F.sum() - math.pi * 0.75) < 1e-3  # the rational circle is exact; quadrature is not
    bc = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    exact = lambda x: sources.ring_log_solution(x, 0.5, 1.0, 1.0, 2.0)
    errs = []
    for nb in ((4, 9, 3), (7, 9, 3)):
        pr = W.small_problem(W.ring(), nb, 2, W.zero_source(), dirichlet=bc)
        u = sparse_iga.solve(pr)
        errs.append(errors.rel_l2(pr, u.reshape(nb), exact))
    assert errs[1] < errs[0] / 4 and errs[1] < 1e-4, errs


def test_traction_load_integrates_the_face_area():
    """A unit flux on a face gives sum_a F_a = the face's area (partition of unity): on the
    quarter annulus r 1..2, 90 degrees, height 1 the outer cylinder (xi0 = 1) has area pi, the
    inner pi / 2, the flat end xi2 = 1 the quarter ring 3 pi / 4."""
    from workloads.problem import BC_TRACTION
    for face, area in ((1, math.pi), (0, math.pi / 2), (5, 0.75 * math.pi)):
        kind = [BC_NATURAL] * 6
        kind[face] = BC_TRACTION
        val = [0.0] * 6
        val[face] = 1.0
        pr = W.small_problem(W.annulus_sector(), (5, 7, 4), 2, W.zero_source(),
                             dirichlet=Dirichlet(kind=tuple(kind), value=tuple(val)))
        Fs = sparse_iga.traction_load(pr)
        # the arc's length element is rational, so the Gauss rule is accurate, not exact
        assert abs(Fs.sum() - area) <= 1e-6 * area, (face, Fs.sum(), area)
        assert np.all(Fs.reshape(5, 7, 4)[tuple(slice(None) if d != face // 2 else (0 if face % 2 == 0 else -1)
                                                for d in range(3))] >= 0.0)


def test_ring_with_traction_reaches_the_log_solution():
    """Dirichlet u = 1 at r = 1 and the flux du/dr = 1 / (r_out ln 2) at r = 2 (Section 5.2's
    radial solution with its outer condition written as a traction): the solution converges to
    u = 1 + ln(r) / ln 2, the same log solution as with u = 2 there."""
    from workloads.problem import BC_TRACTION
    g = 1.0 / (2.0 * math.log(2.0))
    bc = Dirichlet(kind=(BC_CONSTANT, BC_TRACTION) + (BC_NATURAL,) * 4, value=(1.0, g, 0, 0, 0, 0))
    exact = lambda x: sources.ring_log_solution(x, 1.0, 2.0, 1.0, 2.0)
    errs = []
    for nb in ((4, 4, 3), (8, 4, 3)):
        pr = W.small_problem(W.annulus_sector(), nb, 2, W.zero_source(), dirichlet=bc)
        u = sparse_iga.solve(pr)
        errs.append(errors.rel_l2(pr, u.reshape(nb), exact))
    assert errs[1] < errs[0] / 5 and errs[1] < 1e-4, errs
