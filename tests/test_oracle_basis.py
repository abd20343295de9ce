"""Pins for the oracle's B-spline basis, NURBS map and quadrature (Sections 2.1-2.3)."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import workloads as W
from oracle import bspline, nurbs, quadrature

KNOT_CASES = [
    (bspline.open_uniform_knots(7, 2), 2),
    (bspline.open_uniform_knots(9, 3), 3),
    (bspline.open_uniform_knots(4, 1), 1),
    (np.array([0, 0, 0, 0.1, 0.4, 0.4, 0.7, 1, 1, 1.0]), 2),  # non-uniform, repeated interior knot
]


@pytest.mark.parametrize("knots,p", KNOT_CASES)
def test_partition_of_unity_and_derivative_sum(knots, p):
    xi = np.linspace(0, 1, 301)
    N = bspline.basis(knots, p, xi)
    dN = bspline.basis_derivative(knots, p, xi)
    assert np.max(np.abs(N.sum(axis=1) - 1)) < 1e-14
    inner = (xi > 0) & (xi < 1)
    assert np.max(np.abs(dN[inner].sum(axis=1))) < 1e-11
    assert N.min() >= -1e-15


@pytest.mark.parametrize("knots,p", KNOT_CASES)
def test_support(knots, p):
    xi = np.linspace(0, 1, 401)[:-1]
    N = bspline.basis(knots, p, xi)
    for i in range(N.shape[1]):
        outside = (xi < knots[i]) | (xi >= knots[i + p + 1])
        assert np.all(N[outside, i] == 0.0)


@pytest.mark.parametrize("knots,p", KNOT_CASES)
def test_against_scipy_bspline(knots, p):
    xi = np.linspace(0, 1, 257)[:-1]
    N = bspline.basis(knots, p, xi)
    dN = bspline.basis_derivative(knots, p, xi)
    n = len(knots) - p - 1
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        s = BSpline(knots, c, p, extrapolate=False)
        assert np.max(np.abs(s(xi) - N[:, i])) < 1e-14
        assert np.max(np.abs(s.derivative()(xi) - dN[:, i])) < 1e-11


@pytest.mark.parametrize("knots,p", KNOT_CASES)
def test_greville_linear_precision(knots, p):
    xi = np.linspace(0, 1, 201)
    N = bspline.basis(knots, p, xi)
    assert np.max(np.abs(N @ bspline.greville(knots, p) - xi)) < 1e-14


def test_open_knot_end_values():
    kn = bspline.open_uniform_knots(10, 3)
    N = bspline.basis(kn, 3, np.array([0.0, 1.0]))
    assert N[0, 0] == 1.0 and N[1, -1] == 1.0


def test_fig1_circle_is_exact():
    """Fig. 1 knot vector and weights give an exact unit circle."""
    p, kn, P, w = W.nurbs_circle_fig1()
    t = np.linspace(0, 1, 1001)
    C = nurbs.curve(kn, p, P, w, t)
    assert np.max(np.abs(np.linalg.norm(C, axis=1) - 1.0)) < 2e-16 * 8
    # first quarter: rational quadratic arc, theta(t) = pi/4 + 2 atan(tan(pi/8)(2s-1)), s = 4t
    s = np.linspace(0, 1, 101)
    Cq = nurbs.curve(kn, p, P, w, s / 4)
    theta = np.arctan2(Cq[:, 1], Cq[:, 0])
    expect = math.pi / 4 + 2 * np.arctan(math.tan(math.pi / 8) * (2 * s - 1))
    assert np.max(np.abs(theta - expect)) < 1e-14


def test_nurbs_basis_partition_and_derivative():
    p, kn, P, w = W.nurbs_circle_fig1()
    t = np.linspace(0.003, 0.997, 97)
    t = t[np.min(np.abs(t[:, None] - kn[None, :]), axis=1) > 1e-4]  # C0 knots: one-sided slopes
    R, dR = nurbs.nurbs_basis(kn, p, w, t)
    assert np.max(np.abs(R.sum(axis=1) - 1)) < 1e-15
    h = 1e-6
    Rp, _ = nurbs.nurbs_basis(kn, p, w, t + h)
    Rm, _ = nurbs.nurbs_basis(kn, p, w, t - h)
    fd = (Rp - Rm) / (2 * h)
    assert np.max(np.abs(fd - dR)) < 1e-6


@pytest.mark.parametrize("geo", [W.annulus_sector(), W.twisted_box(1.2), W.bumpy_cube()])
def test_solid_jacobian_against_finite_differences(geo):
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.05, 0.95, size=(40, 3))
    x, J = nurbs.solid_map_points(geo, pts)
    h = 1e-6
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        xp, _ = nurbs.solid_map_points(geo, pts + e)
        xm, _ = nurbs.solid_map_points(geo, pts - e)
        assert np.max(np.abs((xp - xm) / (2 * h) - J[..., i])) < 1e-7


def test_annulus_map_closed_form():
    geo = W.annulus_sector(1.0, 2.0, math.pi / 2, 1.0)
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, size=(50, 3))
    x, _ = nurbs.solid_map_points(geo, pts)
    r = np.hypot(x[:, 0], x[:, 1])
    assert np.max(np.abs(r - (1 + pts[:, 0]))) < 1e-14
    assert np.max(np.abs(x[:, 2] - pts[:, 2])) < 1e-15
    th = np.arctan2(x[:, 1], x[:, 0])
    expect = math.pi / 4 + 2 * np.arctan(math.tan(math.pi / 8) * (2 * pts[:, 1] - 1))
    assert np.max(np.abs(th - expect)) < 1e-14


@pytest.mark.parametrize("g", [1, 2, 3, 4, 5])
def test_gauss_exactness(g):
    kn = np.array([0, 0, 0, 0.13, 0.5, 0.5, 0.77, 1, 1, 1.0])
    x, w = quadrature.gauss_points(kn, g)
    assert len(x) == 4 * g
    for deg in range(2 * g):
        exact = 1.0 / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-14
    # degree 2g is not integrated exactly on a single span
    x1, w1 = quadrature.gauss_points(np.array([0.0, 1.0]), g)
    assert abs(np.sum(w1 * x1 ** (2 * g)) - 1.0 / (2 * g + 1)) > 1e-8
