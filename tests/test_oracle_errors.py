"""Pins for the oracle's accuracy measures (eq. L2norm of Section 5) and its condition estimate.

The error integrals are pinned by closed forms on geometries where the integrand is a
polynomial that the p+3-point Gauss rule integrates exactly:

* quarter annulus (radii 1..2, sweep pi/2, height 1): x = rho(xi_0) C(xi_1) + xi_2 e_z with
  rho = 1 + xi_0 linear, so dOmega = r dr dtheta dz.  The discrete field u_h(xi) = xi_0 (the
  Greville abscissae as coefficients: linear precision) is r - 1 in physical space; against
  the exact function 1 the squared error integrand (r - 2)^2 r and the weight r are
  polynomials in xi_0, and the angular and vertical factors cancel from the ratios:
      rel_l2^2 = int_1^2 (r - 2)^2 r dr / int_1^2 r dr = (5/12) / (3/2) = 5/18,
      l1_ratio = int_1^2 (2 - r) r dr / int_1^2 r dr  = (2/3)  / (3/2) = 4/9.
* identity cube: u_h(xi) = xi_0 + c against the exact x_0 has the constant error c, so
      rel_l2 = |c| / sqrt(int x^2) = |c| sqrt(3),   l1_ratio = |c| / int |x| = 2 |c|.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bspline, errors, sparse_iga


def _greville_field(pr, d, offset=0.0):
    """Coefficients of u_h(xi) = xi_d + offset (linear precision of the Greville abscissae)."""
    p = pr.disc.degree
    n = pr.disc.n_basis
    g = bspline.greville(bspline.open_uniform_knots(n[d], p), p)
    shape = [1, 1, 1]
    shape[d] = n[d]
    return np.broadcast_to(g.reshape(shape), tuple(n)).copy() + offset


def _annulus(n=6, p=2):
    return W.small_problem(W.annulus_sector(1.0, 2.0, math.pi / 2, 1.0), n, p, W.zero_source())


def test_error_measures_annulus_closed_form():
    pr = _annulus()
    uh = _greville_field(pr, 0)
    one = lambda x: np.ones(x.shape[:-1])
    assert abs(errors.rel_l2(pr, uh, one) - math.sqrt(5.0 / 18.0)) < 1e-13
    assert abs(errors.l1_ratio(pr, uh, one) - 4.0 / 9.0) < 1e-13


@pytest.mark.parametrize("c", [1e-2, -3e-5])
def test_error_measures_identity_cube_constant_offset(c):
    pr = W.small_problem(W.identity_cube(), 5, 3, W.zero_source())
    uh = _greville_field(pr, 0, offset=c)
    x0 = lambda x: x[..., 0]
    assert abs(errors.rel_l2(pr, uh, x0) / (abs(c) * math.sqrt(3.0)) - 1) < 1e-10
    assert abs(errors.l1_ratio(pr, uh, x0) / (2 * abs(c)) - 1) < 1e-10


def test_error_measures_of_zero_field_are_one():
    pr = W.small_problem(W.bumpy_cube(), 6, 3, W.zero_source())
    f = lambda x: 1.0 + np.sin(x[..., 0]) * x[..., 1] ** 2
    zero = np.zeros(tuple(pr.disc.n_basis))
    assert abs(errors.rel_l2(pr, zero, f) - 1) < 1e-15
    assert abs(errors.l1_ratio(pr, zero, f) - 1) < 1e-15


def test_planted_dropped_detj_weight_is_caught(monkeypatch):
    """Integrating in parameter space (det J left out) gives sqrt(1/3), not sqrt(5/18)."""
    def no_detj(grid, J):
        return np.einsum("i,j,k->ijk", grid[0][2], grid[1][2], grid[2][2])

    monkeypatch.setattr(errors, "_volume_weights", no_detj)
    pr = _annulus()
    val = errors.rel_l2(pr, _greville_field(pr, 0), lambda x: np.ones(x.shape[:-1]))
    assert abs(val - math.sqrt(5.0 / 18.0)) > 1e-2
    assert abs(val - math.sqrt(1.0 / 3.0)) < 1e-13


@pytest.mark.parametrize("geo,n,p", [(W.annulus_sector(), 8, 2), (W.twisted_box(0.8), 7, 3)])
def test_condition_estimate_matches_dense_eigenvalues(geo, n, p):
    pr = W.small_problem(geo, n, p, W.zero_source())
    _, sysd = sparse_iga.solve(pr, return_system=True)
    lam = np.linalg.eigvalsh(sysd["KII"].toarray())
    assert abs(sparse_iga.condition_estimate(sysd["KII"]) / (lam[-1] / lam[0]) - 1) < 1e-8
