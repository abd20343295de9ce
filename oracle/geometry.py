"""Geometry factors at quadrature points (Section 3.3).

J = d x / d xi, J = det J, and the metric factor R = J^-1 J^-T det J
(eq. Rxi), whose entries R_ij weight the stiffness terms K_ij
(eq. K_sum9_matrix_form), together with f(x(xi)) det J for the load vector
(eq. ffinal).  Physical gradients are grad_x N = J^-T grad_xi N.
"""
import numpy as np

from . import nurbs, quadrature, sources

# Unique entries of the symmetric R, in the order used for the TT factors.
R_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def factors_from_jacobian(J):
    """det J and R = det J * J^-1 J^-T from Jacobians (..., 3, 3)."""
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    R = detJ[..., None, None] * (Jinv @ np.swapaxes(Jinv, -1, -2))
    return detJ, R


def gauss_grid(problem):
    """Gauss nodes and weights per direction for the solution knots of the problem."""
    from . import bspline
    p = problem.disc.degree
    out = []
    for d in range(3):
        kn = bspline.open_uniform_knots(problem.disc.n_basis[d], p)
        out.append(quadrature.gauss_points(kn, problem.disc.g))
    return out


def sample_factors_grid(problem, grid=None):
    """The seven factor tensors on the Gauss grid: R_00, R_11, R_22, R_01, R_02, R_12, f det J.

    Returns (factors (7, Q0, Q1, Q2), detJ (Q0, Q1, Q2)).
    """
    if grid is None:
        grid = gauss_grid(problem)
    x, J = nurbs.solid_map_grid(problem.geometry, grid[0][0], grid[1][0], grid[2][0])
    detJ, R = factors_from_jacobian(J)
    f = sources.evaluate(problem.source, x)
    out = [R[..., i, j] for (i, j) in R_PAIRS] + [f * detJ]
    return np.stack(out), detJ


def sample_factors_points(problem, pts):
    """The seven factors at scattered parametric points (N, 3): shape (7, N), plus det J."""
    x, J = nurbs.solid_map_points(problem.geometry, pts)
    detJ, R = factors_from_jacobian(J)
    f = sources.evaluate(problem.source, x)
    return np.stack([R[:, i, j] for (i, j) in R_PAIRS] + [f * detJ]), detJ
