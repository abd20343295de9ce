"""Accuracy of a discrete solution against an exact one (eq. L2norm of Section 5).

The printed formula integrates the unsquared error magnitude; ``l1_ratio``
returns that quantity and ``rel_l2`` the relative L2 norm
sqrt(int (u_h - u)^2 / int u^2).  Both use p+3 Gauss points per span on the
exact geometry, with dOmega = det J dxi.
"""
import numpy as np

from . import bspline, nurbs, quadrature


def _error_grid(problem, extra=3):
    p = problem.disc.degree
    out = []
    for d in range(3):
        kn = bspline.open_uniform_knots(problem.disc.n_basis[d], p)
        nodes, wts = quadrature.gauss_points(kn, p + extra)
        out.append((kn, nodes, wts))
    return out


def _volume_weights(grid, J):
    """Quadrature weight of each grid point in physical space: w0 w1 w2 det J."""
    return np.einsum("i,j,k->ijk", grid[0][2], grid[1][2], grid[2][2]) * np.linalg.det(J)


def _fields(problem, u_coeff, exact):
    p = problem.disc.degree
    grid = _error_grid(problem)
    B = [bspline.basis(kn, p, nodes) for kn, nodes, _ in grid]
    uh = np.einsum("abc,ia,jb,kc->ijk", u_coeff, B[0], B[1], B[2], optimize=True)
    x, J = nurbs.solid_map_grid(problem.geometry, grid[0][1], grid[1][1], grid[2][1])
    return uh, exact(x), _volume_weights(grid, J)


def rel_l2(problem, u_coeff, exact):
    uh, ue, W = _fields(problem, u_coeff, exact)
    return float(np.sqrt(np.sum(W * (uh - ue) ** 2) / np.sum(W * ue ** 2)))


def l1_ratio(problem, u_coeff, exact):
    uh, ue, W = _fields(problem, u_coeff, exact)
    return float(np.sum(W * np.abs(uh - ue)) / np.sum(W * np.abs(ue)))
