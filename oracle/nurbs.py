"""NURBS curves and solids (Section 2.3), evaluated in homogeneous form.

A NURBS point is the weighted B-spline sum of w P divided by the weighted sum
of the basis, x = (sum N w P) / (sum N w).  Parametric derivatives follow the
quotient rule of the univariate NURBS basis derivative, lifted to the map:
d x / d xi_i = (d X / d xi_i - x d W / d xi_i) / W, with X = sum N w P and
W = sum N w.  The solid is the trivariate tensor product of Section 2.2.
"""
import numpy as np

from . import bspline


def nurbs_basis(knots, p, w, xi):
    """Univariate rational basis R_i = N_i w_i / W and its derivative (Section 2.3)."""
    N = bspline.basis(knots, p, xi)
    dN = bspline.basis_derivative(knots, p, xi)
    W = N @ w
    dW = dN @ w
    R = N * w / W[:, None]
    dR = (dN * w * W[:, None] - N * w * dW[:, None]) / (W[:, None] ** 2)
    return R, dR


def curve(knots, p, ctrl, w, t):
    """NURBS curve C(t) = sum N_i w_i P_i / sum N_i w_i."""
    N = bspline.basis(knots, p, t)
    W = N @ w
    return (N * w) @ ctrl / W[:, None]


def solid_map_grid(geometry, xi0, xi1, xi2):
    """Map x and Jacobian J[k, i] = d x_k / d xi_i on the tensor grid xi0 x xi1 x xi2.

    Returns x with shape (Q0, Q1, Q2, 3) and J with shape (Q0, Q1, Q2, 3, 3).
    """
    pg = geometry.degree
    B = [bspline.basis(geometry.knots[d], pg[d], x) for d, x in enumerate((xi0, xi1, xi2))]
    D = [bspline.basis_derivative(geometry.knots[d], pg[d], x)
         for d, x in enumerate((xi0, xi1, xi2))]
    w = geometry.weights_or_ones()
    Pw = np.concatenate([geometry.ctrl * w[..., None], w[..., None]], axis=-1)  # (X, W)
    H = np.einsum("ia,jb,kc,abcs->ijks", B[0], B[1], B[2], Pw, optimize=True)
    dH = [np.einsum("ia,jb,kc,abcs->ijks", D[0], B[1], B[2], Pw, optimize=True),
          np.einsum("ia,jb,kc,abcs->ijks", B[0], D[1], B[2], Pw, optimize=True),
          np.einsum("ia,jb,kc,abcs->ijks", B[0], B[1], D[2], Pw, optimize=True)]
    W = H[..., 3:4]
    x = H[..., :3] / W
    J = np.stack([(dH[i][..., :3] - x * dH[i][..., 3:4]) / W for i in range(3)], axis=-1)
    return x, J


def solid_map_points(geometry, pts):
    """Map x and Jacobian at scattered parametric points pts (N, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    pg = geometry.degree
    B = [bspline.basis(geometry.knots[d], pg[d], pts[:, d]) for d in range(3)]
    D = [bspline.basis_derivative(geometry.knots[d], pg[d], pts[:, d]) for d in range(3)]
    w = geometry.weights_or_ones()
    Pw = np.concatenate([geometry.ctrl * w[..., None], w[..., None]], axis=-1)
    H = np.einsum("qa,qb,qc,abcs->qs", B[0], B[1], B[2], Pw)
    dH = [np.einsum("qa,qb,qc,abcs->qs", D[0], B[1], B[2], Pw),
          np.einsum("qa,qb,qc,abcs->qs", B[0], D[1], B[2], Pw),
          np.einsum("qa,qb,qc,abcs->qs", B[0], B[1], D[2], Pw)]
    W = H[:, 3:4]
    x = H[:, :3] / W
    J = np.stack([(dH[i][:, :3] - x * dH[i][:, 3:4]) / W for i in range(3)], axis=-1)
    return x, J
