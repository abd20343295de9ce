"""Univariate B-spline basis (Section 2.1).

Zero-degree basis on half-open knot spans, the Cox-de Boor recursion for
degree p, and the derivative formula, all evaluated for every basis function
at once.  The convention 0/0 := 0 is used for repeated knots.  The right end
of the parameter range is assigned to the last non-empty span so that
N_{n-1}(1) = 1 for an open knot vector.
"""
import numpy as np


def open_uniform_knots(n, p):
    """Open knot vector with n basis functions of degree p: end multiplicity p+1, E = n-p spans."""
    if n < p + 1:
        raise ValueError("need n >= p + 1")
    E = n - p
    interior = [e / E for e in range(1, E)]
    return np.array([0.0] * (p + 1) + interior + [1.0] * (p + 1))


def _div(a, b):
    """a / b with the convention 0/0 := 0 (b is a knot difference, a scalar)."""
    return 0.0 if b == 0.0 else a / b


def basis_degree0(knots, xi):
    """N_i^0 at points xi: 1 on [knot_i, knot_{i+1}), right end closed on the last non-empty span."""
    knots = np.asarray(knots, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    m = len(knots) - 1
    N = np.zeros((len(xi), m))
    for i in range(m):
        N[:, i] = (knots[i] <= xi) & (xi < knots[i + 1])
    last = max(i for i in range(m) if knots[i] < knots[i + 1])
    N[xi == knots[-1], last] = 1.0
    return N


def basis(knots, p, xi):
    """All n = len(knots)-p-1 basis functions N_i^p at points xi, shape (len(xi), n)."""
    knots = np.asarray(knots, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    N = basis_degree0(knots, xi)
    for q in range(1, p + 1):
        m = N.shape[1] - 1
        Nq = np.zeros((len(xi), m))
        for i in range(m):
            left = _div(1.0, knots[i + q] - knots[i])
            right = _div(1.0, knots[i + q + 1] - knots[i + 1])
            Nq[:, i] = (xi - knots[i]) * left * N[:, i] + (knots[i + q + 1] - xi) * right * N[:, i + 1]
        N = Nq
    return N


def basis_derivative(knots, p, xi):
    """dN_i^p/dxi = p/(k_{i+p}-k_i) N_i^{p-1} - p/(k_{i+p+1}-k_{i+1}) N_{i+1}^{p-1}."""
    knots = np.asarray(knots, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(knots) - p - 1
    if p == 0:
        return np.zeros((len(xi), n))
    Nm = basis(knots, p - 1, xi)  # n + 1 functions of degree p-1
    dN = np.zeros((len(xi), n))
    for i in range(n):
        dN[:, i] = (p * _div(1.0, knots[i + p] - knots[i]) * Nm[:, i]
                    - p * _div(1.0, knots[i + p + 1] - knots[i + 1]) * Nm[:, i + 1])
    return dN


def greville(knots, p):
    """Greville abscissae (knot averages) of the n basis functions."""
    knots = np.asarray(knots, dtype=np.float64)
    n = len(knots) - p - 1
    if p == 0:
        return 0.5 * (knots[:-1] + knots[1:])[:n]
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n)])

