"""Tensor Gauss-Legendre quadrature on the knot spans of the solution space.

The paper integrates the 1-D factors of Section 4.2 over the parametric
domain; the rule is not stated, so g Gauss-Legendre points are placed on each
non-empty knot span (g = p+1 unless given), with weights scaled by half the
span length.
"""
import numpy as np


def gauss_points(knots, g):
    """Nodes and weights of g-point Gauss-Legendre rules on every non-empty span, in order."""
    knots = np.asarray(knots, dtype=np.float64)
    t, wt = np.polynomial.legendre.leggauss(g)
    breaks = np.unique(knots)
    nodes, weights = [], []
    for a, b in zip(breaks[:-1], breaks[1:]):
        nodes.append(0.5 * (a + b) + 0.5 * (b - a) * t)
        weights.append(0.5 * (b - a) * wt)
    return np.concatenate(nodes), np.concatenate(weights)
