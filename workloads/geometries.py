"""Control nets of the synthetic geometries (NURBS solids of Section 2.3).

Only control points, weights and knot vectors are produced here.
"""
import math

import numpy as np

from .problem import Geometry


def _open_knots(degree, interior=()):
    return np.array([0.0] * (degree + 1) + list(interior) + [1.0] * (degree + 1))


def annulus_sector(r_in=1.0, r_out=2.0, sweep=math.pi / 2, height=1.0):
    """Thick annular sector extruded along z: degree (1, 2, 1), one element.

    Direction 0 is radial (r_in -> r_out), direction 1 angular (0 -> sweep)
    as a single rational quadratic arc whose middle weight is cos(sweep/2)
    (for sweep = pi/2 this is one quarter of the circle of Fig. 1), and
    direction 2 is the height 0 -> height.
    """
    half = 0.5 * sweep
    arc = [(1.0, 0.0), (1.0, math.tan(half)), (math.cos(sweep), math.sin(sweep))]
    w_arc = [1.0, math.cos(half), 1.0]
    ctrl = np.zeros((2, 3, 2, 3))
    wts = np.zeros((2, 3, 2))
    for a, rho in enumerate((r_in, r_out)):
        for b, (cx, cy) in enumerate(arc):
            for c, z in enumerate((0.0, height)):
                ctrl[a, b, c] = (rho * cx, rho * cy, z)
                wts[a, b, c] = w_arc[b]
    knots = [_open_knots(1), _open_knots(2), _open_knots(1)]
    return Geometry(degree=(1, 2, 1), knots=knots, ctrl=ctrl, weights=wts)


def twisted_box(twist=0.5 * math.pi):
    """Box [-1/2, 1/2]^2 x [0, 1] twisted about z: B-spline of degree (1, 1, 3).

    The 2 x 2 x 4 net places the corners of the square rotated by twist * z_c
    at the Greville heights z_c = 0, 1/3, 2/3, 1.  All weights are one, and the
    single Bezier element makes the map a polynomial of degree (1, 1, 3).
    """
    ctrl = np.zeros((2, 2, 4, 3))
    for a in range(2):
        for b in range(2):
            x0, y0 = a - 0.5, b - 0.5
            for c in range(4):
                z = c / 3.0
                ang = twist * z
                ctrl[a, b, c] = (x0 * math.cos(ang) - y0 * math.sin(ang),
                                 x0 * math.sin(ang) + y0 * math.cos(ang), z)
    knots = [_open_knots(1), _open_knots(1), _open_knots(3)]
    return Geometry(degree=(1, 1, 3), knots=knots, ctrl=ctrl, weights=None)


def lshape(height=1.0):
    """The L-shaped solid of Section 5.1: [-1, 1]^2 x [0, height] with [0, 1]^2 x [0, height]
    removed, as one bilinear-by-linear B-spline patch with a C0 knot.

    Direction 0 runs along the L through its corner (knots {0, 0, 1/2, 1, 1}, the kink of the
    map at 1/2): cross-sections from the end of the left leg (outer point (-1, 1), inner (0, 1))
    through the corner ((-1, -1) to (0, 0)) to the end of the lower leg ((1, -1) to (1, 0)).
    Direction 1 runs across the leg from the outer side to the inner (re-entrant) side, which
    makes det J positive, direction 2 along the height.  Both halves are bilinear quadrilaterals: the left leg minus
    the triangle (0, 0), (0, -1), (-1, -1), and the lower leg plus that triangle.
    """
    sections = [((-1.0, 1.0), (0.0, 1.0)), ((-1.0, -1.0), (0.0, 0.0)), ((1.0, -1.0), (1.0, 0.0))]
    ctrl = np.zeros((3, 2, 2, 3))
    for a, sec in enumerate(sections):
        for b, (x, y) in enumerate(sec):
            for c, z in enumerate((0.0, height)):
                ctrl[a, b, c] = (x, y, z)
    knots = [_open_knots(1, (0.5,)), _open_knots(1), _open_knots(1)]
    return Geometry(degree=(1, 1, 1), knots=knots, ctrl=ctrl, weights=None)


def ring(r_in=0.5, r_out=1.0, height=1.0):
    """The full ring of Section 5.2: radii r_in..r_out, height 0..height, as one NURBS patch.

    Direction 0 is radial, direction 1 goes once around the circle (the standard nine-point
    rational quadratic circle: knots {0, 0, 0, 1/4, 1/4, 1/2, 1/2, 3/4, 3/4, 1, 1, 1}, corner
    weights 1, edge-midpoint weights 1/sqrt(2)), direction 2 the height.  The faces xi1 = 0 and
    xi1 = 1 meet at the seam theta = 0; they are left natural, which is exact for data and
    solutions that do not depend on the angle.
    """
    circ = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)]
    w_c = [1.0 if i % 2 == 0 else 1.0 / math.sqrt(2.0) for i in range(9)]
    ctrl = np.zeros((2, 9, 2, 3))
    wts = np.zeros((2, 9, 2))
    for a, rho in enumerate((r_in, r_out)):
        for b, (cx, cy) in enumerate(circ):
            for c, z in enumerate((0.0, height)):
                ctrl[a, b, c] = (rho * cx, rho * cy, z)
                wts[a, b, c] = w_c[b]
    knots = [_open_knots(1), _open_knots(2, (0.25, 0.25, 0.5, 0.5, 0.75, 0.75)), _open_knots(1)]
    return Geometry(degree=(1, 2, 1), knots=knots, ctrl=ctrl, weights=wts)


CUBE_KNOTS_P3 = (0.2, 0.4, 0.6, 0.8)
CUBE_GREVILLE_P3 = (0.0, 1.0 / 15.0, 0.2, 0.4, 0.6, 0.8, 14.0 / 15.0, 1.0)


def identity_cube():
    """Unit cube as a degree-3 B-spline with control points at the Greville abscissae."""
    g = np.array(CUBE_GREVILLE_P3)
    ctrl = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).copy()
    knots = [_open_knots(3, CUBE_KNOTS_P3) for _ in range(3)]
    return Geometry(degree=(3, 3, 3), knots=knots, ctrl=ctrl, weights=None)


def bumpy_cube(seed=2025_0913_03, n_bumps=6, amp=0.05, width=0.2, w_lo=0.8, w_hi=1.2):
    """Degree-3 NURBS solid: the 8^3 Greville net of the unit cube displaced by Gaussian bumps.

    Each control point P moves by sum_b amp * v_b * exp(-|P - c_b|^2 / (2 width^2)),
    with centres c_b ~ U[0,1]^3 and unit directions v_b; weights ~ U[w_lo, w_hi].
    """
    rng = np.random.default_rng(seed)
    base = identity_cube()
    centres = rng.uniform(0.0, 1.0, size=(n_bumps, 3))
    dirs = rng.normal(size=(n_bumps, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    P = base.ctrl.copy()
    disp = np.zeros_like(P)
    for b in range(n_bumps):
        d2 = np.sum((P - centres[b]) ** 2, axis=-1)
        disp += amp * np.exp(-d2 / (2.0 * width * width))[..., None] * dirs[b]
    wts = rng.uniform(w_lo, w_hi, size=P.shape[:3])
    return Geometry(degree=(3, 3, 3), knots=base.knots, ctrl=P + disp, weights=wts)


def nurbs_circle_fig1():
    """The full circle of Fig. 1: quadratic NURBS with 9 control points on the unit square.

    Returns (degree, knots, control points [9][2], weights [9]).
    """
    knots = np.array([0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1], dtype=np.float64)
    s = 1.0 / math.sqrt(2.0)
    w = np.array([1, s, 1, s, 1, s, 1, s, 1], dtype=np.float64)
    P = np.array([(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)],
                 dtype=np.float64)
    return 2, knots, P, w
