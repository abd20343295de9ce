"""Seeded, synthetic problem descriptions shared by the oracle and the HIP path.

This package only *describes* inputs: control nets, weights, knot vectors,
source-term parameters, boundary data, tolerances and random TT cores for
operator tests.  It performs none of the method's arithmetic (no basis
evaluation, no geometry map, no quadrature, no TT algebra); both the oracle
and the HIP library evaluate everything from these descriptions on their own.

Geometry follows the NURBS solid description of Section 2.3 (control points,
weights, open knot vectors with end multiplicity p+1); the discretisation
follows Section 3.3 (B-spline solution space of degree p with n basis
functions per direction, obtained by h-refinement); the source term and the
Dirichlet data follow the model problem of Section 3.1.
"""
from .problem import (  # noqa: F401
    Geometry,
    Discretization,
    Source,
    Dirichlet,
    Options,
    Problem,
    SOURCE_ZERO,
    SOURCE_MANUFACTURED_ANNULUS,
    SOURCE_FOURIER,
    BC_NATURAL,
    BC_ZERO,
    BC_CONSTANT,
    BC_TRACTION,
    PREC_FP64,
    PREC_FP32,
    PREC_BF16,
)
from .geometries import (  # noqa: F401
    annulus_sector,
    twisted_box,
    bumpy_cube,
    identity_cube,
    lshape,
    nurbs_circle_fig1,
    ring,
)
from .sources import (  # noqa: F401
    fourier_source,
    manufactured_annulus_source,
    sine_product_source,
    sine_xy_source,
    zero_source,
)
from .configs import c1_problem, c2_problem, c3_problem, c4_requests, small_problem  # noqa: F401
