"""Plain data records for one TT-IGA problem (model problem of Section 3.1).

Conventions shared by every consumer:

* Parametric directions are numbered 0, 1, 2 (the paper's xi_1, xi_2, xi_3).
* Control nets are stored C-order ``[m0][m1][m2][3]``; weights ``[m0][m1][m2]``.
* A flattened degree of freedom index is ``(i0 * n1 + i1) * n2 + i2``
  (first direction slowest), the lexicographic order of Section 4.1.1.
* Dirichlet faces are ordered xi0=0, xi0=1, xi1=0, xi1=1, xi2=0, xi2=1.
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

SOURCE_ZERO = 0
SOURCE_MANUFACTURED_ANNULUS = 1
SOURCE_FOURIER = 2

BC_NATURAL = 0
BC_ZERO = 1
BC_CONSTANT = 2
BC_TRACTION = 3  # natural face with a constant outward normal derivative du/dn = value

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16 = 2


@dataclass
class Geometry:
    """Trivariate NURBS solid: degrees, open knot vectors, control points, weights."""

    degree: Sequence[int]
    knots: Sequence[np.ndarray]
    ctrl: np.ndarray  # [m0][m1][m2][3]
    weights: Optional[np.ndarray] = None  # [m0][m1][m2]; None means all ones (B-spline)

    @property
    def n_ctrl(self):
        return tuple(int(s) for s in self.ctrl.shape[:3])

    def weights_or_ones(self):
        if self.weights is None:
            return np.ones(self.ctrl.shape[:3])
        return np.asarray(self.weights, dtype=np.float64)


@dataclass
class Discretization:
    """Solution space: degree p, n basis per direction, g Gauss points per element."""

    degree: int
    n_basis: Sequence[int]
    n_gauss: int = 0  # 0 means degree + 1

    @property
    def g(self):
        return self.n_gauss if self.n_gauss > 0 else self.degree + 1


@dataclass
class Source:
    """Source term f of the Poisson problem.

    kind SOURCE_FOURIER: f(x) = sum_m a[m] * sin(pi * k[m] . (x - origin) / scale + phi[m]).
    kind SOURCE_MANUFACTURED_ANNULUS: the forcing of u = sin(pi r) sin(2 theta) sin(pi z)
    in cylindrical coordinates about the z axis.
    """

    kind: int = SOURCE_ZERO
    a: np.ndarray = field(default_factory=lambda: np.zeros(0))
    k: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    phi: np.ndarray = field(default_factory=lambda: np.zeros(0))
    origin: np.ndarray = field(default_factory=lambda: np.zeros(3))
    scale: float = 1.0


@dataclass
class Dirichlet:
    """Per-face boundary condition; face order xi0=0, xi0=1, xi1=0, xi1=1, xi2=0, xi2=1.

    BC_ZERO / BC_CONSTANT faces carry Dirichlet data u = value; BC_NATURAL and BC_TRACTION
    faces are natural boundaries (Section 3.1), the latter with the flux du/dn = value."""

    kind: Sequence[int] = (BC_ZERO,) * 6
    value: Sequence[float] = (0.0,) * 6


@dataclass
class Options:
    tt_eps: float = 1e-10
    rel_res_tol: float = 1e-10
    max_iter: int = 500
    max_rank: int = 256
    precision: int = PREC_FP64
    refine: int = 1
    sample_chunk_bytes: int = 0  # 0: automatic; > 0: stream the Gauss-grid sampling in chunks
    compression: int = 0  # 0: cross approximation where it pays, verified, TT-SVD fallback; 1: TT-SVD only
    assembly_eps: float = 0.0  # 0: tt_eps; > 0: tolerance of the assembly alone
    solver: int = 0  # 0: TT-CG (preconditioned per precond); 1: AMEn


@dataclass
class Problem:
    name: str
    geometry: Geometry
    disc: Discretization
    source: Source
    dirichlet: Dirichlet
    options: Options
