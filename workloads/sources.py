"""Source-term descriptions for the model problem of Section 3.1 (parameters only)."""
import numpy as np

from .problem import SOURCE_FOURIER, SOURCE_MANUFACTURED_ANNULUS, SOURCE_ZERO, Source


def zero_source():
    return Source(kind=SOURCE_ZERO)


def manufactured_annulus_source():
    """Forcing whose exact solution is u = sin(pi r) sin(2 theta) sin(pi z)."""
    return Source(kind=SOURCE_MANUFACTURED_ANNULUS)


def fourier_source(geometry, seed, n_modes=8, k_max=4):
    """f(x) = sum_m a_m sin(pi k_m . (x - origin)/scale + phi_m).

    k_m is drawn from {0..k_max}^3 without the zero vector, a_m = z_m / |k_m|^2 with
    z_m ~ N(0, 1), phi_m ~ U[0, 2 pi).  origin and scale are the lower corner and the
    largest extent of the control net's bounding box (which contains the solid).
    """
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(0, k_max + 1, size=3)
        if np.any(k):
            ks.append(k)
    k = np.array(ks, dtype=np.float64)
    z = rng.normal(size=n_modes)
    a = z / np.sum(k * k, axis=1)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    pts = geometry.ctrl.reshape(-1, 3)
    lo = pts.min(axis=0)
    scale = float(np.max(pts.max(axis=0) - lo))
    return Source(kind=SOURCE_FOURIER, a=a, k=k, phi=phi, origin=lo, scale=scale)


def sine_product_source():
    """f = sin(pi x) sin(pi y) sin(pi z), written as four Fourier modes.

    sin A sin B sin C = (sin(C+A-B) + sin(C-A+B) - sin(C+A+B) - sin(C-A-B)) / 4.
    """
    k = np.array([[1, -1, 1], [-1, 1, 1], [1, 1, 1], [-1, -1, 1]], dtype=np.float64)
    a = np.array([0.25, 0.25, -0.25, -0.25])
    return Source(kind=SOURCE_FOURIER, a=a, k=k, phi=np.zeros(4), origin=np.zeros(3), scale=1.0)


def sine_xy_source():
    """f = sin(pi x) sin(pi y) (the L-shape experiment of Section 5.1), as two Fourier modes:
    sin A sin B = (sin(A - B + pi/2) - sin(A + B + pi/2)) / 2."""
    k = np.array([[1, -1, 0], [1, 1, 0]], dtype=np.float64)
    a = np.array([0.5, -0.5])
    return Source(kind=SOURCE_FOURIER, a=a, k=k, phi=np.full(2, 0.5 * np.pi), origin=np.zeros(3), scale=1.0)
