"""Source terms f(x) of the Poisson problem (Section 3.1) and exact solutions used as pins."""
import numpy as np

from workloads.problem import SOURCE_FOURIER, SOURCE_MANUFACTURED_ANNULUS, SOURCE_ZERO


def evaluate(source, x):
    """f at physical points x (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    if source.kind == SOURCE_ZERO:
        return np.zeros(x.shape[:-1])
    if source.kind == SOURCE_MANUFACTURED_ANNULUS:
        r = np.sqrt(x[..., 0] ** 2 + x[..., 1] ** 2)
        th = np.arctan2(x[..., 1], x[..., 0])
        radial = (2.0 * np.pi ** 2 + 4.0 / r ** 2) * np.sin(np.pi * r) - (np.pi / r) * np.cos(np.pi * r)
        return radial * np.sin(2.0 * th) * np.sin(np.pi * x[..., 2])
    if source.kind == SOURCE_FOURIER:
        xh = (x - np.asarray(source.origin)) / source.scale
        f = np.zeros(x.shape[:-1])
        for a, k, ph in zip(source.a, source.k, source.phi):
            f += a * np.sin(np.pi * (xh @ np.asarray(k)) + ph)
        return f
    raise ValueError("unknown source kind")


def manufactured_annulus_solution(x):
    """u = sin(pi r) sin(2 theta) sin(pi z), the exact solution paired with the forcing above."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(x[..., 0] ** 2 + x[..., 1] ** 2)
    th = np.arctan2(x[..., 1], x[..., 0])
    return np.sin(np.pi * r) * np.sin(2.0 * th) * np.sin(np.pi * x[..., 2])


def ring_log_solution(x, r_in, r_out, u_in, u_out):
    """Radial Laplace solution between two cylinders (Section 5.2)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(x[..., 0] ** 2 + x[..., 1] ** 2)
    return (u_in * np.log(r_out / r) + u_out * np.log(r / r_in)) / np.log(r_out / r_in)


def lshape_solution(x):
    """u = sin(pi x) sin(pi y) / (2 pi^2), the exact solution of the L-shape experiment
    (Section 5.1) for f = sin(pi x) sin(pi y): it vanishes on the lateral faces of the L
    (x or y in {-1, 0, 1}) and does not depend on z (natural faces at z = 0 and z = 1)."""
    x = np.asarray(x, dtype=np.float64)
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) / (2.0 * np.pi ** 2)
