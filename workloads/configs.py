"""The benchmark workloads as seeded problem descriptions.

* quarter annulus, p=2, n=16 (4,096 DOF), manufactured solution, eps 1e-10 (plain FP64 case);
* quarter annulus, p=3, n=256 (16.7M DOF), 8 seeded Fourier modes, eps 1e-6 (plain vs mixed);
* bumpy degree-3 NURBS cube, p=3, n=512 (1.3e8 DOF), eps 1e-6, FP32 cores;
* 256 seeded requests of mixed size, degree and geometry (batched / served).
"""
import math

import numpy as np

from .geometries import annulus_sector, bumpy_cube, twisted_box
from .problem import (BC_ZERO, PREC_FP32, PREC_FP64, Dirichlet, Discretization, Options,
                      Problem)
from .sources import fourier_source, manufactured_annulus_source

C2_SEED = 2025_0913_02
C3_GEOM_SEED = 2025_0913_03
C3_SOURCE_SEED = 2025_0913_13
C4_SEED_BASE = 10_000


def _all_zero():
    return Dirichlet(kind=(BC_ZERO,) * 6, value=(0.0,) * 6)


def c1_problem(eps=1e-10, tol=1e-10, n=16, p=2, g=3):
    geo = annulus_sector(1.0, 2.0, math.pi / 2, 1.0)
    return Problem(
        name=f"annulus_p{p}_n{n}_manufactured",
        geometry=geo,
        disc=Discretization(degree=p, n_basis=(n, n, n), n_gauss=g),
        source=manufactured_annulus_source(),
        dirichlet=_all_zero(),
        options=Options(tt_eps=eps, rel_res_tol=tol, max_iter=400, precision=PREC_FP64),
    )


def c2_problem(n=256, p=3, precision=PREC_FP64, eps=1e-6, tol=1e-7, seed=C2_SEED):
    geo = annulus_sector(1.0, 2.0, math.pi / 2, 1.0)
    return Problem(
        name=f"annulus_p{p}_n{n}_fourier8",
        geometry=geo,
        disc=Discretization(degree=p, n_basis=(n, n, n), n_gauss=p + 1),
        source=fourier_source(geo, seed),
        dirichlet=_all_zero(),
        options=Options(tt_eps=eps, rel_res_tol=tol, max_iter=400, precision=precision),
    )


def c3_problem(n=512, p=3, eps=1e-6, tol=1e-7, geom_seed=C3_GEOM_SEED,
               source_seed=C3_SOURCE_SEED, precision=PREC_FP32):
    geo = bumpy_cube(seed=geom_seed)
    return Problem(
        name=f"bumpy_cube_p{p}_n{n}_fourier8",
        geometry=geo,
        disc=Discretization(degree=p, n_basis=(n, n, n), n_gauss=p + 1),
        source=fourier_source(geo, source_seed),
        dirichlet=_all_zero(),
        # the products of the solve reach ranks near 270 before rounding settles them
        options=Options(tt_eps=eps, rel_res_tol=tol, max_iter=400, max_rank=1024, precision=precision),
    )


def small_problem(geometry, n, p, source, dirichlet=None, eps=1e-10, tol=1e-10, g=0,
                  name="small"):
    return Problem(
        name=name,
        geometry=geometry,
        disc=Discretization(degree=p, n_basis=(n, n, n) if np.isscalar(n) else tuple(n),
                            n_gauss=g),
        source=source,
        dirichlet=dirichlet if dirichlet is not None else _all_zero(),
        options=Options(tt_eps=eps, rel_res_tol=tol, max_iter=400, precision=PREC_FP64),
    )


def c4_requests(count=256, sizes=(32, 64, 128, 256), degrees=(2, 3), precision=PREC_FP32,
                eps=1e-6, tol=1e-7, assembly_eps=0.0, max_rank=256):
    """Request b draws n, p and a geometry (annulus sector or twisted box) from seed 10000+b.
    assembly_eps (0: eps) is the tolerance of the assembly alone."""
    out = []
    for b in range(count):
        rng = np.random.default_rng(C4_SEED_BASE + b)
        n = int(rng.choice(sizes))
        p = int(rng.choice(degrees))
        if rng.uniform() < 0.5:
            r_in = rng.uniform(0.5, 1.5)
            thick = rng.uniform(0.5, 1.5)
            sweep = rng.uniform(math.pi / 6, math.pi / 2)
            height = rng.uniform(0.5, 2.0)
            geo = annulus_sector(r_in, r_in + thick, sweep, height)
            gname = "annulus"
        else:
            geo = twisted_box(rng.uniform(0.0, math.pi / 2))
            gname = "twisted_box"
        src = fourier_source(geo, int(rng.integers(0, 2**31 - 1)))
        out.append(Problem(
            name=f"req{b}_{gname}_p{p}_n{n}",
            geometry=geo,
            disc=Discretization(degree=p, n_basis=(n, n, n), n_gauss=p + 1),
            source=src,
            dirichlet=_all_zero(),
            options=Options(tt_eps=eps, rel_res_tol=tol, max_iter=400, precision=precision,
                            assembly_eps=assembly_eps, max_rank=max_rank),
        ))
    return out
