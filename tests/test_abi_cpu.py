"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and
validates problem descriptions without touching a GPU."""
import copy
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2509_13224_amd import ttiga
from workloads.problem import BC_CONSTANT, BC_NATURAL, Dirichlet

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ttiga.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(ttiga_\w+)\s*\(", txt, flags=re.M)))


def test_header_matches_binding_list():
    assert declared_functions() == sorted(ttiga.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ttiga.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version():
    import ctypes
    lib = ttiga.load()
    a, b = ctypes.c_int(), ctypes.c_int()
    assert lib.ttiga_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) == (0, 1)


def test_validate_accepts_workloads():
    for pr in (W.c1_problem(), W.c2_problem(n=64), W.c3_problem(n=64, precision=0)):
        assert ttiga.validate(pr)[0] == 0, pr.name
    for pr in W.c4_requests(6, precision=0):
        assert ttiga.validate(pr)[0] == 0, pr.name


def _bad(mutate):
    pr = copy.deepcopy(W.c1_problem())
    mutate(pr)
    return ttiga.validate(pr)


def test_validate_rejects_bad_knots():
    def nonmono(pr):
        pr.geometry.knots[1] = np.array([0, 0, 0.5, 0.2, 1, 1.0])
    assert _bad(nonmono)[0] == ttiga.TTIGA_E_KNOTS

    def short_mult(pr):
        pr.geometry.knots[1] = np.array([0, 0, 0.5, 1, 1, 1.0])
    assert _bad(short_mult)[0] == ttiga.TTIGA_E_KNOTS

    def not_unit(pr):
        pr.geometry.knots[2] = np.array([0, 0, 2, 2.0])
    assert _bad(not_unit)[0] == ttiga.TTIGA_E_KNOTS

    def too_few_ctrl(pr):
        pr.geometry.ctrl = pr.geometry.ctrl[:, :2]
        pr.geometry.weights = pr.geometry.weights[:, :2]
    assert _bad(too_few_ctrl)[0] == ttiga.TTIGA_E_ARG


def test_validate_rejects_nonpositive_weight():
    def neg(pr):
        pr.geometry.weights = pr.geometry.weights.copy()
        pr.geometry.weights[0, 1, 0] = -0.5
    assert _bad(neg)[0] == ttiga.TTIGA_E_GEOM


def test_validate_rejects_bad_discretisation_and_options():
    def small_n(pr):
        pr.disc.n_basis = (2, 16, 16)
    assert _bad(small_n)[0] == ttiga.TTIGA_E_ARG

    def bad_eps(pr):
        pr.options.tt_eps = 0.0
    assert _bad(bad_eps)[0] == ttiga.TTIGA_E_ARG

    def bad_prec(pr):
        pr.options.precision = 7
    assert _bad(bad_prec)[0] == ttiga.TTIGA_E_ARG


def test_validate_constant_dirichlet_rules():
    geo = W.annulus_sector(0.5, 1.0, math.pi / 2, 1.0)
    ok = Dirichlet(kind=(BC_CONSTANT, BC_CONSTANT) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    assert ttiga.validate(W.small_problem(geo, 8, 2, W.zero_source(), dirichlet=ok))[0] == 0
    # constants on faces of several directions are lifted too (the later face wins at edges)
    two_dirs = Dirichlet(kind=(BC_CONSTANT,) * 2 + (BC_CONSTANT,) + (BC_NATURAL,) * 3,
                         value=(1.0, 2.0, 3.0, 0, 0, 0))
    assert ttiga.validate(W.small_problem(geo, 8, 2, W.zero_source(), dirichlet=two_dirs))[0] == 0
    bad_kind = Dirichlet(kind=(BC_CONSTANT, 7) + (BC_NATURAL,) * 4, value=(1.0, 2.0, 0, 0, 0, 0))
    code, msg = ttiga.validate(W.small_problem(geo, 8, 2, W.zero_source(), dirichlet=bad_kind))
    assert code == ttiga.TTIGA_E_ARG and "boundary kind" in msg


def test_footprint_estimate_orders_requests():
    """Admission estimates (host only): grow with the grid, and the slab-streamed sampling
    keeps the n=256 problem far below the 58 GB of whole-grid factor samples."""
    from workloads.problem import PREC_FP64
    f16 = ttiga.footprint(W.c1_problem(n=16))
    f64 = ttiga.footprint(W.c2_problem(n=64))
    f256 = ttiga.footprint(W.c2_problem(n=256))
    c3 = W.c3_problem(n=512)
    c3.options.precision = PREC_FP64
    f512 = ttiga.footprint(c3)
    assert 0 < f16 < f64 < f256 < f512
    whole_256 = 7 * 1012 ** 3 * 8
    assert f256 < whole_256 / 4 and f256 < 16 << 30
    assert f512 < 64 << 30
    # forcing small chunks shrinks the estimate of a mid-size problem
    pr = W.c2_problem(n=64)
    pr.options.sample_chunk_bytes = 64 << 20
    assert ttiga.footprint(pr) < f64


def test_validate_mixed_precision_rules():
    """FP32/BF16 refine around the preconditioned solver: accepted with precond=1 only."""
    from workloads.problem import PREC_BF16, PREC_FP32
    for prec in (PREC_FP32, PREC_BF16):
        pr = W.c2_problem(n=64, precision=prec)
        assert ttiga.validate(pr, precond=1)[0] == ttiga.TTIGA_OK
        code, msg = ttiga.validate(pr, precond=0)
        assert code == ttiga.TTIGA_E_ARG and "precond" in msg
    for pr in W.c4_requests(4):  # the batched family is FP32 by default
        assert ttiga.validate(pr, precond=1)[0] == ttiga.TTIGA_OK


def test_validate_assembly_eps_range():
    """assembly_eps: 0 (use tt_eps) or a tolerance in (0, 1); anything else is E_ARG."""
    pr = W.c2_problem(n=64)
    for ok in (0.0, 1e-9):
        pr.options.assembly_eps = ok
        assert ttiga.validate(pr)[0] == ttiga.TTIGA_OK
    for bad in (-1e-9, 1.0, 2.0):
        pr.options.assembly_eps = bad
        code, msg = ttiga.validate(pr)
        assert code == ttiga.TTIGA_E_ARG and "assembly_eps" in msg


def test_c4_requests_follow_the_recipe():
    """Request b is drawn from seed 10000 + b: n from the size set, p in {2, 3}, annulus sector or
    twisted box about half each; the draws repeat, and the options reach every request."""
    a, b = W.c4_requests(64), W.c4_requests(64)
    assert [r.name for r in a] == [r.name for r in b]
    assert {r.disc.n_basis[0] for r in a} == {32, 64, 128, 256}
    assert {r.disc.degree for r in a} == {2, 3}
    share = sum("annulus" in r.name for r in a) / len(a)
    assert 0.3 < share < 0.7
    s = W.c4_requests(32, sizes=(32, 64, 128, 256, 512), assembly_eps=1e-9, max_rank=1024)
    assert any(r.disc.n_basis[0] == 512 for r in s)
    assert all(r.options.assembly_eps == 1e-9 and r.options.max_rank == 1024 for r in s)
