"""Batched and serving modes: every result equals the same problem solved alone, failures stay
with their problem, and admission refuses what can never fit."""
import threading
import time

import numpy as np
import pytest

import workloads as W
from oracle import sparse_iga, tt_iga
from tests.gpu_helpers import same_tt, say, tt_rel_diff
from workloads.problem import PREC_FP64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=8 << 30)


def _mix(count=6):
    """Small requests of the batched family: annulus sectors and twisted boxes, p in {2, 3}."""
    return W.c4_requests(count=count, sizes=(12, 16, 24), precision=PREC_FP64, eps=1e-8, tol=1e-9)


def _alone(ctx, pr):
    h = ctx.problem_create(pr, precond=1)
    h.assemble()
    st = h.solve(allow_notconv=True)
    u = h.solution()
    h.close()
    return st, u


def test_batch_equals_alone(ctx):
    say("batch alone-vs-mix")
    reqs = _mix()
    out = ctx.solve_batch(reqs, lanes=3)
    lanes = set()
    for pr, (res, u) in zip(reqs, out):
        say("batch", pr.name)
        assert res["status"] == 0, res
        assert res["peak_bytes"] > 0 and res["latency_ms"] >= res["run_ms"] > 0
        lanes.add(res["lane"])
        st, u0 = _alone(ctx, pr)
        assert res["iterations"] == st["iterations"]
        # the same kernels with the same shapes in the same order: the same bits
        assert same_tt(u, u0), (pr.name, tt_rel_diff(u, u0))
    assert len(lanes) > 1
    # and one of them against the sparse direct solution of the oracle
    pr, (res, u) = reqs[0], out[0]
    u_h = sparse_iga.solve(pr)
    x = tt_iga.full_solution(pr, u).ravel()
    assert np.linalg.norm(x - u_h) <= 1e-6 * np.linalg.norm(u_h)


def test_batch_isolates_failures(ctx):
    from paper_2509_13224_amd import ttiga
    say("batch failures")
    good = _mix(2)
    folded = W.twisted_box(0.3)
    folded.ctrl = folded.ctrl.copy()
    folded.ctrl[..., 0] *= -1.0
    bad_geo = W.small_problem(folded, 6, 2, W.zero_source())
    capped = W.c1_problem(n=10)
    capped.options.max_iter = 1
    reqs = [good[0], bad_geo, capped, good[1]]
    out = ctx.solve_batch(reqs, lanes=2)
    codes = [r["status"] for r, _ in out]
    assert codes == [0, ttiga.TTIGA_E_DETJ, ttiga.TTIGA_E_NOTCONV, 0], codes
    assert out[1][1] is None and out[2][1] is not None
    assert "det J" in out[1][0]["error"]


def test_server_alone_vs_mix(ctx):
    """Requests submitted from three threads while others run: each result equals its solve
    alone (same iterations, bit-identical TT cores)."""
    say("server mix")
    reqs = _mix(9)
    srv = ctx.server(hbm_budget=4 << 30, lanes=4)
    tickets = [None] * len(reqs)
    errors = []

    def client(k):
        try:
            for i in range(k, len(reqs), 3):
                tickets[i] = srv.submit(reqs[i])
                time.sleep(0.01 * (i % 4))
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=client, args=(k,)) for k in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    results = [srv.poll(t, wait_ms=-1) for t in tickets]
    for pr, t, res in zip(reqs, tickets, results):
        say("server", pr.name)
        assert res["status"] == 0, res
        assert res["queue_ms"] >= 0 and res["latency_ms"] >= res["run_ms"]
        u = srv.solution(t)
        st, u0 = _alone(ctx, pr)
        assert res["iterations"] == st["iterations"]
        assert same_tt(u, u0), (pr.name, tt_rel_diff(u, u0))
        srv.release(t)
    assert len({r["lane"] for r in results}) > 1
    srv.close()


def test_server_admission(ctx):
    from paper_2509_13224_amd import ttiga
    say("server admission")
    srv = ctx.server(hbm_budget=256 << 20, lanes=2)
    big = W.c2_problem(n=64)
    assert ttiga.footprint(big) > 256 << 20
    with pytest.raises(ttiga.TTIGAError) as e:
        srv.submit(big)
    assert e.value.code == ttiga.TTIGA_E_ADMISSION
    small = _mix(1)[0]
    t = srv.submit(small)
    res = srv.poll(t, wait_ms=-1)
    assert res["status"] == 0 and res["footprint_bytes"] <= 256 << 20
    with pytest.raises(ttiga.TTIGAError):
        srv.release(t + 100)
    srv.release(t)
    srv.close()


def test_server_tight_pool_keeps_resident_solutions(ctx):
    """A pool that holds about two footprints, two lanes and eight requests whose solutions stay
    resident until the end: admission charges the resident solutions, a lane that finds the pool
    fragmented waits only while another problem is running, and every request finishes with the
    result it has alone."""
    from paper_2509_13224_amd import ttiga
    say("server tight pool")
    reqs = _mix(8)
    fp = max(ttiga.footprint(pr) for pr in reqs)
    srv = ctx.server(hbm_budget=int(2.2 * fp), lanes=2)
    tickets = [srv.submit(pr) for pr in reqs]
    results = [srv.poll(t, wait_ms=-1) for t in tickets]
    for pr, t, res in zip(reqs, tickets, results):
        assert res["status"] == 0, res
        st, u0 = _alone(ctx, pr)
        assert same_tt(srv.solution(t), u0), pr.name
    for t in tickets:
        srv.release(t)
    srv.close()
