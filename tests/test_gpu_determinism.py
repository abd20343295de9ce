"""Bit-reproducibility across processes: the same problem solved in two fresh processes, once alone
and once after and beside other problems on the executor, gives identical TT cores, the same
compression path and the same iteration count.  Every kernel's summation order is fixed by the
shapes alone (no timing-driven choices, no atomics in reductions), and the random draws of the
cross approximation and of the randomised roundings restart from fixed seeds in every assembly
and solve."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
import numpy as np
sys.path.insert(0, {root!r})
import workloads as W
from paper_2509_13224_amd import ttiga
from workloads.problem import Discretization
mode, out = sys.argv[1], sys.argv[2]

def shrink(pr):
    pr.disc = Discretization(degree=pr.disc.degree, n_basis=(36, 12, 12), n_gauss=pr.disc.n_gauss)
    return pr

target = shrink(W.c2_problem(seed=W.configs.C2_SEED + 1))
ctx = ttiga.Context(workspace_bytes=8 << 30)
if mode == "alone":
    res, cores = ctx.solve_batch([target], lanes=1)[0]
else:
    others = [shrink(W.c2_problem(seed=W.configs.C2_SEED + 5))] + W.c4_requests(count=3, sizes=(16, 24))
    ctx.solve_batch(others[:2], lanes=2)  # other problems first, on the same context
    outs = ctx.solve_batch(others[2:] + [target] + others[:1], lanes=3)
    res, cores = outs[2]
np.savez(out, *cores)
print(json.dumps(dict(status=res["status"], path=res["compression_path"], iterations=res["iterations"])))
"""


def _run(mode, tmp_path):
    out = str(tmp_path / f"{mode}.npz")
    code = SCRIPT.format(root=ROOT)
    say("determinism: fresh process", mode)
    r = subprocess.run([sys.executable, "-c", code, mode, out], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    info = json.loads(r.stdout.strip().splitlines()[-1])
    with np.load(out) as z:
        cores = [z[f"arr_{k}"] for k in range(3)]
    return info, cores


def test_same_bits_in_fresh_processes_alone_and_in_a_mix(tmp_path):
    a_info, a = _run("alone", tmp_path)
    b_info, b = _run("mix", tmp_path)
    say("determinism:", a_info, b_info)
    assert a_info["status"] == 0 and b_info == a_info
    assert all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b))
