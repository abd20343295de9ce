"""Host-side pieces of bench.py: the one-GPU contract, the accuracy metric behind the solves/s
gate (relative coefficient 2-norm of a TT difference) and the CPU oracle baseline leg."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _rand_tt(rng, n, r):
    ranks = [1, r[0], r[1], 1]
    return [rng.standard_normal((ranks[k], n[k], ranks[k + 1])) for k in range(3)]


def _full(cores):
    a = np.tensordot(cores[0], cores[1], axes=([2], [0]))
    a = np.tensordot(a, cores[2], axes=([3], [0]))
    return a.reshape(cores[0].shape[1], cores[1].shape[1], cores[2].shape[1])


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_rel_diff_matches_dense_difference():
    rng = np.random.default_rng(11)
    n = (7, 5, 6)
    a, b = _rand_tt(rng, n, (3, 4)), _rand_tt(rng, n, (2, 3))
    ref = np.linalg.norm(_full(a) - _full(b)) / np.linalg.norm(_full(b))
    assert abs(bench.tt_rel_diff(a, b) - ref) <= 1e-12 * ref
    # a tiny perturbation is resolved without cancellation
    c = [x.copy() for x in b]
    c[1] = c[1] * (1.0 + 1e-12)
    assert abs(bench.tt_rel_diff(c, b) - 1e-12) <= 1e-15
    assert bench.tt_rel_diff(b, b) <= 1e-15


def test_percentile():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.percentile(xs, 50) == 3.0
    assert bench.percentile(xs, 0) == 1.0
    assert bench.percentile(xs, 100) == 5.0
    assert bench.percentile([], 50) is None


def test_cpu_baseline_reports_the_contract_fields():
    out = bench.cpu_baseline(16, 1)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "solves/s"
    assert out["value"] > 0 and out["seconds_sampled"] > 0
    assert "1 of" in out["sample"]


def test_roofline_entry_arithmetic():
    """achieved = algorithmic work / time, frac = achieved / peak, the unit by the class's bound."""
    st = {"total_ms": 2.0, "launches": 4, "flops": 4.0e9, "bytes": 8.0e9}
    alu = bench.roofline_entry("tsqr_factor", st)
    assert alu["bound"] == "alu" and alu["unit"] == "TFLOP/s"
    assert abs(alu["achieved"] - 2.0) < 1e-12 and abs(alu["frac"] - 2.0 / 78.6) < 1e-12
    assert abs(alu["avg_launch_us"] - 500.0) < 1e-9 and alu["algorithmic_per_launch"] == 1.0e9
    hbm = bench.roofline_entry("tt_matvec_banded", st)
    assert hbm["bound"] == "hbm" and hbm["unit"] == "GB/s"
    assert abs(hbm["achieved"] - 4000.0) < 1e-9 and abs(hbm["frac"] - 0.5) < 1e-12
