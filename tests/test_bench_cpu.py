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
    """A whole oracle solve at a small n, on the host's cores, with the core count, CPU model and
    BLAS threads recorded, and the full-size sampling bound beside it."""
    out = bench.cpu_baseline(8, 1, 16)
    cores, affinity = bench.host_cores()
    assert out["kind"] == "oracle" and out["cores"] == cores and out["unit"] == "solves/s"
    assert out["value"] > 0 and out["seconds"] > 0 and out["n"] == 8
    assert out["affinity_cores"] == affinity >= cores >= 1
    assert "n=8" in out["sample"] and "1 of" in out["full_size_sampling_bound"]["note"]
    assert out["full_size_sampling_bound"]["solves_per_s"] > 0


def test_measured_traffic_needs_the_recorded_source(tmp_path, monkeypatch):
    """The PMC traffic line counts only while the kernel's source file is unchanged."""
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text("kernel v1")
    sha = hashlib.sha256(b"kernel v1").hexdigest()
    summary = tmp_path / "pmc.md"
    summary.write_text(f"traffic: kernel=kx fetch_kib=10.0 write_kib=6.0 source=k.hip sha256={sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    val, note = bench.measured_traffic("kx")
    assert val == 16.0 * 1024 and "pmc" in note
    assert bench.measured_traffic("other")[0] is None
    src.write_text("kernel v2")
    val, note = bench.measured_traffic("kx")
    assert val is None and "changed" in note


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
