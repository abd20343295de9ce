#!/usr/bin/env python3
"""Throughput of TT-IGA solves on one MI355X.

One solve is the whole hot path for one problem: TT assembly (basis tables, geometry
factors on the Gauss grid compressed by cross approximation, TT cores of K and F, summation
with rounding, boundary reduction), the TT solve (the paper's AMEn by default, `--solver cg`
for the preconditioned TT-CG), and the solution cores resident on the device.  The workload is the plain-vs-mixed annulus case:
quarter annulus (radii 1..2, 90 degrees) extruded over z in [0, 1], degree-3 B-splines
with 256 basis functions per direction (16.7M DOF), f from 8 seeded Fourier modes, TT
tolerance 1e-6.

One timed step is a batch of --batch such problems (Fourier seeds seed0 + b) run on
--lanes concurrent lanes of the library's executor (FP64 path); `value` is solves per
second over the timed steps, counting only solves within 1e-6 (relative, coefficient
2-norm) of an FP64 reference solve of the same problem at eps/10, tol/10 by the other method
(preconditioned TT-CG references for AMEn solves).  Problem
descriptions (a few KB each) are host inputs; everything else happens on the device.

Beside it the JSON line reports: the same batches and single solve with the other solver
(`solver_comparison`); the single-solve latency of the plain FP64 path with
the roofline of its dominant kernel class (HIP events around every launch of that
class, on the library's stream) and the TT-matvec rate; the mixed-precision (FP32
operator, FP64 refinement) batch; the batched family (256 requests of mixed sizes and
geometries, FP32) with its throughput; Poisson-arrival serving of requests drawn the same
way with sizes up to n = 512, at 0.25x to 2x the family's throughput, with p50/p99 latency;
and the oracle's CPU rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "fp64_tflops": 78.6,
}
# bound of each kernel class: memory traffic or FP64 arithmetic (a contraction class whose
# arithmetic intensity lies below the ridge is held to the HBM roof instead: roofline_entry)
KERNEL_BOUND = {
    "gemm_f64": "mfma",
    "tt_matvec_banded": "hbm",
    "tt_matvec_fp32": "hbm",
    "tt_matvec_bf16": "hbm",
    "tt_axpby": "hbm",
    "precond_scaling": "hbm",
    "geometry_factors": "alu",
    "tsqr_factor": "alu",
    "tsqr_apply": "alu",
    "jacobi_svd": "alu",
    "jacobi_eig": "alu",
    "geometry_detj": "alu",
    "assemble_cores": "alu",
}
SERVE_SEED = 2025_0913_05
SERVE_SIZES = (32, 64, 128, 256, 512)
# arrival rates as fractions of the served mix's own saturation throughput (all requests offered
# at once to the same server), a geometric sweep
SERVE_RATES = (0.5, 1.0, 2.0)
# the n = 512 FP32 refinements reach ranks of about 360 in their corrections
SERVE_MAX_RANK = 1024
# tolerance of the family's assembly (eps / 1000; its references: eps / 10000): on twisted boxes a
# compressed operator that drops a singular value near eps = 1e-6 moves the solution by up to 1e-3,
# and at 1e-8 some requests (and at 1e-9 some references) still sit above 1e-6
ASSEMBLY_EPS = 1e-9
# HBM bytes per dispatch of the roofline kernel, measured by two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) of `bench.py --single-only` and written, with the copy-kernel calibration, into
# this summary as `traffic:` lines; a line counts only while the sha256 of the kernel's source files
# (the kernel and, for the GEMM, its plan table) still equals the one recorded with it (after a
# change to either the field is null).
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic.md")


def measured_traffic(kernel):
    """(bytes per dispatch, note) of `kernel` from the committed PMC summary, or (None, reason)."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None, "no PMC summary"
    for line in open(TRAFFIC_SUMMARY):
        m = re.match(r"\s*traffic: kernel=(\S+) fetch_kib=([\d.]+) write_kib=([\d.]+) source=(\S+) sha256=([0-9a-f]+)",
                     line)
        if not m or m.group(1) != kernel:
            continue
        # source: one file, or several joined by '+' (hashed in that order, concatenated)
        h = hashlib.sha256()
        for rel in m.group(4).split("+"):
            src = os.path.join(ROOT, rel)
            if not os.path.exists(src):
                return None, f"source {rel} missing"
            h.update(open(src, "rb").read())
        if h.hexdigest() != m.group(5):
            return None, f"{m.group(4)} changed since the counters were taken"
        return 1024.0 * (float(m.group(2)) + float(m.group(3))), f"rocprofv3 --pmc, {TRAFFIC_SUMMARY[len(ROOT) + 1:]}"
    return None, f"no PMC line for {kernel}"


def roofline_entry(name, st):
    """Roofline of a kernel class from its measured time and algorithmic flops and bytes.  A
    contraction class is held to the roof its arithmetic intensity meets: the FP64 MFMA peak at
    or above the ridge (peak flops / peak bandwidth, 9.8 flop/byte), HBM bandwidth below it (the
    short-contraction products of the small TT ranks move more bytes than MFMA time)."""
    bound = KERNEL_BOUND.get(name, "alu")
    secs = st["total_ms"] * 1e-3
    ridge = PEAKS["fp64_tflops"] * 1e12 / (PEAKS["hbm_GBps"] * 1e9)
    intensity = st["flops"] / st["bytes"] if st["bytes"] > 0 else None
    if bound == "mfma" and intensity is not None and intensity < ridge:
        bound = "hbm"
    if bound == "hbm":
        achieved = st["bytes"] / secs / 1e9
        peak, unit = PEAKS["hbm_GBps"], "GB/s"
    else:
        achieved = st["flops"] / secs / 1e12
        peak, unit = PEAKS["fp64_tflops"], "TFLOP/s"
    return {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "launches": st["launches"],
            "avg_launch_us": 1e3 * st["total_ms"] / max(st["launches"], 1),
            "algorithmic_per_launch": (st["bytes"] if bound == "hbm" else st["flops"]) / max(st["launches"], 1),
            "arithmetic_intensity": intensity, "ridge": ridge,
            "achieved_tflops": st["flops"] / secs / 1e12, "achieved_GBps": st["bytes"] / secs / 1e9}


def tt_rel_diff(a, b):
    """||a - b|| / ||b|| for host TT cores: the difference train left-orthogonalised by QR,
    its norm read from the last core (no cancellation between <a,a>, <a,b>, <b,b>)."""
    import numpy as np

    def orth_norm(cores):
        cores = [c.copy() for c in cores]
        for k in range(len(cores) - 1):
            r0, n, r1 = cores[k].shape
            q, r = np.linalg.qr(cores[k].reshape(r0 * n, r1))
            cores[k + 1] = np.tensordot(r, cores[k + 1], axes=([1], [0]))
        return float(np.linalg.norm(cores[-1]))

    d = []
    for k, (A, B) in enumerate(zip(a, b)):
        if k == 0:
            d.append(np.concatenate([A, -B], axis=2))
        elif k == len(a) - 1:
            d.append(np.concatenate([A, B], axis=0))
        else:
            C = np.zeros((A.shape[0] + B.shape[0], A.shape[1], A.shape[2] + B.shape[2]))
            C[:A.shape[0], :, :A.shape[2]] = A
            C[A.shape[0]:, :, A.shape[2]:] = B
            d.append(C)
    return orth_norm(d) / orth_norm(b)


def host_cores():
    """Threads the oracle may use: the machine's CPU share (OMP_NUM_THREADS when the environment sets
    it), else the cores this process may run on."""
    aff = len(os.sched_getaffinity(0))
    try:
        omp = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        omp = 0
    return min(aff, omp) if omp > 0 else aff, aff


def cpu_model():
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return None


def cpu_baseline(n, slabs, n_full):
    """The oracle's whole TT pipeline (Gauss-grid sampling, TT-SVD, assembly with rounding,
    truncated TT-CG) on one problem of the benchmark's family at n basis functions per
    direction, with BLAS threads set to the host cores; plus the oracle's factor sampling on
    `slabs` first-direction slabs of the full-size grid, extrapolated, as a bound for the
    full-size problem."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads as W
    from oracle import geometry, tt_iga
    cores, affinity = host_cores()
    pr = W.c2_problem(n=n)
    with threadpool_limits(limits=cores):
        blas = [f"{i.get('internal_api')}:{i.get('num_threads')}" for i in threadpool_info()]
        t0 = time.perf_counter()
        tt_iga.solve(pr)
        dt = time.perf_counter() - t0
        full = W.c2_problem(n=n_full)
        grid = geometry.gauss_grid(full)
        Q0 = len(grid[0][0])
        sub = [(grid[0][0][:slabs], grid[0][1][:slabs]), grid[1], grid[2]]
        t1 = time.perf_counter()
        geometry.sample_factors_grid(full, sub)
        ds = time.perf_counter() - t1
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"one whole oracle TT solve (sampling, TT-SVD, assembly, truncated TT-CG) of the same "
                       f"annulus / Fourier family at n={n}/dir ({n ** 3} DOF), eps and tol as the benchmark; "
                       f"{dt:.1f} s on {cores} BLAS threads"),
            "seconds": dt, "n": n, "cpu_model": cpu_model(), "affinity_cores": affinity, "blas": blas,
            "full_size_sampling_bound": {
                "solves_per_s": 1.0 / (ds * Q0 / slabs),
                "note": (f"factor sampling alone on {slabs} of {Q0} first-direction slabs at n={n_full} "
                         f"({ds:.1f} s), extrapolated to the whole grid ({ds * Q0 / slabs:.0f} s): an upper "
                         f"bound on the oracle's full-size solve rate")}}


# seeded synthetic sweep of the TT-matrix x TT-vector product: random banded operator cores of
# ranks (rK, rK), vector cores of ranks (rx, rx), N(0, 1) entries
SWEEP_RK = (2, 4, 8, 16, 32)
SWEEP_RX = (8, 16, 32, 64, 128)
SWEEP_N = (256, 512)
SWEEP_P = (2, 3)
SWEEP_DTYPES = ((0, "fp64", "tt_matvec_banded"), (1, "fp32", "tt_matvec_fp32"), (2, "bf16", "tt_matvec_bf16"))
# points whose product cores exceed this are left out (the largest, rK 32 x rx 128 at n = 512,
# would write 69 GB)
SWEEP_MAX_OUT_BYTES = 8 << 30
SWEEP_SEED = 2025_0913_07


def matvec_sweep(ctx, reps=3, only=None):
    """Achieved HBM GB/s and TFLOP/s of the banded TT-matvec over the synthetic sweep, from the
    library's per-launch HIP events (algorithmic bytes: operator, vector and product cores).
    only = (rK, rx, n, p) restricts the sweep to that point (profiling runs)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(SWEEP_SEED)
    points, skipped = [], 0
    for n in SWEEP_N:
        for p in SWEEP_P:
            band = 2 * p + 1
            mask = np.array([[0 <= i + t - p < n for t in range(band)] for i in range(n)], dtype=np.float64)
            for rK in SWEEP_RK:
                for rx in SWEEP_RX:
                    if only and (rK, rx, n, p) != only:
                        continue
                    out_bytes = 8 * n * ((rK * rx) ** 2 + 2 * rK * rx)
                    if out_bytes > SWEEP_MAX_OUT_BYTES:
                        skipped += len(SWEEP_DTYPES)
                        continue
                    rKs, rxs = (1, rK, rK, 1), (1, rx, rx, 1)
                    K = [torch.from_numpy(rng.normal(size=(rKs[k], n, band, rKs[k + 1])) *
                                          mask[None, :, :, None]).cuda() for k in range(3)]
                    x = [torch.from_numpy(rng.normal(size=(rxs[k], n, rxs[k + 1]))).cuda() for k in range(3)]
                    for code, dname, cls in SWEEP_DTYPES:
                        ctx.tt_matvec(K, p, x, dtype=code or None, copy=False)  # warm-up
                        ctx.profile(-1)
                        ctx.profile(1)
                        for _ in range(reps):
                            ctx.tt_matvec(K, p, x, dtype=code or None, copy=False)
                        ctx.profile(0)
                        st = ctx.profile_read()[cls]
                        secs = st["total_ms"] * 1e-3
                        gbs = st["bytes"] / secs / 1e9
                        points.append({"rK": rK, "rx": rx, "n": n, "p": p, "dtype": dname,
                                       "GBps": gbs, "TFLOPps": st["flops"] / secs / 1e12,
                                       "hbm_frac": gbs / PEAKS["hbm_GBps"],
                                       "us_per_product": 1e6 * secs / reps})
                    del K, x
    torch.cuda.synchronize()
    big = [q for q in points if q["rK"] * q["rx"] >= 256]
    return {"points": points, "skipped_points": skipped,
            "max_hbm_frac": max(q["hbm_frac"] for q in points),
            "median_hbm_frac_large": (sorted(q["hbm_frac"] for q in big)[len(big) // 2] if big else None),
            "max_tflops": {d: max(q["TFLOPps"] for q in points if q["dtype"] == d) for _, d, _ in SWEEP_DTYPES},
            "recipe": (f"seed {SWEEP_SEED}; banded operator cores of ranks (rK, rK), vector cores of ranks "
                       f"(rx, rx), N(0,1) entries; rK in {SWEEP_RK}, rx in {SWEEP_RX}, n in {SWEEP_N}, p in "
                       f"{SWEEP_P}; points whose product exceeds {SWEEP_MAX_OUT_BYTES >> 30} GiB left out; "
                       f"{reps} timed products per point after one warm-up; bytes = operator + vector + "
                       f"product cores (FP64 product, operator in the point's dtype)")}


def log(*a):
    """Progress on stderr (the JSON result line is the only stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def serve(ctx, reqs, rate, lanes, seed):
    """Poisson arrivals at `rate` requests/s into a server (rate None: all at once); returns the
    results, the solutions and the seconds from the first submission to the last result."""
    import threading

    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(reqs)) if rate else np.zeros(len(reqs))
    srv = ctx.server(lanes=lanes)
    tickets = [None] * len(reqs)
    t0 = time.perf_counter()

    def producer():
        t = t0
        for i, pr in enumerate(reqs):
            t += gaps[i]
            delay = t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[i] = srv.submit(pr)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    results = []
    for i, t in enumerate(tickets):
        results.append(srv.poll(t, wait_ms=-1))
        if (i + 1) % 50 == 0 and i + 1 < len(tickets):
            log(f"  {i + 1} of {len(tickets)} requests done")
    t1 = time.perf_counter()
    sols = [srv.solution(t) if r["status"] in (0, -7) else None for t, r in zip(tickets, results)]
    for t in tickets:
        srv.release(t)
    srv.close()
    return results, sols, t1 - t0


def serving_phase(ctx, count, lanes, solver=1):
    """C5: `count` requests of the batched family with sizes up to n = 512 (FP64 AMEn solves, or with
    solver 0 FP32 mixed TT-CG), served by one server under Poisson arrivals at fractions of the
    mix's own saturation throughput; latency percentiles, offered and achieved rates, and every
    result against its FP64 TT-CG reference."""
    import workloads as W
    from workloads.problem import PREC_FP32, PREC_FP64
    sreqs = W.c4_requests(count=count, sizes=SERVE_SIZES, precision=PREC_FP64 if solver else PREC_FP32,
                          assembly_eps=ASSEMBLY_EPS, max_rank=SERVE_MAX_RANK)
    for pr in sreqs:
        pr.options.solver = solver
    log("serving references")
    ref_pr = W.c4_requests(count=count, sizes=SERVE_SIZES, precision=PREC_FP64, eps=1e-7, tol=1e-8,
                           assembly_eps=ASSEMBLY_EPS / 10, max_rank=SERVE_MAX_RANK)
    srefs = []
    for b in range(0, count, 50):
        srefs += [u for _, u in ctx.solve_batch(ref_pr[b:b + 50], lanes=lanes)]
        log(f"  references: {len(srefs)} of {count}")

    def summarise(res, sols, secs, offered):
        serr = [tt_rel_diff(u, ur) if (u is not None and ur is not None) else float("inf")
                for u, ur in zip(sols, srefs)]
        lat = [r["latency_ms"] for r in res]
        ok = sum(e <= 1e-6 for e in serr)
        return {"offered_per_s": offered, "achieved_per_s": len(res) / secs, "solves_per_s": ok / secs,
                "passed": ok, "p50_ms": percentile(lat, 50), "p90_ms": percentile(lat, 90),
                "p99_ms": percentile(lat, 99), "max_ms": max(lat),
                "mean_queue_ms": sum(r["queue_ms"] for r in res) / len(res), "rel_err_max": max(serr)}

    log("serving: saturation (all requests at once)")
    res, sols, secs = serve(ctx, sreqs, None, lanes, SERVE_SEED)
    sat_line = summarise(res, sols, secs, None)
    sat = sat_line["achieved_per_s"]
    lines = []
    for frac in SERVE_RATES:
        log("serving at", frac, "x saturation")
        res, sols, secs = serve(ctx, sreqs, frac * sat, lanes, SERVE_SEED)
        line = summarise(res, sols, secs, frac * sat)
        line["fraction_of_saturation"] = frac
        lines.append(line)
    return {"requests": count, "arrival": f"Poisson, seed {SERVE_SEED}", "lanes": lanes,
            "workload": ("n in {32,64,128,256,512}, p in {2,3}, annulus sector or twisted box, seeded Fourier "
                         f"source, {'FP64 AMEn' if solver else 'FP32 mixed TT-CG'}, assembly at {ASSEMBLY_EPS:g}, "
                         "seeds 10000+b"),
            "saturation": sat_line, "rates": lines,
            "percentiles": f"nearest rank over {count} requests per rate"}



def c3_amen_phase(ctx):
    """The complex-geometry configuration (bumpy cube, degree 3, n = 512, 1.3e8 DOF, FP64) solved by
    AMEn once, with the rate of its GEMMs (the local products contract the operator rank 84)."""
    import workloads as W
    from paper_2509_13224_amd import ttiga
    from workloads.problem import PREC_FP64
    pr = W.c3_problem(n=512, precision=PREC_FP64)
    pr.options.solver = ttiga.TTIGA_SOLVER_AMEN
    h = ctx.problem_create(pr, precond=1)
    t0 = time.perf_counter()
    ast = h.assemble()
    t1 = time.perf_counter()
    ctx.profile(-1)
    ctx.profile(1)
    st3 = h.solve(allow_notconv=True)
    t2 = time.perf_counter()
    ctx.profile(0)
    p3 = ctx.profile_read()
    h.close()
    g3 = p3.get("gemm_f64")
    return {
        "workload": "bumpy cube (seeded NURBS), degree 3, n=512/dir (1.3e8 DOF), 8-mode Fourier source, "
                    "TT eps 1e-6, tol 1e-7, FP64, AMEn (one solve; the preconditioner plan is built in it)",
        "assembly_ms": 1e3 * (t1 - t0), "solve_ms": 1e3 * (t2 - t1),
        "plan_ms": st3["precond_setup_ms"], "solve_ms_without_plan": 1e3 * (t2 - t1) - st3["precond_setup_ms"],
        "status": st3["status"],
        "half_sweeps": st3["iterations"], "local_iterations": st3["local_iterations"], "rank_u": st3["rank_u"],
        "rank_K": ast["rank_K"], "compression_path": ast["compression_path"], "samples": ast["samples"],
        "rel_pres": st3["rel_pres"], "rel_res": st3["rel_res"],
        "gemm_f64": ({"tflops": g3["flops"] / (g3["total_ms"] * 1e-3) / 1e12,
                      "frac_fp64_peak": g3["flops"] / (g3["total_ms"] * 1e-3) / 1e12 / PEAKS["fp64_tflops"],
                      "ms": g3["total_ms"], "launches": g3["launches"],
                      "avg_launch_us": 1e3 * g3["total_ms"] / max(g3["launches"], 1)} if g3 else None),
        "kernels": {k: {"ms": v["total_ms"], "launches": v["launches"]}
                    for k, v in sorted(p3.items(), key=lambda kv: -kv[1]["total_ms"])[:6]}}

def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed batches")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="basis functions per direction")
    ap.add_argument("--batch", type=int, default=16, help="problems per step")
    ap.add_argument("--lanes", type=int, default=16, help="concurrent executor lanes")
    ap.add_argument("--family", type=int, default=256, help="requests of the batched family (0: skip)")
    ap.add_argument("--serve", type=int, default=32, help="requests per serving rate (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slabs", type=int, default=8)
    ap.add_argument("--cpu-n", type=int, default=32, help="basis functions per direction of the oracle sample")
    ap.add_argument("--workspace-gib", type=float, default=200.0)
    ap.add_argument("--solver", choices=("amen", "cg"), default="amen",
                    help="TT solve of the timed problems: the paper's AMEn, or preconditioned TT-CG")
    ap.add_argument("--single-only", action="store_true",
                    help="only the single-solve phase (value = its solve rate): the run whose kernel "
                         "averages a rocprofv3 trace can be compared with the roofline line")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the timed batched FP64 steps (value = their solve rate, accuracy not "
                         "gated): the run whose rocprofv3 trace shows the lanes side by side")
    ap.add_argument("--calibrate-copy", type=float, default=0.0,
                    help="only copy this many GiB device-to-device three times (scale of the HBM "
                         "byte counters) and exit")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving measurement (use with --serve 300 for resolved percentiles)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the synthetic TT-matvec sweep (value = the best fraction of HBM bandwidth)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the complex-geometry AMEn solve")
    ap.add_argument("--c3-only", action="store_true", help="only the complex-geometry AMEn solve (profiling)")
    ap.add_argument("--sweep-point", type=str, default="",
                    help="rK,rx,n,p: run only this point of the sweep (with --sweep-only)")
    ap.add_argument("--traffic-kib", type=str, default="",
                    help="measured FETCH_SIZE,WRITE_SIZE of the roofline kernel (KiB per dispatch, "
                         "already scaled by the copy calibration) to report as roofline.traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the TT-IGA solve here is a "
              "single-device hot path; independent solves would shard by request, one process per "
              "GPU, with no communication", file=sys.stderr)
        sys.exit(2)
    # one hardware queue per lane plus the context's and torch's streams (HIP's default is 4,
    # and an environment may preset it; two streams on one queue serialise), raised before
    # the runtime starts
    want = min(32, max(4, args.lanes + 2))
    try:
        have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        have = 4
    if have < want:
        os.environ["GPU_MAX_HW_QUEUES"] = str(want)
    log(f"GPU_MAX_HW_QUEUES={os.environ.get('GPU_MAX_HW_QUEUES')}")

    import torch

    if args.calibrate_copy > 0:
        nbytes = int(args.calibrate_copy * 2**30)
        x = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": nbytes, "dispatches": 3}), flush=True)
        return

    import workloads as W
    from paper_2509_13224_amd import ttiga
    from workloads.problem import PREC_FP32, PREC_FP64

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = ttiga.Context(device=0, workspace_bytes=int(args.workspace_gib * 2**30))
    solver = ttiga.TTIGA_SOLVER_AMEN if args.solver == "amen" else ttiga.TTIGA_SOLVER_CG
    other = ttiga.TTIGA_SOLVER_CG if solver == ttiga.TTIGA_SOLVER_AMEN else ttiga.TTIGA_SOLVER_AMEN
    solver_name = {ttiga.TTIGA_SOLVER_AMEN: "amen", ttiga.TTIGA_SOLVER_CG: "tt-cg (preconditioned)"}

    def with_solver(pr, which):
        pr.options.solver = which
        return pr

    base = with_solver(W.c2_problem(n=args.n), solver)
    eps, tol = base.options.tt_eps, base.options.rel_res_tol
    seeds = [W.configs.C2_SEED + b for b in range(args.batch)]
    plain = [with_solver(W.c2_problem(n=args.n, seed=s), solver) for s in seeds]
    plain_other = [with_solver(W.c2_problem(n=args.n, seed=s), other) for s in seeds]
    mixed = [W.c2_problem(n=args.n, seed=s, precision=PREC_FP32) for s in seeds]
    # references by the other method at eps/10, tol/10 (TT-CG for AMEn solves)
    refs_pr = [with_solver(W.c2_problem(n=args.n, seed=s, eps=eps / 10, tol=tol / 10), other) for s in seeds]

    if args.serve_only:
        sv = serving_phase(ctx, args.serve, args.lanes, solver)
        at1 = next(q for q in sv["rates"] if q["fraction_of_saturation"] == 1.0)
        print(json.dumps({
            "metric": "served solves/s at 1e-6 rel-L2 (Poisson arrivals at the mix's saturation rate)",
            "value": at1["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": len(SERVE_RATES) + 1,
            "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if solver else "f32+f64", "data": "synthetic", "config": {"workload": sv["workload"]},
            "serving": sv}),
            flush=True)
        return

    if args.c3_only:
        log("C3 AMEn solve")
        c3 = c3_amen_phase(ctx)
        print(json.dumps({
            "metric": "complex-geometry AMEn solve time", "value": c3["solve_ms"], "unit": "ms", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": c3["solve_ms"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": {"workload": c3["workload"]},
            "c3_amen": c3}), flush=True)
        return

    if args.sweep_only:
        log("TT-matvec sweep")
        only = tuple(int(v) for v in args.sweep_point.split(",")) if args.sweep_point else None
        sw = matvec_sweep(ctx, only=only)
        print(json.dumps({
            "metric": "TT-matvec HBM fraction (synthetic sweep)", "value": sw["max_hbm_frac"], "unit": "fraction",
            "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": {"workload": sw["recipe"]},
            "tt_matvec_sweep": sw}), flush=True)
        return

    if args.batched_only:
        log("batched FP64 steps only")
        for _ in range(args.warmup):
            ctx.solve_batch(plain, lanes=args.lanes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve_batch(plain, lanes=args.lanes)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        print(json.dumps({
            "metric": "solves/s (batched FP64 steps only, accuracy not gated)",
            "value": args.batch * args.steps / elapsed, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{args.batch} C2 problems (annulus degree 3, n={args.n}/dir, TT eps {eps}) "
                                   f"per step on {args.lanes} lanes"}}), flush=True)
        return

    # 1. plain FP64 single solve: latency, roofline of the dominant kernel class
    log("single FP64 solve")
    h = ctx.problem_create(base, precond=1)
    h.assemble()
    h.solve()
    h.close()
    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    lat = []
    for _ in range(2):
        h = ctx.problem_create(base, precond=1)
        t0 = time.perf_counter()
        h.assemble()
        st1 = h.solve()
        u1 = h.solution()
        lat.append(time.perf_counter() - t0)
        h.close()
    ctx.profile(0)
    prof = ctx.profile_read()
    dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    roof = roofline_entry(dom[0], dom[1])
    if args.traffic_kib:
        fetch_kib, write_kib = (float(v) for v in args.traffic_kib.split(","))
        roof["traffic"] = 1024.0 * (fetch_kib + write_kib)
        roof["traffic_source"] = "--traffic-kib"
    else:
        roof["traffic"], roof["traffic_source"] = measured_traffic(dom[0])
    mv = prof.get("tt_matvec_banded")

    if args.single_only:
        print(json.dumps({
            "metric": "solves/s at 1e-6 rel-L2 (plain vs batched/mixed); TT-matvec TFLOP/s; p99 lat",
            "value": 1.0 / (sum(lat) / len(lat)), "unit": "solves/s", "n_gpus": 1, "steps": len(lat),
            "warmup": 1, "ms_per_step": 1e3 * sum(lat) / len(lat), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Fourier source, exact NURBS annulus)",
            "config": {"workload": f"single FP64 solve, annulus degree 3, n={args.n}/dir, TT eps {eps}"},
            "roofline": roof, "iterations": st1["iterations"], "rank_u": st1["rank_u"],
            "kernels": {k: {"ms": v["total_ms"] / len(lat), "launches": v["launches"] / len(lat),
                            "avg_launch_us": 1e3 * v["total_ms"] / max(v["launches"], 1)}
                        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])[:10]}}), flush=True)
        return

    # 2. headline: batches of C2 problems on the executor lanes (FP64)
    log("batched FP64 steps")
    for _ in range(args.warmup):
        ctx.solve_batch(plain, lanes=args.lanes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs, step_ms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        runs.append(ctx.solve_batch(plain, lanes=args.lanes))
        step_ms.append(1e3 * (time.perf_counter() - ts))
        log(f"step {len(runs)}: {step_ms[-1]:.0f} ms, slowest problem "
            f"{max(r['run_ms'] for r, _ in runs[-1]):.0f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # the same steps with the other solver, for the comparison
    log(f"batched FP64 steps, {solver_name[other]}")
    ctx.solve_batch(plain_other, lanes=args.lanes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs_other = [ctx.solve_batch(plain_other, lanes=args.lanes) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed_other = time.perf_counter() - t0
    lat_other = []
    for _ in range(2):
        h = ctx.problem_create(plain_other[0], precond=1)
        t0 = time.perf_counter()
        h.assemble()
        st_other = h.solve()
        lat_other.append(time.perf_counter() - t0)
        h.close()

    # 3. mixed precision batch (FP32 operator inside FP64 refinement)
    log("mixed FP32 batch")
    t0 = time.perf_counter()
    mixed_out = ctx.solve_batch(mixed, lanes=args.lanes)
    mixed_s = time.perf_counter() - t0

    # accuracy gate: FP64 references at eps/10, tol/10
    log("references")
    refs = [u for _, u in ctx.solve_batch(refs_pr, lanes=args.lanes)]
    errs = [[tt_rel_diff(u, refs[b]) if u is not None else float("inf") for b, (_, u) in enumerate(run)]
            for run in runs]
    passed = sum(e <= 1e-6 for run in errs for e in run)
    mixed_err = [tt_rel_diff(u, refs[b]) if u is not None else float("inf") for b, (_, u) in enumerate(mixed_out)]
    single_err = tt_rel_diff(u1, refs[0])
    # the other solver's solves against the same references (by their own method, at eps/10)
    errs_other = [[tt_rel_diff(u, refs[b]) if u is not None else float("inf") for b, (_, u) in enumerate(run)]
                  for run in runs_other]
    passed_other = sum(e <= 1e-6 for run in errs_other for e in run)

    out = {
        "metric": "solves/s at 1e-6 rel-L2 (plain vs batched/mixed); TT-matvec TFLOP/s; p99 lat",
        "value": passed / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "step_ms": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Fourier sources, exact NURBS annulus)",
        "config": {"workload": (f"quarter annulus r 1..2, 90 deg, z 0..1; degree 3, n={args.n}/dir "
                                f"({args.n ** 3} DOF); f = 8 seeded Fourier modes; TT eps {eps}; FP64, "
                                f"{solver_name[solver]} solve; step = {args.batch} such problems "
                                f"(seeds {seeds[0]}..{seeds[-1]}) on {args.lanes} executor lanes"),
                   "precision": "fp64", "solver": args.solver, "tt_eps": eps, "rel_err_tol": tol,
                   "batch": args.batch, "lanes": args.lanes},
        "roofline": roof,
        "accuracy": {"rel_err_vs_ref_max": max(max(r) for r in errs), "passed": passed,
                     "solves": args.batch * args.steps,
                     "reference": (f"FP64 {solver_name[other]} solve of the same problem at eps {eps / 10:g}, "
                                   f"tol {tol / 10:g}")},
        "solver_comparison": {
            solver_name[solver]: {"batched_solves_per_s": passed / elapsed,
                                  "single_latency_ms": 1e3 * sum(lat) / len(lat)},
            solver_name[other]: {"batched_solves_per_s": passed_other / elapsed_other,
                                 "batched_passed": passed_other,
                                 "rel_err_vs_ref_max": max(max(r) for r in errs_other),
                                 "single_latency_ms": 1e3 * sum(lat_other) / len(lat_other),
                                 "iterations": st_other["iterations"], "rank_u": st_other["rank_u"],
                                 "note": "accuracy against the references of its own method at eps/10"}},
        "plain_single": {"solves_per_s": 1.0 / (sum(lat) / len(lat)), "latency_ms": 1e3 * sum(lat) / len(lat),
                         "rel_err": single_err, "iterations": st1["iterations"],
                         "local_iterations": st1.get("local_iterations"), "rank_u": st1["rank_u"],
                         "max_rank_seen": st1["max_rank_seen"], "solver": args.solver},
        "mixed_fp32": {"solves_per_s": sum(e <= 1e-6 for e in mixed_err) / mixed_s,
                       "rel_err_vs_ref_max": max(mixed_err),
                       "refine_steps": [r["refine_steps"] for r, _ in mixed_out],
                       "note": "FP32 operator store and products inside FP64 iterative refinement"},
        "tt_matvec_tflops": (mv["flops"] / (mv["total_ms"] * 1e-3) / 1e12) if mv else None,
        "kernels_single_solve": {k: {"ms": v["total_ms"] / 2, "launches": v["launches"] / 2}
                                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])[:8]},
    }

    # the plain FP64 parity configuration (annulus, degree 2, n = 16, eps = tol = 1e-10): latency of
    # one assembly + solve with each solver, warm context
    log("C1 latency")
    c1 = {}
    for which in (solver, other):
        pr = with_solver(W.configs.c1_problem(), which)
        ts, st = [], None
        for _ in range(4):
            h = ctx.problem_create(pr, precond=1)
            t0 = time.perf_counter()
            h.assemble()
            st = h.solve()
            ts.append(1e3 * (time.perf_counter() - t0))
            h.close()
        c1[solver_name[which]] = {"latency_ms": sum(ts[1:]) / 3, "min_ms": min(ts[1:]), "iterations": st["iterations"],
                                  "rel_res": st["rel_res"], "rank_u": st["rank_u"]}
    out["c1_latency"] = {"workload": "annulus degree 2, n=16/dir, manufactured source, eps = tol = 1e-10, FP64; "
                                     "assembly + solve, mean of 3 after one warm-up", **c1}

    if not args.no_c3:
        log("C3 AMEn solve")
        out["c3_amen"] = c3_amen_phase(ctx)

    if not args.no_sweep:
        log("TT-matvec sweep")
        sw = matvec_sweep(ctx)
        out["tt_matvec_sweep"] = {k: v for k, v in sw.items() if k != "points"}
        out["tt_matvec_sweep"]["best"] = max(sw["points"], key=lambda q: q["hbm_frac"])

    # 4. batched family (mixed sizes/geometries, FP32 mixed) and 5. serving of it
    if args.family > 0:
        log("batched family")
        fam = W.c4_requests(count=args.family, precision=PREC_FP32, assembly_eps=ASSEMBLY_EPS)
        fam_ref_pr = W.c4_requests(count=args.family, precision=PREC_FP64, eps=1e-7, tol=1e-8,
                                   assembly_eps=ASSEMBLY_EPS / 10)
        t0 = time.perf_counter()
        fam_out = ctx.solve_batch(fam, lanes=args.lanes)
        fam_s = time.perf_counter() - t0
        fam_refs = [u for _, u in ctx.solve_batch(fam_ref_pr, lanes=args.lanes)]
        fam_err = [tt_rel_diff(u, ur) if (u is not None and ur is not None) else float("inf")
                   for (_, u), ur in zip(fam_out, fam_refs)]
        fam_ok = sum(e <= 1e-6 for e in fam_err)
        sat = fam_ok / fam_s
        out["batched_family"] = {"requests": args.family, "solves_per_s": sat, "passed": fam_ok,
                                 "rel_err_max": max(fam_err), "seconds": fam_s,
                                 "workload": "n in {32,64,128,256}, p in {2,3}, annulus sector or twisted box, "
                                             "seeded Fourier source, FP32 mixed, seeds 10000+b, "
                                             f"TT eps 1e-6, assembly at {ASSEMBLY_EPS:g}"}
    if args.serve > 0:
        log("serving")
        out["serving"] = serving_phase(ctx, args.serve, args.lanes, solver)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_slabs, args.n)
        # the GPU's rate on the same problem as the oracle sample (single FP64 solve, warm context)
        small = with_solver(W.c2_problem(n=args.cpu_n), solver)
        ts = []
        for _ in range(3):
            h = ctx.problem_create(small, precond=1)
            t0 = time.perf_counter()
            h.assemble()
            h.solve()
            ts.append(time.perf_counter() - t0)
            h.close()
        out["cpu_baseline"]["gpu_same_problem_solves_per_s"] = 1.0 / min(ts[1:])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
