#!/usr/bin/env python3
"""Offline tile tuner of the FP64 GEMM kernel (writes csrc/gemm_table.inc).

The library picks the tile (64x64, 128x64, 64x128, 64x16 or 16x64) and the contraction split of every
product from a table compiled into it, keyed by shape bucket (transposes, ceil log2 of M, N,
K, batched or not), with a fixed rule for shapes the table does not list.  So the choice is
deterministic at run time and the same in every process; this script is what fills the table,
once per hardware, by measurement:

1. trace: run representative workloads (the annulus at n = 256, the complex geometry at
   n = 128 and a slice of the serving mix, each by preconditioned TT-CG and by AMEn) in a child
   process with TTIGA_GEMM_TRACE=1, which makes the library print the shape of every product;
2. time: for the most frequent shape of every bucket, every tile with contraction chunks of
   {whole K, 2048, 1024, 512, 256, 128, 64} (multiples of 32) through ttiga_gemm_f64 on random
   operands: the mean kernel time of 10 products from the library's per-kernel events (so the
   host round trip of each synchronous call is not counted), median of 3 such runs after a
   warm-up;
3. choose: a bucket gets a table entry when its best plan differs from the rule's plan and
   still beats it by more than 5% when the two are timed again, alternately, three times each;
   the entry stores the tile and the contraction chunk.

Usage (on the GPU): python paper_2509_13224_amd/tune_gemm.py [--out csrc/gemm_table.inc]
The table is a build input: rebuild after writing it.
"""
import argparse
import collections
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

TILES = ((64, 64), (128, 64), (64, 128), (64, 16), (16, 64))
CHUNKS = (0, 2048, 1024, 512, 256, 128, 64)  # 0: the whole contraction in one pass
GAIN = 1.05

TRACE_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import workloads as W
from paper_2509_13224_amd import ttiga
from workloads.problem import PREC_FP64
ctx = ttiga.Context(workspace_bytes=64 << 30)
probs = []
for solver in (0, 1):  # preconditioned TT-CG, AMEn
    batch = [W.c2_problem(n=256), W.c3_problem(n=128, precision=PREC_FP64)] + W.c4_requests(count=12,
                                                                                          precision=PREC_FP64)
    for pr in batch:
        pr.options.solver = solver
    probs += batch
for pr in probs:
    h = ctx.problem_create(pr, precond=1)
    h.assemble()
    h.solve(allow_notconv=True)
    h.close()
"""


def ceil_log2(v):
    b = 0
    while (1 << b) < v:
        b += 1
    return b


def bucket(ta, tb, M, N, K, batch):
    return (ta, tb, ceil_log2(M), ceil_log2(N), ceil_log2(K), 1 if batch > 1 else 0)


def trace_shapes():
    env = dict(os.environ, TTIGA_GEMM_TRACE="1")
    r = subprocess.run([sys.executable, "-c", TRACE_SCRIPT.format(root=ROOT)], capture_output=True, text=True,
                       env=env, timeout=1200)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-3000:])
    shapes = collections.Counter()
    for line in r.stderr.splitlines():
        m = re.match(r"\[gemm-shape\] ta=(\d) tb=(\d) M=(\d+) N=(\d+) K=(\d+) batch=(\d+)", line)
        if m:
            shapes[tuple(int(v) for v in m.groups())] += 1
    return shapes


def time_plan(ctx, torch, shape, plan, reps=3, inner=10):
    """Median over `reps` runs of the mean kernel time (ms) of `inner` products: the library's
    own per-kernel events (taken at each kernel's start and end, split-K reduction included), so
    the host round trip of the synchronous entry point between products is not counted."""
    ta, tb, M, N, K, batch = shape
    a_shape = (batch, K, M) if ta else (batch, M, K)
    b_shape = (batch, N, K) if tb else (batch, K, N)
    A = torch.randn(a_shape, dtype=torch.float64, device="cuda")
    B = torch.randn(b_shape, dtype=torch.float64, device="cuda")
    C = torch.zeros((batch, M, N), dtype=torch.float64, device="cuda")
    args = dict(batch=batch, sA=a_shape[1] * a_shape[2], sB=b_shape[1] * b_shape[2], sC=M * N, plan=plan)
    times = []
    for r in range(reps + 1):
        ctx.profile(-1)
        ctx.profile(1)
        for _ in range(inner):
            ctx.gemm_f64(ta, tb, M, N, K, 1.0, A, a_shape[2], B, b_shape[2], 0.0, C, N, **args)
        ctx.profile(0)
        st = ctx.profile_read()["gemm_f64"]
        if r >= 1:
            times.append(st["total_ms"] / inner)
    return sorted(times)[len(times) // 2]


def confirmed_gain(ctx, torch, shape, rule, best, rounds=3):
    """rule time / best time, each the sum of `rounds` alternate measurements."""
    tr = tb = 0.0
    for _ in range(rounds):
        tr += time_plan(ctx, torch, shape, rule)
        tb += time_plan(ctx, torch, shape, best)
    return tr / tb


def rule_plan(M, N, K, batch):
    """The library's rule (gemm_plan without a table entry) as (bm, bn, kchunk), for the
    comparison."""
    bm = bn = 64
    square_tiles = ((M + 63) // 64) * ((N + 63) // 64) * batch
    if N <= 16 and (M > 16 or M >= N):
        bn = 16
    elif M <= 16:
        bm = 16
    elif square_tiles < 512:
        bm, bn = (64, 16) if M >= N else (16, 64)
    tiles = ((M + bm - 1) // bm) * ((N + bn - 1) // bn) * batch
    kchunk = 0
    if tiles < 256 and K >= 320:
        s = min((K + 255) // 256, max(1, 512 // tiles))
        kchunk = (K + s - 1) // s
        kchunk = (kchunk + 31) // 32 * 32
    return (bm, bn, kchunk)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "gemm_table.inc"))
    args = ap.parse_args()
    import torch

    from paper_2509_13224_amd import ttiga
    shapes = trace_shapes()
    buckets = collections.defaultdict(collections.Counter)
    for sh, cnt in shapes.items():
        buckets[bucket(*sh)][sh] += cnt
    print(f"{sum(shapes.values())} products, {len(shapes)} shapes, {len(buckets)} buckets", file=sys.stderr)
    ctx = ttiga.Context(workspace_bytes=8 << 30)
    entries = []
    for bi, key in enumerate(sorted(buckets)):
        sh, cnt = buckets[key].most_common(1)[0]
        print(f"bucket {bi + 1}/{len(buckets)} {key} {sh} x{cnt}", file=sys.stderr, flush=True)
        ta, tb, M, N, K, batch = sh
        if M * N * batch * 8 > (1 << 31) or M * K * batch * 8 > (1 << 31) or K * N * batch * 8 > (1 << 31):
            continue
        rule = rule_plan(M, N, K, batch)
        base = time_plan(ctx, torch, sh, rule)
        best, best_t = None, base
        for bm, bn in TILES:
            for ch in CHUNKS:
                if ch and ch >= K:
                    continue
                splits = 1 if ch == 0 else (K + ch - 1) // ch
                if batch * splits > 65535:
                    continue
                t = time_plan(ctx, torch, sh, (bm, bn, ch))
                if t * GAIN < best_t:
                    best, best_t = (bm, bn, ch), t
        if best and best != rule:
            gain = confirmed_gain(ctx, torch, sh, rule, best)
            if gain < GAIN:
                print(f"{key} {sh}: {best} not confirmed ({gain:.3f})", file=sys.stderr)
                continue
            entries.append((key, best, base, best_t))
            print(f"{key} {sh} x{cnt}: rule {base * 1e3:.1f} us -> {best} {best_t * 1e3:.1f} us", file=sys.stderr)
    with open(args.out, "w") as f:
        f.write("// Generated by paper_2509_13224_amd/tune_gemm.py from timings on MI355X; rebuild after\n")
        f.write("// regenerating.  {ta, tb, ceil log2 M, N, K, batched, tile rows, tile cols, contraction\n")
        f.write("// chunk (0: whole K)}, sorted by key; buckets not listed follow gemm_plan's rule.\n")
        for (key, (bm, bn, ch), base, t) in entries:
            f.write("{%d, %d, %d, %d, %d, %d, %d, %d, %d},  // rule %.1f us, tuned %.1f us\n"
                    % (*key, bm, bn, ch, base * 1e3, t * 1e3))
    print(f"wrote {len(entries)} entries to {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
