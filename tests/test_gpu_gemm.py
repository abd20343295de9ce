"""The FP64 MFMA product behind every TT contraction, against numpy's product on the host.

Every entry must lie within the standard forward error bound of a length-K dot product,
|C - C_ref| <= 2 K u (|op(A)| |op(B)|) + |beta| u |C0| (u = 2^-53), for every tile variant,
transpose combination, K split, batch and ragged edge; a repeated call gives the same bits.
"""
import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

U = 2.0 ** -53

SHAPES = [
    # (M, N, K, batch): ragged tails in every dimension, the 128-wide tile cases, long
    # contractions that split, and a batch
    (1, 1, 1, 1),
    (3, 9, 254, 1),
    (75, 300, 728, 1),
    (300, 75, 536, 1),
    (64, 64, 64, 1),
    (65, 129, 33, 1),
    (17, 5000, 18, 1),
    (254, 67, 254, 7),
    (40, 30, 3000, 1),
    (130, 140, 100, 3),
    # skinny tiles (N or M at most 16): the preconditioner's 1-D transforms, dot-like products
    (254, 3, 254, 15),
    (5, 300, 700, 2),
    (16, 16, 1012, 1),
    (1, 2286, 1, 1),
]


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2509_13224_amd import ttiga
    return ttiga.Context(workspace_bytes=2 << 30)


def _run(ctx, ta, tb, M, N, K, batch, alpha, beta, plan, seed):
    import torch
    rng = np.random.default_rng(seed)
    a_shape = (batch, K, M) if ta else (batch, M, K)
    b_shape = (batch, N, K) if tb else (batch, K, N)
    A = rng.normal(size=a_shape)
    B = rng.normal(size=b_shape)
    C0 = rng.normal(size=(batch, M, N))
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = alpha * np.matmul(opA, opB) + beta * C0
    bound = 2 * K * U * abs(alpha) * np.matmul(np.abs(opA), np.abs(opB)) + 2 * U * abs(beta) * np.abs(C0)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    outs = []
    for _ in range(2):
        dC = torch.from_numpy(C0).cuda()
        ctx.gemm_f64(ta, tb, M, N, K, alpha, dA, a_shape[2], dB, b_shape[2], beta, dC, N, batch=batch,
                     sA=a_shape[1] * a_shape[2], sB=b_shape[1] * b_shape[2], sC=M * N, plan=plan)
        outs.append(dC.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]), "repeated product differs"
    err = np.abs(outs[0] - ref)
    assert np.all(err <= bound + 1e-300), (float(np.max(err / (bound + 1e-300))), M, N, K, ta, tb, plan)
    return outs[0]


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_default_plan(ctx, ta, tb, shape):
    M, N, K, batch = shape
    say("gemm", ta, tb, shape)
    _run(ctx, ta, tb, M, N, K, batch, 1.0, 0.0, None, seed=M * 7 + N * 13 + K)
    _run(ctx, ta, tb, M, N, K, batch, -0.5, 2.0, None, seed=M + N + K)


@pytest.mark.parametrize("plan", [(64, 64, 0), (128, 64, 0), (64, 128, 0), (64, 64, 64), (128, 64, 96),
                                  (64, 128, 160), (64, 16, 0), (16, 64, 0), (64, 16, 64), (16, 64, 96)])
def test_gemm_every_plan(ctx, plan):
    say("gemm plan", plan)
    for ta in (0, 1):
        for tb in (0, 1):
            _run(ctx, ta, tb, 131, 77, 333, 2, 1.5, 0.25, plan, seed=plan[0] + plan[2])


def test_gemm_rejects_bad_arguments(ctx):
    import torch

    from paper_2509_13224_amd import ttiga
    say("gemm bad args")
    A = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(ttiga.TTIGAError):
        ctx.gemm_f64(0, 0, 4, 4, 4, 1.0, A, 2, A, 4, 0.0, A, 4)  # lda shorter than a row
    with pytest.raises(ttiga.TTIGAError):
        ctx.gemm_f64(0, 0, 4, 4, 4, 1.0, A, 4, A, 4, 0.0, A, 4, plan=(32, 32, 0))
    with pytest.raises(ttiga.TTIGAError):
        ctx.gemm_f64(0, 0, 4, 4, 4, 1.0, A, 4, A, 4, 0.0, A, 4, plan=(64, 64, 48))  # chunk not a multiple of 32


def _round_lowp(x, dtype):
    """The operand rounding of the low-precision product: FP64 -> FP32 (nearest even), and for
    BF16 FP32 -> BF16 (nearest even on the upper 16 bits), exactly as the host can emulate it."""
    f = x.astype(np.float32)
    if dtype == 2:
        u = f.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        f = u.astype(np.uint32).view(np.float32)
    return f.astype(np.float64)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("shape", [(70, 130, 300, 1), (5, 9, 33, 3), (200, 64, 1200, 1)])
def test_gemm_lowp_matches_rounded_operands(ctx, dtype, ta, tb, shape):
    """The low-precision MFMA product equals the exact product of the rounded operands within the
    FP32 accumulation bound 2 K u32 (|A_r| |B_r|): the operand rounding, the MFMA operand and
    result layouts and the K splits are all checked by it."""
    import torch
    M, N, K, batch = shape
    say("gemm lowp", dtype, ta, tb, shape)
    rng = np.random.default_rng(M + N + K + dtype)
    a_shape = (batch, K, M) if ta else (batch, M, K)
    b_shape = (batch, N, K) if tb else (batch, K, N)
    A = rng.normal(size=a_shape)
    B = rng.normal(size=b_shape)
    C0 = rng.normal(size=(batch, M, N))
    Ar, Br = _round_lowp(A, dtype), _round_lowp(B, dtype)
    opA = np.swapaxes(Ar, 1, 2) if ta else Ar
    opB = np.swapaxes(Br, 1, 2) if tb else Br
    alpha, beta = 0.75, -0.5
    ref = alpha * np.matmul(opA, opB) + beta * C0
    bound = 2 * K * 2.0 ** -24 * abs(alpha) * np.matmul(np.abs(opA), np.abs(opB)) + 2 * U * abs(beta) * np.abs(C0)
    dC = torch.from_numpy(C0).cuda()
    ctx.gemm_lowp(dtype, ta, tb, M, N, K, alpha, torch.from_numpy(A).cuda(), a_shape[2], torch.from_numpy(B).cuda(),
                  b_shape[2], beta, dC, N, batch=batch, sA=a_shape[1] * a_shape[2], sB=b_shape[1] * b_shape[2],
                  sC=M * N)
    err = np.abs(dC.cpu().numpy() - ref)
    assert np.all(err <= bound + 1e-300), float(np.max(err / (bound + 1e-300)))
