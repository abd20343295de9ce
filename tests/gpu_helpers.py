"""Shared helpers of the GPU parity tests (data reshaping only; comparisons use the oracle)."""
import sys

import numpy as np


def say(*a):
    """Flush the name of the case before each GPU step, so a failure names it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def banded_to_dense_cores(cores, p):
    """Banded TT-matrix cores [r][n][2p+1][r'] -> dense [r][n][n][r']."""
    out = []
    for M in cores:
        r0, n, band, r1 = M.shape
        D = np.zeros((r0, n, n, r1))
        for i in range(n):
            for t in range(band):
                j = i + t - p
                if 0 <= j < n:
                    D[:, i, j, :] = M[:, i, t, :]
        out.append(D)
    return out


def dense_to_banded_cores(cores, p):
    out = []
    for D in cores:
        r0, n, _, r1 = D.shape
        M = np.zeros((r0, n, 2 * p + 1, r1))
        for i in range(n):
            for t in range(2 * p + 1):
                j = i + t - p
                if 0 <= j < n:
                    M[:, i, t, :] = D[:, i, j, :]
        out.append(M)
    return out


def rand_tt(shape, ranks, rng):
    r = [1] + list(ranks) + [1]
    return [rng.normal(size=(r[k], n, r[k + 1])) for k, n in enumerate(shape)]


def rand_banded(shape, ranks, p, rng):
    r = [1] + list(ranks) + [1]
    cores = []
    for k, n in enumerate(shape):
        M = rng.normal(size=(r[k], n, 2 * p + 1, r[k + 1]))
        for i in range(n):
            for t in range(2 * p + 1):
                if not 0 <= i + t - p < n:
                    M[:, i, t, :] = 0.0
        cores.append(M)
    return cores


def to_dev(cores, device="cuda:0"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in cores]


def tt_rel_diff(a, b):
    """||a - b|| / ||b|| for host TT cores (3 cores): the difference train [a, -b] is
    left-orthogonalised by QR and its norm read from the last core, so differences far below
    ||b|| are resolved (no cancellation between <a,a>, <a,b> and <b,b>)."""
    def orth_norm(cores):
        cores = [c.copy() for c in cores]
        for k in range(len(cores) - 1):
            r0, n, r1 = cores[k].shape
            _, r = np.linalg.qr(cores[k].reshape(r0 * n, r1))
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


def same_tt(a, b):
    """True when two host TTs have the same ranks and bit-identical cores."""
    return len(a) == len(b) and all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b))
