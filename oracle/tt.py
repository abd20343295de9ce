"""Tensor-train format (Section 4.1.1) and its standard algorithms.

A TT tensor is a list of cores G_k of shape (r_{k-1}, n_k, r_k) with
r_0 = r_d = 1; X(i_1..i_d) = G_1(:, i_1, :) ... G_d(:, i_d, :).  A TT matrix
has cores M_k of shape (r_{k-1}, n_k, n_k, r_k) (row index first).  A rank-0
tensor (the exact zero) is represented by ``None``.

TT-SVD and TT-rounding are the algorithms of Oseledets (2011), cited by the
paper as the basis of its TT format and of the rounding applied after each
summation (Section 4.2.1): sequential truncated SVDs of the unfoldings with
per-unfolding threshold delta = eps ||X||_F / sqrt(d-1); rounding first makes
the train right-orthogonal with QR factorisations and then truncates the
unfoldings from left to right.
"""
import numpy as np


def trunc_rank(s, delta):
    """Smallest r with sqrt(sum_{i >= r} s_i^2) <= delta (s sorted descending)."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[r] = ||s[r:]||
    for r in range(len(s)):
        if tail[r] <= delta:
            return r
    return len(s)


def full(cores):
    """Dense tensor of shape (n_1, ..., n_d)."""
    if cores is None:
        raise ValueError("zero tensor has no shape here")
    X = cores[0]
    for G in cores[1:]:
        X = np.tensordot(X, G, axes=([-1], [0]))
    return X[0, ..., 0]


def tt_svd(A, eps=None, delta=None, max_rank=None):
    """TT-SVD: eps-relative (delta = eps ||A|| / sqrt(d-1)) or an absolute per-unfolding delta."""
    A = np.asarray(A, dtype=np.float64)
    d = A.ndim
    if delta is None:
        delta = eps * np.linalg.norm(A) / np.sqrt(d - 1)
    cores = []
    r = 1
    C = A.reshape(1, -1)
    for k in range(d - 1):
        C = C.reshape(r * A.shape[k], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = trunc_rank(s, delta)
        if max_rank is not None:
            rk = min(rk, max_rank)
        if rk == 0:
            return None
        cores.append(U[:, :rk].reshape(r, A.shape[k], rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, A.shape[-1], 1))
    return cores


def ranks(cores):
    if cores is None:
        return None
    return [1] + [G.shape[-1] for G in cores]


def add(a, b):
    """Sum of two TT tensors: block-diagonal middle cores, concatenated end cores."""
    if a is None:
        return b
    if b is None:
        return a
    d = len(a)
    out = []
    for k, (A, B) in enumerate(zip(a, b)):
        ra0, n, ra1 = A.shape
        rb0, _, rb1 = B.shape
        if k == 0:
            C = np.concatenate([A, B], axis=2)
        elif k == d - 1:
            C = np.concatenate([A, B], axis=0)
        else:
            C = np.zeros((ra0 + rb0, n, ra1 + rb1))
            C[:ra0, :, :ra1] = A
            C[ra0:, :, ra1:] = B
        out.append(C)
    return out


def scale(a, alpha):
    if a is None:
        return None
    out = [G.copy() for G in a]
    out[0] = out[0] * alpha
    return out


def dot(a, b):
    """<a, b> by the left-to-right contraction of the two trains."""
    if a is None or b is None:
        return 0.0
    L = np.ones((1, 1))
    for A, B in zip(a, b):
        L = np.einsum("xy,xiu,yiv->uv", L, A, B)
    return float(L[0, 0])


def norm(a):
    """||a||_F computed from an orthogonalised train (no cancellation)."""
    if a is None:
        return 0.0
    c = orthogonalize_left(a)
    return float(np.linalg.norm(c[-1]))


def orthogonalize_left(a):
    """Left-orthogonal copy: QR of each unfolding (r_{k-1} n_k) x r_k, R pushed to the right."""
    cores = [G.copy() for G in a]
    for k in range(len(cores) - 1):
        r0, n, r1 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r0 * n, r1))
        cores[k] = Q.reshape(r0, n, Q.shape[1])
        cores[k + 1] = np.tensordot(R, cores[k + 1], axes=([1], [0]))
    return cores


def round_(a, eps=None, delta=None, max_rank=None):
    """TT-rounding (Oseledets 2011): right-to-left QR sweep, then left-to-right truncated SVD.

    The threshold per unfolding is eps ||a|| / sqrt(d-1), or an absolute delta.
    """
    if a is None:
        return None
    d = len(a)
    cores = [G.copy() for G in a]
    for k in range(d - 1, 0, -1):
        r0, n, r1 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r0, n * r1).T)
        cores[k] = Q.T.reshape(Q.shape[1], n, r1)
        cores[k - 1] = np.tensordot(cores[k - 1], R.T, axes=([2], [0]))
    nrm = np.linalg.norm(cores[0])
    if delta is None:
        delta = eps * nrm / np.sqrt(d - 1)
    for k in range(d - 1):
        r0, n, r1 = cores[k].shape
        U, s, Vt = np.linalg.svd(cores[k].reshape(r0 * n, r1), full_matrices=False)
        rk = trunc_rank(s, delta)
        if max_rank is not None:
            rk = min(rk, max_rank)
        if rk == 0:
            return None
        cores[k] = U[:, :rk].reshape(r0, n, rk)
        cores[k + 1] = np.tensordot(s[:rk, None] * Vt[:rk], cores[k + 1], axes=([1], [0]))
    return cores


# ---------------------------------------------------------------- TT matrices

def mat_full(mcores):
    """Dense matrix of a TT matrix, rows and columns flattened with the first index slowest."""
    X = mcores[0]
    for M in mcores[1:]:
        X = np.tensordot(X, M, axes=([-1], [0]))
    X = X[0, ..., 0]  # (n1, m1, n2, m2, ..., nd, md)
    d = len(mcores)
    perm = list(range(0, 2 * d, 2)) + list(range(1, 2 * d, 2))
    X = X.transpose(perm)
    N = int(np.prod([M.shape[1] for M in mcores]))
    Mc = int(np.prod([M.shape[2] for M in mcores]))
    return X.reshape(N, Mc)


def mat_as_tt(mcores):
    """View a TT matrix as a TT tensor with merged physical index (i_k, j_k)."""
    if mcores is None:
        return None
    return [M.reshape(M.shape[0], M.shape[1] * M.shape[2], M.shape[3]) for M in mcores]


def tt_as_mat(cores, shapes):
    if cores is None:
        return None
    return [G.reshape(G.shape[0], n, m, G.shape[2]) for G, (n, m) in zip(cores, shapes)]


def mat_add(a, b):
    if a is None:
        return b
    if b is None:
        return a
    shapes = [(M.shape[1], M.shape[2]) for M in a]
    return tt_as_mat(add(mat_as_tt(a), mat_as_tt(b)), shapes)


def mat_round(a, eps=None, delta=None):
    if a is None:
        return None
    shapes = [(M.shape[1], M.shape[2]) for M in a]
    return tt_as_mat(round_(mat_as_tt(a), eps=eps, delta=delta), shapes)


def matvec(mcores, x):
    """y = K x in TT: cores y_k[(b, a), i, (b', a')] = sum_j M_k[b, i, j, b'] x_k[a, j, a']."""
    if mcores is None or x is None:
        return None
    out = []
    for M, X in zip(mcores, x):
        Y = np.einsum("bijc,ajd->baicd", M, X)
        b, a, n, c, dd = Y.shape
        out.append(Y.reshape(b * a, n, c * dd))
    return out
