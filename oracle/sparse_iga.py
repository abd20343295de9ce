"""Full-grid sparse IGA: K, F, Dirichlet reduction and a direct solve (Section 3.3).

K[I, J] = sum_q w_q sum_{i,j} dN_I/dxi_i(q) R_ij(q) dN_J/dxi_j(q)   (eqs. Kfinal, K_sum9_matrix_form)
F[I]    = sum_q w_q f(x(q)) N_I(q) det J(q)                          (eq. ffinal)

with q running over the tensor Gauss grid and I = (i0 * n1 + i1) * n2 + i2.
The directional derivative of the tensor-product basis puts the derivative
only in direction i (Section 4.2.1), so the matrix of dN/dxi_i values at the
grid is the Kronecker product of 1-D value / derivative matrices.  This is the
comparison baseline the paper calls full-grid IGA with a sparse solver.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads.problem import BC_CONSTANT, BC_NATURAL, BC_TRACTION, BC_ZERO

from . import bspline, geometry, nurbs


def one_d_tables(problem):
    """Per direction: knots, Gauss nodes, weights, basis values B (Q x n) and derivatives D."""
    p = problem.disc.degree
    tabs = []
    for d, (nodes, wts) in enumerate(geometry.gauss_grid(problem)):
        kn = bspline.open_uniform_knots(problem.disc.n_basis[d], p)
        tabs.append(dict(knots=kn, nodes=nodes, weights=wts,
                         B=bspline.basis(kn, p, nodes), D=bspline.basis_derivative(kn, p, nodes)))
    return tabs


def _kron3(a, b, c):
    return sp.kron(sp.kron(sp.csr_matrix(a), sp.csr_matrix(b)), sp.csr_matrix(c)).tocsr()


def assemble(problem, factors=None):
    """Sparse K (N x N, CSR) and dense F (N) before boundary conditions."""
    tabs = one_d_tables(problem)
    if factors is None:
        factors, _ = geometry.sample_factors_grid(problem)
    W = np.einsum("i,j,k->ijk", tabs[0]["weights"], tabs[1]["weights"], tabs[2]["weights"]).ravel()
    G = [_kron3(tabs[0]["D"], tabs[1]["B"], tabs[2]["B"]),
         _kron3(tabs[0]["B"], tabs[1]["D"], tabs[2]["B"]),
         _kron3(tabs[0]["B"], tabs[1]["B"], tabs[2]["D"])]
    Rfull = np.zeros((3, 3, W.size))
    for idx, (i, j) in enumerate(geometry.R_PAIRS):
        Rfull[i, j] = factors[idx].ravel()
        Rfull[j, i] = factors[idx].ravel()
    N = G[0].shape[1]
    K = sp.csr_matrix((N, N))
    for i in range(3):
        for j in range(3):
            K = K + G[i].T @ sp.diags(W * Rfull[i, j]) @ G[j]
    B0 = _kron3(tabs[0]["B"], tabs[1]["B"], tabs[2]["B"])
    F = B0.T @ (W * factors[6].ravel())
    return K.tocsr(), np.asarray(F).ravel() + traction_load(problem, tabs)


def traction_load(problem, tabs=None):
    """Boundary term of the weak form on natural faces with a flux (Section 3.1):
    F_a += g_f int_face N_a dS, dS = |dx/dxi_i x dx/dxi_j| dxi_i dxi_j over the face's two
    tangential directions, by the tensor Gauss rule of the volume in those directions."""
    if tabs is None:
        tabs = one_d_tables(problem)
    n = problem.disc.n_basis
    F = np.zeros(tuple(n))
    for face in range(6):
        if problem.dirichlet.kind[face] != BC_TRACTION:
            continue
        d, side = divmod(face, 2)
        i, j = [e for e in range(3) if e != d]
        nodes = [tabs[e]["nodes"] for e in range(3)]
        nodes[d] = np.array([float(side)])
        _, J = nurbs.solid_map_grid(problem.geometry, *nodes)
        Js = np.linalg.norm(np.cross(J[..., :, i], J[..., :, j]), axis=-1)
        Js = Js.reshape(len(tabs[i]["nodes"]), len(tabs[j]["nodes"]))
        Wf = np.outer(tabs[i]["weights"], tabs[j]["weights"]) * Js
        S = tabs[i]["B"].T @ Wf @ tabs[j]["B"]  # (n_i, n_j)
        sl = [slice(None)] * 3
        sl[d] = 0 if side == 0 else n[d] - 1
        F[tuple(sl)] += problem.dirichlet.value[face] * S
    return F.ravel()


def dirichlet_values(problem):
    """Boundary DOF mask and prescribed coefficients (constant faces; later faces win)."""
    n = problem.disc.n_basis
    mask = np.zeros(tuple(n), dtype=bool)
    vals = np.zeros(tuple(n))
    for face in range(6):
        kind = problem.dirichlet.kind[face]
        if kind in (BC_NATURAL, BC_TRACTION):
            continue
        d, side = divmod(face, 2)
        sl = [slice(None)] * 3
        sl[d] = 0 if side == 0 else n[d] - 1
        mask[tuple(sl)] = True
        vals[tuple(sl)] = problem.dirichlet.value[face] if kind == BC_CONSTANT else 0.0
        if kind not in (BC_ZERO, BC_CONSTANT):
            raise ValueError("unknown boundary kind")
    return mask.ravel(), vals.ravel()


def solve(problem, K=None, F=None, return_system=False):
    """Solve K_II u_I = F_I - K_IB u_B by sparse LU; returns the full coefficient vector."""
    if K is None:
        K, F = assemble(problem)
    mask, vals = dirichlet_values(problem)
    I = np.flatnonzero(~mask)
    Bd = np.flatnonzero(mask)
    KII = K[I][:, I].tocsc()
    rhs = F[I] - K[I][:, Bd] @ vals[Bd]
    uI = spla.splu(KII).solve(rhs)
    u = vals.copy()
    u[I] = uI
    if return_system:
        return u, dict(KII=KII, rhs=rhs, interior=I, boundary=Bd, u_B=vals[Bd])
    return u


def condition_estimate(KII):
    """kappa(K_II) from the extreme eigenvalues (Lanczos)."""
    lmax = spla.eigsh(KII, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(KII, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return float(lmax / lmin)
