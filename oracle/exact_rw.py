"""Basic ("exact") random walker (oracle; test infrastructure only).

Sec. II-A: seeded voxels are ordered first (eq. (1)), L is split into blocks [L_s, B; B^T, L_n]
(eq. (4)), and for every label k the minimiser of eq. (3) solves eq. (5):

    (L_n + gamma I_n) U_n = gamma P_n - B^T U_s.

U_s is the 0/1 matrix of the seeds (one 1 per row).  With gamma = 0 this is the pure seeded random
walker; the answer is the same whether L or L_hat is used (Sec. II-C substitution U_hat = D^{1/2} U),
so the oracle always solves with the unnormalized L here.

Solvers: Jacobi-preconditioned CG in FP64 to a relative residual (the benchmark's 1e-12), a sparse
direct LU (scipy splu), or a dense numpy solve for tiny graphs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def seed_split(N, seed_node):
    s = np.asarray(seed_node, dtype=np.int64)
    is_seed = np.zeros(N, dtype=bool)
    is_seed[s] = True
    n = np.flatnonzero(~is_seed)
    return s, n


def one_hot(seed_label, C):
    Us = np.zeros((len(seed_label), C))
    Us[np.arange(len(seed_label)), np.asarray(seed_label)] = 1.0
    return Us


def pcg(A, b, tol=1e-12, max_iter=100000, x0=None):
    """Jacobi-preconditioned conjugate gradients (textbook, FP64).  Stops when
    ||b - A x|| <= tol * ||b||.  Returns (x, iterations, final relative residual)."""
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * bn and it < max_iter:
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(b - A @ x) / bn


def exact_rw(graph, seed_node, seed_label, C, method="cg", tol=1e-12, gamma=0.0, prior=None,
             return_info=False):
    """Label probabilities U (N x C) of the basic random walker, Sec. II-A eq. (5).

    prior: N x C matrix P (only used when gamma > 0)."""
    L = graph.L()
    N = graph.N
    s, n = seed_split(N, seed_node)
    Us = one_hot(seed_label, C)
    Ln = L[n][:, n].tocsc()
    B = L[s][:, n]
    rhs = -(B.T @ Us)
    if gamma > 0.0:
        Ln = (Ln + gamma * sp.eye(n.size)).tocsc()
        rhs = rhs + gamma * np.asarray(prior)[n]
    Un = np.zeros((n.size, C))
    iters = []
    if method == "cg":
        for k in range(C):
            Un[:, k], it, _ = pcg(Ln, np.ascontiguousarray(rhs[:, k]), tol=tol)
            iters.append(it)
    elif method == "direct":
        lu = spla.splu(Ln)
        Un = lu.solve(np.ascontiguousarray(rhs))
    elif method == "dense":
        Un = np.linalg.solve(Ln.toarray(), rhs)
    else:
        raise ValueError(method)
    U = np.zeros((N, C))
    U[s] = Us
    U[n] = Un
    if return_info:
        return U, {"cg_iters": iters}
    return U
