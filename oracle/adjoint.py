"""Exact adjoint of the basic random walker (oracle; test infrastructure only).

The forward map is the gamma = 0 system of Sec. II-A eq. (5): L_n U_n = -B^T U_s, with L = D - W and
the weights of eq. (2).  Writing L = sum_e w_e (e_i - e_j)(e_i - e_j)^T and differentiating,
L_n dU_n = -[dL U]_n.  With the adjoint A_n = L_n^{-1} G_n for a loss gradient G = dl/dU (A = 0 on
the seed rows),  dl/dw_e = -sum_k (a_i^k - a_j^k)(u_i^k - u_j^k).  The chain rule through
w_e = s_e exp(-beta (J_i - J_j)^2) gives the gradients for intensities, beta and per-edge scales.

The loss (a reading; the paper trains nothing): mean over non-seed voxels of -log max(p_{i,y_i}, 1e-12)
for a ground-truth label y_i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .exact_rw import exact_rw, pcg, seed_split

P_FLOOR = 1e-12


def ce_loss(U, gt, seed_node):
    N = U.shape[0]
    _, n = seed_split(N, seed_node)
    p = np.maximum(U[n, np.asarray(gt)[n]], P_FLOOR)
    return float(-np.mean(np.log(p)))


def ce_grad(U, gt, seed_node):
    """dl/dU for ce_loss (zero on seeds and where the floor is active)."""
    N, C = U.shape
    _, n = seed_split(N, seed_node)
    G = np.zeros((N, C))
    y = np.asarray(gt)[n]
    p = U[n, y]
    act = p > P_FLOOR
    G[n[act], y[act]] = -1.0 / (n.size * p[act])
    return G


def adjoint_grads(graph, seed_node, seed_label, C, G, U=None, method="direct", tol=1e-12):
    """(dl/dw [per edge, graph.edge_id order], dl/dJ [N], dl/dbeta, dl/ds [per edge]) for a loss
    gradient G = dl/dU (N x C) at the exact forward solution.  The adjoint system L_n A_n = G_n is solved
    by sparse LU (method "direct") or, on graphs too large to factor, by the Jacobi-preconditioned CG of
    exact_rw (method "cg", relative residual tol per label)."""
    if U is None:
        U = exact_rw(graph, seed_node, seed_label, C, method=method, tol=tol)
    L = graph.L()
    s, n = seed_split(graph.N, seed_node)
    A = np.zeros_like(U)
    if method == "direct":
        lu = spla.splu(L[n][:, n].tocsc())
        A[n] = lu.solve(np.ascontiguousarray(G[n]))
    elif method == "cg":
        Ln = L[n][:, n].tocsr()
        for k in range(C):
            A[n, k] = pcg(Ln, np.ascontiguousarray(G[n, k]), tol=tol)[0]
    else:
        raise ValueError(method)
    t, h = graph.tail, graph.head
    dw = -np.sum((A[t] - A[h]) * (U[t] - U[h]), axis=1)
    w = graph.w
    diff = graph.J[t] - graph.J[h]
    if graph.weight_form != "squared":
        raise NotImplementedError("adjoint implemented for the squared weight form")
    dJ = np.zeros(graph.N)
    np.add.at(dJ, t, dw * w * (-2.0 * graph.beta * diff))
    np.add.at(dJ, h, dw * w * (2.0 * graph.beta * diff))
    dbeta = float(np.sum(dw * w * (-diff * diff)))
    ds = np.where(graph.present, dw * graph.base_weight(), 0.0)
    return dw, dJ, dbeta, ds


def loss_of(graph, seed_node, seed_label, C, gt):
    U = exact_rw(graph, seed_node, seed_label, C, method="direct")
    return ce_loss(U, gt, seed_node)
