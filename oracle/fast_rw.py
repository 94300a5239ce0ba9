"""Precomputed-eigenvector ("fast") random walker (oracle; test infrastructure only).

Sec. II-B.  With E = Q (Lambda + gamma I)^{-1} Q^T (eq. (7)) split into blocks
[E_s, R; R^T, E_n] (eqs. (8)-(9)) and the auxiliary unknown F = (L + gamma I) U (eqs. (10)-(13)),
left-multiplying by E gives U_n = R^T F_s + gamma E_n P_n (eq. (15)), and eliminating U_n from
eq. (11) gives the S x S seed system  (I - B R^T) F_s = L_s U_s + gamma (U_s + B E_n P_n)  (eq. (17)).

gamma = 0 (the paragraph after eq. (17)): L has the null vector g, so E L = I - g g^T and eq. (14)
must be altered; the paper points to first computing g_n^T U_n (the column sums of U_n) and using
them to obtain F_s, without giving the equations.  Reading used here (derived from the same
equations): write U = E F + g c^T with c^T = g^T U, where E = Q' Lambda'^{-1} Q'^T is built from the
eigenpairs other than the null pair.  Then, with F_n = 0 (eq. (13) with gamma = 0):

    U_n = R^T F_s + g_n c^T,                 R^T = Q'_n Lambda'^{-1} Q'_s^T
    (I - B R^T) F_s - B g_n c^T = L_s U_s    (eq. (11) with U_n substituted)
    g_s^T F_s = 0                            (g^T F = g^T L U = 0 and F_n = 0)

an (S+1) x (S+1) bordered system in (F_s, c).  It is exact when Q holds all N eigenvectors, and the
rows of U sum to 1 for any truncation.

Normalized Laplacian (Sec. II-C): every quantity is taken in hat variables, L -> L_hat,
U_s -> D_s^{1/2} U_s, g -> D^{1/2} 1 / ||D^{1/2} 1||, and U = D^{-1/2} U_hat at the end.
A node with d = 0 (no edges at all) gets U = 0.
"""
from __future__ import annotations

import numpy as np

from .eigen import insert_null
from .exact_rw import one_hot, seed_split


def _seed_blocks(graph, seed_node):
    M = graph.M().tocsr()
    N = graph.N
    s, n = seed_split(N, seed_node)
    Ms_rows = M[s]                       # S x N
    Ms = Ms_rows[:, s]                   # L_s  (seed-seed block)
    B_full = Ms_rows.tolil(copy=True)    # B with the seed columns zeroed, kept N wide
    B_full[:, s] = 0.0
    B_full = B_full.tocsr()
    return M, s, n, Ms, B_full


def fast_rw_coeffs(graph, Q, lam, seed_node, seed_label, C, m=None):
    """Solve the gamma = 0 bordered system.  Returns (Qp, Y, c) such that the hat-variable
    probabilities at a non-seed node i are  Qp[i] @ Y + ghat[i] * c."""
    m = Q.shape[1] if m is None else m
    ghat = graph.ghat()
    Qm, lm = insert_null(np.asarray(Q, dtype=np.float64)[:, :m], np.asarray(lam, dtype=np.float64)[:m], ghat)
    Qp, lp = Qm[:, 1:], lm[1:]                       # Q', Lambda' (null pair removed)
    M, s, n, Ms, B = _seed_blocks(graph, seed_node)
    S = s.size
    Uhat_s = graph.hat_scale()[s][:, None] * one_hot(seed_label, C)
    Qs = Qp[s]                                       # Q'_s
    BQn = B @ Qp                                     # B Q'_n      (S x m')
    BRt = BQn @ (Qs / lp[None, :]).T                 # B R^T = B Q'_n Lambda'^{-1} Q'_s^T   (S x S)
    Bg = B @ ghat                                    # B g_n
    K = np.zeros((S + 1, S + 1))
    K[:S, :S] = np.eye(S) - BRt
    K[:S, S] = -Bg
    K[S, :S] = ghat[s]
    rhs = np.zeros((S + 1, C))
    rhs[:S] = Ms @ Uhat_s
    sol = np.linalg.solve(K, rhs)                   # LU with partial pivoting (LAPACK gesv)
    Fs, c = sol[:S], sol[S]
    Y = (Qs.T @ Fs) / lp[:, None]                    # Lambda'^{-1} Q'_s^T F_s
    return Qp, Y, c


def fast_rw(graph, Q, lam, seed_node, seed_label, C, m=None, rows=None):
    """Label probabilities U (N x C, or len(rows) x C) of the gamma = 0 fast random walker."""
    Qp, Y, c = fast_rw_coeffs(graph, Q, lam, seed_node, seed_label, C, m)
    ghat = graph.ghat()
    hs = graph.hat_scale()
    N = graph.N
    rows = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    Uhat = Qp[rows] @ Y + np.outer(ghat[rows], c)
    with np.errstate(divide="ignore", invalid="ignore"):
        U = np.where(hs[rows, None] > 0, Uhat / hs[rows, None], 0.0)
    # seed rows are fixed (eq. (1)): one-hot
    seed_node = np.asarray(seed_node)
    lab = np.asarray(seed_label)
    pos = {int(v): k for k, v in enumerate(seed_node)}
    for r, i in enumerate(rows):
        k = pos.get(int(i))
        if k is not None:
            U[r] = 0.0
            U[r, lab[k]] = 1.0
    return U


def fast_rw_prior(graph, Q, lam, seed_node, seed_label, C, gamma, prior, m=None):
    """gamma > 0 fast random walker, eqs. (15) and (17) as printed, in the variables of the
    operator graph.M() (with the normalized Laplacian this applies the prior in hat variables,
    P_hat = D^{1/2} P, as the substitution of Sec. II-C prescribes)."""
    m = Q.shape[1] if m is None else m
    Q = np.asarray(Q, dtype=np.float64)[:, :m]
    lam = np.asarray(lam, dtype=np.float64)[:m]
    M, s, n, Ms, B = _seed_blocks(graph, seed_node)
    hs = graph.hat_scale()
    Uhat_s = hs[s][:, None] * one_hot(seed_label, C)
    Phat = hs[:, None] * np.asarray(prior, dtype=np.float64)
    Phat_n = Phat.copy()
    Phat_n[s] = 0.0                                   # P_n, embedded N wide
    inv = 1.0 / (lam + gamma)
    Qs = Q[s]
    # E_n P_n = Q_n (Lambda + gamma)^{-1} Q_n^T P_n
    QnTPn = Q.T @ Phat_n
    EnPn = Q @ (inv[:, None] * QnTPn)                 # evaluated on all rows; only rows n are used
    EnPn[s] = 0.0
    BRt = (B @ Q) @ (Qs * inv[None, :]).T             # B R^T,  R^T = Q_n (Lambda+gamma)^{-1} Q_s^T
    S = s.size
    lhs = np.eye(S) - BRt
    rhs = Ms @ Uhat_s + gamma * (Uhat_s + B @ EnPn)
    Fs = np.linalg.solve(lhs, rhs)
    Uhat = Q @ (inv[:, None] * (Qs.T @ Fs)) + gamma * EnPn   # eq. (15) on the non-seed rows
    with np.errstate(divide="ignore", invalid="ignore"):
        U = np.where(hs[:, None] > 0, Uhat / hs[:, None], 0.0)
    U[s] = one_hot(seed_label, C)
    return U
