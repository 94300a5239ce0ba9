"""Updating the precomputed eigenbasis after the Laplacian changes (oracle; test infrastructure only).

Sec. III-B: when beta (or any edge weight) changes online, the new normalized Laplacian is built,
the Rayleigh quotient / relaxed Ncut value (eq. (26)) of every stored eigenvector is evaluated on it,
lambda_hat_i = q_i^T L_hat q_i (eq. (27)), and E is approximated by Q (Lambda_hat + gamma I)^{-1} Q^T
with Q unchanged (eq. (28)).

Readings:
  * lambda_hat uses the new (online) Laplacian, the formula of eq. (27).
  * Under the normalized Laplacian the null vector D^{1/2} 1 / ||.|| moves with D, so the new null
    vector replaces the stored one and the remaining columns are re-orthonormalized by Gram-Schmidt
    in their stored order (the process the paper uses after eq. (33)) before the quotients.
  * Rayleigh-Ritz (beyond the paper's diagonal update): the same basis, then the eigenpairs of the
    projected matrix H = Q'^T L_hat Q' rotate it.
  * Bank of bases for several beta (the end of Sec. III-B: eigenvectors precomputed for several beta and
    eq. (26) used to "interpolate" between them): for the requested operator, every bank basis gets its
    diagonal update, and the basis whose quotients sum lowest is used with its lambda_hat.  Among
    orthonormal bases of m columns the sum of the Rayleigh quotients is smallest for the eigenbasis of the
    m smallest eigenvalues (Ky Fan), so the sum ranks the bases by how well they span the new low
    spectrum.
"""
from __future__ import annotations

import numpy as np

from .eigen import fix_signs


def gram_schmidt_after(ghat, Q):
    """[ghat, GS(Q[:,1:]) against ghat and each other in order] (modified Gram-Schmidt, FP64)."""
    Q = np.asarray(Q, dtype=np.float64)
    out = np.zeros_like(Q)
    out[:, 0] = ghat
    for j in range(1, Q.shape[1]):
        v = Q[:, j].copy()
        for i in range(j):
            v -= out[:, i] * (out[:, i] @ v)
        out[:, j] = v / np.linalg.norm(v)
    return out


def diag_rq(graph_new, Q):
    """Paper's update: (Q_new, lambda_hat) with lambda_hat_i = q_i^T L_hat_new q_i."""
    Qn = gram_schmidt_after(graph_new.ghat(), Q)
    M = graph_new.M()
    lam = np.einsum("ij,ij->j", Qn, M @ Qn)
    lam[0] = 0.0
    return Qn, lam


def rayleigh_ritz(graph_new, Q):
    """Rayleigh-Ritz on span([ghat_new, Q[:,1:]]): (Q_new, lambda) sorted increasing."""
    Qn = gram_schmidt_after(graph_new.ghat(), Q)
    Qp = Qn[:, 1:]
    H = Qp.T @ (graph_new.M() @ Qp)
    H = 0.5 * (H + H.T)
    th, V = np.linalg.eigh(H)
    out = np.concatenate([Qn[:, :1], Qp @ V], axis=1)
    return fix_signs(out), np.concatenate([[0.0], th])


def bank_select(graph_new, bank):
    """Choose among the bases of a bank (a list of N x m arrays) for the operator of graph_new:
    (index, Q_new, lambda_hat, traces) with traces[b] = sum of the diagonal quotients of basis b."""
    best = None
    traces = []
    for b, Q in enumerate(bank):
        Qn, lam = diag_rq(graph_new, Q)
        t = float(lam.sum())
        traces.append(t)
        if best is None or t < best[3]:
            best = (b, Qn, lam, t)
    return best[0], best[1], best[2], np.array(traces)
