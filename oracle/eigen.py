"""The m smallest eigenpairs of the (normalized) Laplacian (oracle; test infrastructure only).

Sec. II-B eq. (6): L = Q Lambda Q^T with eigenvalues in increasing order; only the m smallest are
kept (paragraph after eq. (9)).  The Laplacian is positive semi-definite with one zero eigenvalue
whose eigenvector is the normalized constant vector g (paragraph after eq. (6)); under the
normalized Laplacian of Sec. II-C the null vector is D^{1/2} 1 / ||D^{1/2} 1||.

Readings:
  * m counts the null pair.  The computed lambda ~ 0 vector is replaced by the analytic null vector,
    and the other columns are made orthogonal to it (Gram-Schmidt against it, then renormalized).
  * stored sign of each eigenvector: its entry of largest magnitude is positive (lowest index on a
    tie).

For small graphs the pairs come from a dense symmetric eigendecomposition (numpy.linalg.eigh).  For
any size, `certify` returns the residuals ||M q_i - lambda_i q_i|| and ||Q^T Q - I|| of a given basis,
and `principal_angle_sines` compares two spans.
"""
from __future__ import annotations

import numpy as np


def fix_signs(Q):
    Q = Q.copy()
    for j in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, j])))
        if Q[i, j] < 0:
            Q[:, j] = -Q[:, j]
    return Q


def insert_null(Q, lam, ghat):
    """Drop the column closest to the null vector, put ghat first with eigenvalue 0, and project
    ghat out of the remaining columns (Gram-Schmidt against ghat), renormalizing them."""
    Q = np.asarray(Q, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    k = int(np.argmax(np.abs(ghat @ Q)))
    keep = [j for j in range(Q.shape[1]) if j != k]
    rest = Q[:, keep]
    rest = rest - np.outer(ghat, ghat @ rest)
    rest = rest / np.linalg.norm(rest, axis=0)
    Qn = np.concatenate([ghat[:, None], rest], axis=1)
    ln = np.concatenate([[0.0], lam[keep]])
    return Qn, ln


def dense_eigpairs(graph, m):
    """(lam, Q): the m smallest eigenpairs of graph.M() by dense eigh, null vector inserted."""
    M = graph.M().toarray()
    w, V = np.linalg.eigh(M)
    Q, lam = insert_null(V[:, :m], w[:m], graph.ghat())
    return lam, fix_signs(Q)


def full_spectrum(graph):
    return np.linalg.eigh(graph.M().toarray())[0]


def certify(graph, Q, lam):
    """Per-column residual norms ||M q_i - lam_i q_i|| and the orthonormality error ||Q^T Q - I||_max."""
    M = graph.M()
    Q = np.asarray(Q, dtype=np.float64)
    R = M @ Q - Q * np.asarray(lam)[None, :]
    G = Q.T @ Q - np.eye(Q.shape[1])
    return np.linalg.norm(R, axis=0), float(np.abs(G).max())


def rayleigh_quotients(graph, Q):
    M = graph.M()
    Q = np.asarray(Q, dtype=np.float64)
    return np.einsum("ij,ij->j", Q, M @ Q) / np.einsum("ij,ij->j", Q, Q)


def principal_angle_sines(Q1, Q2):
    """Sines of the min(k1, k2) principal angles between span(Q1) and span(Q2) (orthonormal columns):
    the singular values of the part of the narrower basis outside the span of the wider one,
    (I - Q1 Q1^T) Q2 with Q2 the narrower (Bjorck & Golub 1973).  Unlike sqrt(1 - cos^2) this keeps its
    accuracy for small angles."""
    Q1 = np.asarray(Q1, dtype=np.float64)
    Q2 = np.asarray(Q2, dtype=np.float64)
    if Q2.shape[1] > Q1.shape[1]:
        Q1, Q2 = Q2, Q1
    R = Q2 - Q1 @ (Q1.T @ Q2)
    s = np.linalg.svd(R, compute_uv=False)
    return np.clip(s, 0.0, 1.0)
