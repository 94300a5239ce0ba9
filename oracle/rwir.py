"""Random walker with priors and no seeds, at registration label counts (oracle; test infrastructure only).

Registration (Sec. II-A with the seed set empty; Sec. IV-A): every vertex is unseeded, the labels are
displacement vectors, thousands of them, and the walker is driven by the priors alone,

    (L + gamma I) U = gamma P,

the gamma term of eq. (5) with no boundary term.  The fast walker (Sec. II-B, eq. (15) with no seed rows)
replaces the operator by its m stored eigenpairs:

    U_hat = Q (Lambda + gamma I)^{-1} gamma Q^T P_hat,

and the registration result is, at each voxel, the label of largest probability (its displacement).  The
choice of m from the priors (eq. (25), one label in every r^d) is priors.choose_m_prior on the same inputs.

Readings:
  * under the normalized Laplacian the system is taken in hat variables, (L_hat + gamma I) U_hat =
    gamma P_hat with U_hat = D^{1/2} U and P_hat = D^{1/2} P, the substitution of Sec. II-C (as with
    seeds); in the original variables this is (L + gamma D) U = gamma D P.  A vertex of degree 0 gets U = 0;
  * the stored basis is read as with seeds (eigen.insert_null): the analytic null vector takes the place of
    the stored column closest to it, with eigenvalue 0, and the other columns are made orthogonal to it;
  * the label of a voxel is the smallest k among those of largest U_k.
"""
from __future__ import annotations

import numpy as np

from .eigen import insert_null


def rwir_coefficients(graph, Q, lam, prior, gamma, m=None):
    """(Qn, Y): the basis with the null vector inserted (N x m) and Y = gamma (Lambda + gamma I)^{-1} Qn^T
    P_hat (m x C), so that U_hat = Qn Y."""
    m = Q.shape[1] if m is None else m
    Qn, ln = insert_null(np.asarray(Q, dtype=np.float64)[:, :m], np.asarray(lam, dtype=np.float64)[:m],
                         graph.ghat())
    Phat = graph.hat_scale()[:, None] * np.asarray(prior, dtype=np.float64)
    Z = Qn.T @ Phat
    return Qn, (gamma / (ln + gamma))[:, None] * Z


def rwir_probabilities(graph, Q, lam, prior, gamma, m=None, rows=None):
    """U (N x C, or len(rows) x C) of the seedless fast walker: U = D^{-1/2} Qn Y."""
    Qn, Y = rwir_coefficients(graph, Q, lam, prior, gamma, m)
    hs = graph.hat_scale()
    r = np.arange(graph.N) if rows is None else np.asarray(rows, dtype=np.int64)
    Uhat = Qn[r] @ Y
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(hs[r][:, None] > 0, Uhat / hs[r][:, None], 0.0)


def rwir_labels(U):
    """(label, probability) per row: the first index of the row maximum and the maximum."""
    U = np.asarray(U)
    k = np.argmax(U, axis=1)
    return k.astype(np.int32), U[np.arange(U.shape[0]), k]
