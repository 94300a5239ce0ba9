"""Online choice of the number of eigenvectors from the seeds (oracle; test infrastructure only).

Sec. III-A1: for every label k, the fit of the seeds by the first m eigenvectors is

    f(u_s^k) = min_{||alpha|| <= rho} || Q_s alpha - u_s^k ||^2          (eq. (24))

with rho = sqrt(N) (the labels lie in [0, 1], eq. (23)), replaced by sqrt(1^T D 1) under the
normalized Laplacian.  If any f exceeds f_max = S * eps^2 (eps = 1/10 in the paper) more eigenvectors
are added and the test repeated.

Readings:
  * alpha has m entries (the paper's "alpha_k in R^K" is a typo for R^m);
  * under the normalized Laplacian the fitted seed vector is the hat variable D_s^{1/2} u_s^k;
  * "add more eigenvectors and repeat" = the smallest m in [m_min, m_avail] whose worst label
    satisfies max_k f_k(m) <= f_max; the oracle scans m upward one at a time;
  * Q_s holds the seed rows of the stored basis, null vector included.

The constrained least-squares problem (a trust-region subproblem, Golub & Van Loan Sec. 12.1) is
solved through the SVD of Q_s: for the compact SVD A = U S V^T and u = U^T b,
||alpha(mu)||^2 = sum u_i^2 s_i^2 / (s_i^2 + mu)^2; mu = 0 if the minimum-norm least-squares
solution is feasible, otherwise mu > 0 solves ||alpha(mu)|| = rho (bisection), and the residual is
f = ||b_perp||^2 + sum u_i^2 (mu / (s_i^2 + mu))^2.
"""
from __future__ import annotations

import numpy as np


def lsqi(A, b, rho):
    """min ||A alpha - b||^2 subject to ||alpha|| <= rho.  Returns (f, mu, alpha)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    u = U.T @ b
    tol = (s[0] if s.size else 0.0) * max(A.shape) * np.finfo(float).eps
    r = int(np.sum(s > tol))
    b_perp = b - U[:, :r] @ u[:r]
    base = float(b_perp @ b_perp)
    s2 = s[:r] ** 2
    ur = u[:r]

    def norm_alpha_sq(mu):
        return float(np.sum(ur * ur * s2 / (s2 + mu) ** 2))

    if norm_alpha_sq(0.0) <= rho * rho:
        mu = 0.0
    else:
        lo, hi = 0.0, float(np.linalg.norm(A.T @ b)) / rho
        while norm_alpha_sq(hi) > rho * rho:
            hi *= 2.0
        for _ in range(400):
            mid = 0.5 * (lo + hi)
            if norm_alpha_sq(mid) > rho * rho:
                lo = mid
            else:
                hi = mid
            if hi - lo <= 1e-15 * hi:
                break
        mu = hi
    f = base + float(np.sum(ur * ur * (mu / (s2 + mu)) ** 2))
    alpha = Vt[:r].T @ (ur * s[:r] / (s2 + mu))
    return f, mu, alpha


def seed_targets(graph, seed_node, seed_label, C):
    """(B, rho): the S x C matrix of fitted seed vectors and the norm bound."""
    s = np.asarray(seed_node, dtype=np.int64)
    B = np.zeros((s.size, C))
    B[np.arange(s.size), np.asarray(seed_label)] = 1.0
    if graph.normalized:
        d = graph.degree()
        B = np.sqrt(d[s])[:, None] * B
        rho = float(np.sqrt(d.sum()))
    else:
        rho = float(np.sqrt(graph.N))
    return B, rho


def f_values(graph, Q, seed_node, seed_label, C, m):
    """f_k(m) for every label k (eq. (24))."""
    B, rho = seed_targets(graph, seed_node, seed_label, C)
    A = np.asarray(Q, dtype=np.float64)[np.asarray(seed_node, dtype=np.int64), :m]
    return np.array([lsqi(A, B[:, k], rho)[0] for k in range(C)])


def choose_m(graph, Q, seed_node, seed_label, C, eps=0.1, m_min=2, m_avail=None):
    """Smallest m with max_k f_k(m) <= S eps^2; m_avail if none qualifies.
    Returns (m, f_max, f_at_m)."""
    m_avail = Q.shape[1] if m_avail is None else m_avail
    S = len(seed_node)
    fmax = S * eps * eps
    f = None
    for m in range(m_min, m_avail + 1):
        f = f_values(graph, Q, seed_node, seed_label, C, m)
        if f.max() <= fmax:
            return m, fmax, f
    return m_avail, fmax, f
