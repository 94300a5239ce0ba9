"""Prior probabilities and the prior-based choice of the number of eigenvectors (oracle; test
infrastructure only).

Priors (Sec. IV-A): for segmentation the prior probabilities are computed by fitting a Gaussian to the
intensities of each label's seeds; the prior of label k at voxel i is that Gaussian's density at J_i,
normalized to sum to 1 over the labels at each voxel.

Choice of m from the priors (Sec. III-A2, eq. (25)): g(p^k) = || p^k - Q Q^T p^k ||^2 measures how
well the columns of Q represent prior k.  It is evaluated for one label in every r^d, uniformly spaced
(d the image dimension, r = 4 in the paper), and eigenvectors are added while any of them exceeds
g_max = n eps^2 (eps = 1/10 in the paper).  The paper keeps the residual p^k - Q Q^T p^k so that adding
eigenvectors only projects it onto the new ones; here g is evaluated from its definition for each m.

Readings:
  * the Gaussian fit takes the mean and the maximum-likelihood (population) variance of the seed
    intensities of label k, floored at VAR_FLOOR (a label with a single seed, or with equal seed
    intensities, has zero variance); a label without seeds has prior 0 everywhere and takes no part
    in the normalization;
  * the normalization is carried out on the log-densities (a softmax), which is the normalized density
    without the underflow of exp far from every mean;
  * sampled labels: k = 0, r^d, 2 r^d, ... below C;
  * under the normalized Laplacian the columns of Q are eigenvectors of L_hat and the prior enters the
    method as p_hat = D^{1/2} p (Sec. II-C), so g is evaluated on p_hat and g_max = eps^2 1^T D 1 (the
    D-weighted form of n eps^2, as rho of eq. (24) is sqrt(1^T D 1)); with L, g on p and g_max = N eps^2;
  * "add eigenvectors while any g exceeds g_max" = the smallest m in [m_min, m_avail] whose sampled
    labels all satisfy g_k(m) <= g_max, m_avail when none does.
"""
from __future__ import annotations

import numpy as np

VAR_FLOOR = 1e-6


def gaussian_fit(J, seed_node, seed_label, C):
    """(mu, var, present): per-label mean and floored ML variance of the seed intensities."""
    J = np.asarray(J, dtype=np.float64)
    s = np.asarray(seed_node, dtype=np.int64)
    lab = np.asarray(seed_label)
    mu = np.zeros(C)
    var = np.full(C, VAR_FLOOR)
    present = np.zeros(C, dtype=bool)
    for k in range(C):
        v = J[s[lab == k]]
        if v.size == 0:
            continue
        present[k] = True
        mu[k] = v.mean()
        var[k] = max(float(np.mean((v - mu[k]) ** 2)), VAR_FLOOR)
    return mu, var, present


def gaussian_priors(J, seed_node, seed_label, C):
    """N x C prior probabilities from the per-label Gaussian fits (Sec. IV-A)."""
    J = np.asarray(J, dtype=np.float64)
    mu, var, present = gaussian_fit(J, seed_node, seed_label, C)
    logd = np.full((J.size, C), -np.inf)
    for k in range(C):
        if present[k]:
            logd[:, k] = -0.5 * (J - mu[k]) ** 2 / var[k] - 0.5 * np.log(2.0 * np.pi * var[k])
    top = logd.max(axis=1, keepdims=True)
    e = np.exp(logd - top)
    return e / e.sum(axis=1, keepdims=True)


def sampled_labels(C, r, d):
    """One label in every r^d: 0, r^d, 2 r^d, ... below C."""
    return np.arange(0, C, r ** d)


def prior_targets(graph, prior):
    """(P_used, g_max factor): p_hat = D^{1/2} p and 1^T D 1 (normalized), or p and N."""
    P = np.asarray(prior, dtype=np.float64)
    if graph.normalized:
        d = graph.degree()
        return np.sqrt(d)[:, None] * P, float(d.sum())
    return P, float(graph.N)


def g_values(graph, Q, prior, labels, m):
    """g_k(m) = || p_k - Q_m Q_m^T p_k ||^2 (eq. (25)) for the given labels, Q_m the first m columns."""
    P, _ = prior_targets(graph, prior)
    Qm = np.asarray(Q, dtype=np.float64)[:, :m]
    out = []
    for k in labels:
        p = P[:, k]
        r = p - Qm @ (Qm.T @ p)
        out.append(float(r @ r))
    return np.array(out)


def choose_m_prior(graph, Q, prior, eps=0.1, r=4, m_min=2, m_avail=None):
    """Smallest m in [m_min, m_avail] with g_k(m) <= g_max for every sampled label; m_avail if none.
    Returns (m, g_max, g at m for the sampled labels)."""
    m_avail = Q.shape[1] if m_avail is None else m_avail
    C = np.asarray(prior).shape[1]
    labels = sampled_labels(C, r, graph.ndim)
    _, scale = prior_targets(graph, prior)
    gmax = eps * eps * scale
    g = None
    for m in range(m_min, m_avail + 1):
        g = g_values(graph, Q, prior, labels, m)
        if g.max() <= gmax:
            return m, gmax, g
    return m_avail, gmax, g
