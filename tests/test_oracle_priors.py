"""Pins of the oracle's priors (Sec. IV-A Gaussian fit), the prior-based choice of m (Sec. III-A2,
eq. (25)) and the gamma > 0 fast random walker under the normalized Laplacian (Sec. II-C)."""
import numpy as np
import pytest
import scipy.stats

import rwsynth
from oracle.eigen import dense_eigpairs
from oracle.exact_rw import exact_rw, one_hot, seed_split
from oracle.fast_rw import fast_rw_prior
from oracle.graph import Graph
from oracle.priors import (VAR_FLOOR, choose_m_prior, g_values, gaussian_fit, gaussian_priors, prior_targets,
                           sampled_labels)


def test_gaussian_fit_by_hand():
    J = np.array([0.2, 0.4, 0.8, 0.5, 0.1])
    mu, var, present = gaussian_fit(J, [0, 1, 2], [0, 0, 1], 3)
    np.testing.assert_allclose(mu[:2], [0.3, 0.8], rtol=1e-15)
    np.testing.assert_allclose(var[:2], [0.01, VAR_FLOOR], rtol=1e-12)     # one seed: the floor
    assert list(present) == [True, True, False]


def test_gaussian_priors_against_scipy_densities():
    rng = np.random.default_rng(3)
    J = rng.uniform(0, 1, 500)
    seeds = np.array([3, 17, 40, 41, 99, 120, 200, 333])
    labels = np.array([0, 0, 1, 1, 1, 2, 2, 0])
    mu, var, _ = gaussian_fit(J, seeds, labels, 4)
    P = gaussian_priors(J, seeds, labels, 4)
    dens = np.stack([scipy.stats.norm.pdf(J, loc=mu[k], scale=np.sqrt(var[k])) for k in range(3)], axis=1)
    ref = dens / dens.sum(axis=1, keepdims=True)
    ok = dens.sum(axis=1) > 1e-250                      # where the densities do not underflow
    np.testing.assert_allclose(P[ok, :3], ref[ok], rtol=1e-12, atol=1e-300)
    np.testing.assert_array_equal(P[:, 3], 0.0)          # label 3 has no seeds
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=1e-14)
    assert np.all(P >= 0.0) and np.all(P <= 1.0)


def test_equal_variance_log_odds_are_linear():
    """With two labels of equal variance s^2: log(p0 / p1) = ((J - mu1)^2 - (J - mu0)^2) / (2 s^2)."""
    J = np.linspace(0.0, 1.0, 41)
    seeds, labels = np.array([0, 2, 38, 40]), np.array([0, 0, 1, 1])     # both fits: variance 0.025^2
    P = gaussian_priors(J, seeds, labels, 2)
    mu0, mu1, s2 = 0.025, 0.975, 0.025 ** 2
    expect = ((J - mu1) ** 2 - (J - mu0) ** 2) / (2 * s2)
    mid = np.abs(expect) < 600
    np.testing.assert_allclose(np.log(P[mid, 0]) - np.log(P[mid, 1]), expect[mid], rtol=1e-10, atol=1e-9)


def test_sampled_labels():
    assert list(sampled_labels(40, 4, 2)) == [0, 16, 32]
    assert list(sampled_labels(64, 4, 3)) == [0]
    assert list(sampled_labels(3, 1, 2)) == [0, 1, 2]


@pytest.mark.parametrize("normalized", [True, False])
def test_g_values_span_and_parseval(normalized):
    w = rwsynth.small("tp", (9, 8), 4, C=3, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    g = Graph(J, (9, 8, 1), 4, beta=30.0, normalized=normalized)
    lam, Q = dense_eigpairs(g, g.N)
    N = g.N
    rng = np.random.default_rng(1)
    # priors whose used form (p_hat under L_hat) lies in the span of the first 5 columns, and random ones
    a = rng.standard_normal((5, 2))
    used = Q[:, :5] @ a
    scale = np.sqrt(g.degree()) if normalized else np.ones(N)
    P = np.concatenate([used / scale[:, None], rng.uniform(0, 1, (N, 1))], axis=1)
    Pu, fac = prior_targets(g, P)
    np.testing.assert_allclose(Pu[:, :2], used, rtol=1e-12)
    assert fac == (g.degree().sum() if normalized else N)
    prev = None
    for m in range(1, N + 1, 7):
        gv = g_values(g, Q, P, [0, 1, 2], m)
        parseval = (Pu * Pu).sum(axis=0) - ((Q[:, :m].T @ Pu) ** 2).sum(axis=0)
        np.testing.assert_allclose(gv, parseval, atol=1e-9 * (Pu * Pu).sum())
        if m >= 5:
            assert gv[0] < 1e-20 * fac and gv[1] < 1e-20 * fac
        else:
            assert gv[0] > 1e-6 and gv[1] > 1e-6
        if prev is not None:
            assert np.all(gv <= prev + 1e-12)
        prev = gv
    assert g_values(g, Q, P, [2], N)[0] < 1e-20 * fac          # the full basis represents anything


def test_choose_m_prior_is_minimal():
    w = rwsynth.small("tq", (10, 9), 4, C=2, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    g = Graph(J, (10, 9, 1), 4, beta=30.0)
    lam, Q = dense_eigpairs(g, g.N)
    node, lab = rwsynth.seeds(w, rid)
    P = gaussian_priors(J, node, lab, 2)
    for eps in (0.3, 0.1, 0.03):
        m, gmax, gm = choose_m_prior(g, Q, P, eps=eps, r=4, m_avail=60)
        assert gmax == pytest.approx(eps * eps * g.degree().sum())
        assert gm.max() <= gmax or m == 60
        if m > 2:
            assert g_values(g, Q, P, [0], m - 1).max() > gmax


def test_fast_rw_prior_full_basis_normalized_is_the_degree_weighted_system():
    """gamma > 0 under L_hat (Sec. II-C substitution U_hat = D^{1/2} U, P_hat = D^{1/2} P): with the full
    basis eqs. (15) and (17) solve (L_n + gamma D_n) U_n = gamma D_n P_n - B^T U_s, by brute force."""
    w = rwsynth.small("tr", (8, 7), 8, C=3, seeds_per_label=2, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (8, 7, 1), 8, beta=20.0)
    lam, Q = dense_eigpairs(g, g.N)
    P = gaussian_priors(J, node, lab, 3)
    gamma = 0.05
    U = fast_rw_prior(g, Q, lam, node, lab, 3, gamma=gamma, prior=P)
    L = g.L().toarray()
    d = g.degree()
    s, n = seed_split(g.N, node)
    A = L[np.ix_(n, n)] + gamma * np.diag(d[n])
    rhs = gamma * d[n][:, None] * P[n] - L[np.ix_(n, s)] @ one_hot(lab, 3)
    Ue = np.zeros_like(U)
    Ue[s] = one_hot(lab, 3)
    Ue[n] = np.linalg.solve(A, rhs)
    np.testing.assert_allclose(U, Ue, atol=1e-10)
    np.testing.assert_allclose(U.sum(axis=1), 1.0, atol=1e-10)
    # and it is not the identity-weighted system of eq. (5) when the degrees are not all equal
    Ui = exact_rw(g, node, lab, 3, method="dense", gamma=gamma, prior=P)
    assert np.abs(Ui - U).max() > 1e-3


def test_fast_rw_prior_reads_the_basis_around_the_exact_null_vector():
    """The stored basis is read as in the gamma = 0 case: a perturbed stored null vector and null-vector
    components in the other columns change nothing."""
    w = rwsynth.small("ts", (9, 8), 4, C=2, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (9, 8, 1), 4, beta=30.0)
    lam, Q = dense_eigpairs(g, 20)
    P = gaussian_priors(J, node, lab, 2)
    U = fast_rw_prior(g, Q, lam, node, lab, 2, gamma=0.1, prior=P)
    rng = np.random.default_rng(4)
    Qm = Q.copy()
    Qm[:, 0] += 1e-3 * rng.standard_normal(g.N)
    Qm[:, 1:] += np.outer(g.ghat(), rng.uniform(-0.5, 0.5, 19))     # the stored null vector stays the closest
    np.testing.assert_allclose(fast_rw_prior(g, Qm, lam, node, lab, 2, gamma=0.1, prior=P), U, atol=1e-12)
