"""Pins of the oracle's checkers and of its online helpers against facts fixed by the mathematics.

* `certify` (residual and orthonormality of a given basis): exact beta = 0 eigenpairs of the grid
  Laplacian from the DCT-II closed form (residual ~ 0), and pairs perturbed by a known amount (a shifted
  eigenvalue, a rotation towards a second eigenvector, a scaled or tilted column).
* `principal_angle_sines`: two spans at a known angle, one span in two bases, and an angle of 1e-9.
* `diag_rq` (Sec. III-B eq. (27)) on an *edited* graph: with the new operator's own eigenvectors it
  returns the new eigenvalues, and over a complete orthonormal basis the quotients sum to the trace of
  the new operator (trace invariance), which differs from the old operator's trace.
* `seed_targets` (Sec. III-A1): the norm bound of eq. (23) is attained by the all-ones labelling, the
  targets are the seed rows of D^{1/2} u from the exact random walker, and with the full eigenbasis the
  exact solution is a feasible alpha, so every fit is 0.
"""
import numpy as np
import pytest

import rwsynth
from oracle.choose_m import f_values, seed_targets
from oracle.eigen import certify, dense_eigpairs, principal_angle_sines
from oracle.exact_rw import exact_rw
from oracle.graph import Graph
from oracle.update import diag_rq


def _path_eig(n, k):
    return 4.0 * np.sin(np.pi * k / (2 * n)) ** 2


def _dct_pair(dims, kx, ky):
    """Unit eigenvector and eigenvalue of L on a beta = 0 free-boundary 4-connected grid:
    cos(pi kx (x + 1/2)/nx) cos(pi ky (y + 1/2)/ny), eigenvalue 4 sin^2(pi kx/2nx) + 4 sin^2(pi ky/2ny)."""
    nx, ny, _ = dims
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v = (np.cos(np.pi * kx * (x + 0.5) / nx) * np.cos(np.pi * ky * (y + 0.5) / ny)).reshape(-1)
    return v / np.linalg.norm(v), _path_eig(nx, kx) + _path_eig(ny, ky)


DIMS = (9, 7, 1)


def _beta0_graph():
    J = np.random.default_rng(3).uniform(size=DIMS[0] * DIMS[1])
    return Graph(J, DIMS, 4, beta=0.0, normalized=False)


def test_certify_exact_pairs_have_zero_residual():
    g = _beta0_graph()
    pairs = [_dct_pair(DIMS, kx, ky) for kx, ky in ((0, 0), (1, 0), (2, 1), (3, 4))]
    Q = np.stack([p[0] for p in pairs], axis=1)
    lam = np.array([p[1] for p in pairs])
    res, orth = certify(g, Q, lam)
    assert res.max() < 1e-13 and orth < 1e-14


def test_certify_known_residuals():
    g = _beta0_graph()
    q1, l1 = _dct_pair(DIMS, 1, 0)
    q2, l2 = _dct_pair(DIMS, 2, 1)
    delta, th = 3.5e-4, 0.3
    mix = np.cos(th) * q1 + np.sin(th) * q2
    Q = np.stack([q1, q2, mix], axis=1)
    lam = np.array([l1 + delta, l2, l1])
    res, _ = certify(g, Q, lam)
    # ||L q1 - (l1 + delta) q1|| = delta;  L(mix) - l1 mix = sin(th) (l2 - l1) q2
    np.testing.assert_allclose(res[0], delta, rtol=1e-9)
    assert res[1] < 1e-13
    np.testing.assert_allclose(res[2], np.sin(th) * abs(l2 - l1), rtol=1e-12)


def test_certify_orthonormality_error():
    g = _beta0_graph()
    q1, l1 = _dct_pair(DIMS, 1, 0)
    q2, l2 = _dct_pair(DIMS, 2, 1)
    eps = 1e-5
    _, orth = certify(g, np.stack([q1, (1 + eps) * q2], axis=1), np.array([l1, l2]))
    np.testing.assert_allclose(orth, (1 + eps) ** 2 - 1, rtol=1e-8)
    th = 0.2
    _, orth = certify(g, np.stack([q1, np.cos(th) * q1 + np.sin(th) * q2], axis=1), np.array([l1, l1]))
    np.testing.assert_allclose(orth, np.cos(th), rtol=1e-12)


def test_principal_angles_known():
    rng = np.random.default_rng(5)
    B, _ = np.linalg.qr(rng.standard_normal((40, 6)))     # orthonormal e1..e6 in R^40
    for th in (0.7, 1e-3, 1e-9):
        Q1 = B[:, [0, 1, 2]]
        Q2 = np.stack([B[:, 0], np.cos(th) * B[:, 1] + np.sin(th) * B[:, 3],
                       np.cos(2 * th) * B[:, 2] + np.sin(2 * th) * B[:, 4]], axis=1)
        s = np.sort(principal_angle_sines(Q1, Q2))
        np.testing.assert_allclose(s, np.sort([0.0, np.sin(th), np.sin(2 * th)]), rtol=1e-6, atol=1e-15)
        np.testing.assert_allclose(np.sort(principal_angle_sines(Q2, Q1)), s, rtol=1e-6, atol=1e-15)


def test_principal_angles_same_span_other_basis():
    rng = np.random.default_rng(6)
    Q1, _ = np.linalg.qr(rng.standard_normal((50, 5)))
    O, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    s = principal_angle_sines(Q1, Q1 @ O)
    assert s.shape == (5,) and s.max() < 1e-14
    # orthogonal spans: every sine is 1
    Q2, _ = np.linalg.qr(rng.standard_normal((50, 3)) - Q1 @ (Q1.T @ rng.standard_normal((50, 3))))
    Q2 = Q2 - Q1 @ (Q1.T @ Q2)
    Q2, _ = np.linalg.qr(Q2)
    np.testing.assert_allclose(principal_angle_sines(Q1, Q2), 1.0, atol=1e-14)


def _edited_pair(normalized):
    w = rwsynth.small("pin", (8, 7), 4, n_shapes=3)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (8, 7, 1), 4, beta=90.0, normalized=normalized)
    g2 = g.copy()
    g2.set_beta(150.0)
    g2.scale_box((1, 1, 0), (4, 4, 1), 0.1)
    # isolate node 5 * 8 + 5: remove its four edges (it keeps d = 0 afterwards)
    node = 5 * 8 + 5
    ids = g2.edge_id[((g2.tail == node) | (g2.head == node)) & g2.present]
    g2.remove_edges(ids)
    return g, g2


@pytest.mark.parametrize("normalized", [True, False])
def test_diag_rq_uses_the_edited_operator(normalized):
    g, g2 = _edited_pair(normalized)
    # the new operator's own eigenvectors (null vector first) are returned with its eigenvalues
    lam_new, Q_new = dense_eigpairs(g2, g2.N)
    Qo, lam = diag_rq(g2, Q_new)
    np.testing.assert_allclose(lam, lam_new, atol=1e-12)
    # trace invariance over a complete orthonormal basis (the old operator's eigenvectors): the
    # quotients sum to tr(M_new) = number of nodes with d > 0 (L_hat) or sum of d (L)
    _, Q_old = dense_eigpairs(g, g.N)
    _, lam = diag_rq(g2, Q_old)
    d2, d1 = g2.degree(), g.degree()
    tr_new = float(np.sum(d2 > 0)) if normalized else float(d2.sum())
    tr_old = float(np.sum(d1 > 0)) if normalized else float(d1.sum())
    assert abs(tr_new - tr_old) > 0.5          # the pin tells the two operators apart
    np.testing.assert_allclose(lam.sum(), tr_new, rtol=1e-12)


@pytest.mark.parametrize("normalized", [True, False])
def test_seed_targets_norm_bound_attained_by_all_ones(normalized):
    w = rwsynth.small("pin", (9, 8), 8, n_shapes=3)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (9, 8, 1), 8, beta=90.0, normalized=normalized)
    nodes = np.arange(g.N)
    B, rho = seed_targets(g, nodes, np.zeros(g.N, dtype=np.int32), 1)
    # u = 1 everywhere has every component at its bound, so ||D^{1/2} 1|| (or ||1||) equals rho
    np.testing.assert_allclose(np.linalg.norm(B[:, 0]), rho, rtol=1e-14)
    np.testing.assert_allclose(rho ** 2, g.degree().sum() if normalized else g.N, rtol=1e-14)


@pytest.mark.parametrize("normalized", [True, False])
def test_seed_targets_are_seed_rows_of_exact_solution(normalized):
    dims = (9, 8, 1)
    w = rwsynth.small("pin", dims, 4, C=3, seeds_per_label=3, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, dims, 4, beta=90.0, normalized=normalized)
    U = exact_rw(g, node, lab, 3, method="direct")          # N x C
    Uhat = g.hat_scale()[:, None] * U                        # the fitted variable
    B, rho = seed_targets(g, node, lab, 3)
    np.testing.assert_allclose(B, Uhat[node], rtol=1e-14, atol=0)
    assert np.all(np.linalg.norm(Uhat, axis=0) <= rho * (1 + 1e-12))
    # with the full eigenbasis, alpha = Q^T u_hat reproduces the seeds within the bound: f = 0
    lam, Q = dense_eigpairs(g, g.N)
    alpha = Q.T @ Uhat
    assert np.all(np.linalg.norm(alpha, axis=0) <= rho * (1 + 1e-12))
    np.testing.assert_allclose(Q[node] @ alpha, B, atol=1e-9)
    assert f_values(g, Q, node, lab, 3, g.N).max() < 1e-16
