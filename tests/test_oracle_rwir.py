"""Pins of the oracle's seedless walker with priors at registration label counts (Sec. II-A eq. (5) with
no seeds, Sec. II-B eq. (15) in the eigenbasis, Sec. II-C hat variables), and of the displacement-label
prior generator."""
import numpy as np
import pytest
import torch

import rwsynth
from oracle.eigen import dense_eigpairs
from oracle.exact_rw import exact_rw
from oracle.graph import Graph
from oracle.rwir import rwir_coefficients, rwir_labels, rwir_probabilities

CASES = [((7, 6), 4), ((6, 5), 8), ((4, 4, 3), 6)]


def _case(dims, conn, normalized=True, C=6, seed=0):
    w = rwsynth.small("rwir", dims, conn, C=C, n_shapes=2)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, w.dims, w.conn, w.beta, normalized=normalized)
    rng = np.random.default_rng(seed)
    P = rng.dirichlet(np.full(C, 0.7), size=g.N)
    return g, P


@pytest.mark.parametrize("normalized", [True, False])
@pytest.mark.parametrize("dims,conn", CASES)
@pytest.mark.parametrize("gamma", [0.3, 1.0])
def test_full_basis_equals_the_direct_solve(dims, conn, normalized, gamma):
    """With every eigenpair the eigenbasis solve is exact: (L + gamma D) U = gamma D P under L_hat, and
    (L + gamma I) U = gamma P under L, solved densely from the Laplacian and the degrees."""
    g, P = _case(dims, conn, normalized)
    lam, Q = dense_eigpairs(g, g.N)
    U = rwir_probabilities(g, Q, lam, P, gamma)
    L = g.L().toarray()
    W = np.diag(g.degree()) if normalized else np.eye(g.N)
    ref = np.linalg.solve(L + gamma * W, gamma * W @ P)
    np.testing.assert_allclose(U, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dims,conn", CASES)
def test_without_seeds_matches_the_exact_walker(dims, conn):
    """Under L the full-basis solve equals the basic walker of eq. (5) with an empty seed set (sparse
    solve of (L + gamma I) U = gamma P)."""
    g, P = _case(dims, conn, normalized=False)
    lam, Q = dense_eigpairs(g, g.N)
    U = rwir_probabilities(g, Q, lam, P, 0.5)
    ref = exact_rw(g, np.zeros(0, np.int64), np.zeros(0, np.int32), P.shape[1], method="direct", gamma=0.5,
                   prior=P)
    np.testing.assert_allclose(U, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("normalized", [True, False])
def test_null_vector_alone_gives_the_weighted_mean(normalized):
    """m = 1 keeps only the null pair: every voxel gets sum_x d_x p_x / sum_x d_x (L_hat) or the plain mean
    of the priors (L)."""
    g, P = _case((7, 6), 4, normalized)
    lam, Q = dense_eigpairs(g, 5)
    U = rwir_probabilities(g, Q, lam, P, 0.8, m=1)
    wts = g.degree() if normalized else np.ones(g.N)
    ref = (wts @ P) / wts.sum()
    np.testing.assert_allclose(U, np.broadcast_to(ref, U.shape), rtol=1e-12)


@pytest.mark.parametrize("normalized", [True, False])
@pytest.mark.parametrize("m", [2, 5, 11])
def test_rows_sum_to_one_at_any_m(normalized, m):
    """Priors summing to 1 over the labels give probabilities summing to 1 at every voxel for any m: their
    sum lies along the null vector, which the basis holds exactly."""
    g, P = _case((4, 4, 3), 6, normalized)
    lam, Q = dense_eigpairs(g, 12)
    U = rwir_probabilities(g, Q, lam, P, 1.0, m=m)
    np.testing.assert_allclose(U.sum(axis=1), 1.0, rtol=1e-12)


def test_large_gamma_returns_the_priors():
    g, P = _case((6, 5), 8)
    lam, Q = dense_eigpairs(g, g.N)
    np.testing.assert_allclose(rwir_probabilities(g, Q, lam, P, 1e9), P, rtol=1e-7, atol=1e-9)


def test_rows_and_coefficients_agree_with_the_full_map():
    g, P = _case((7, 6), 4)
    lam, Q = dense_eigpairs(g, 9)
    U = rwir_probabilities(g, Q, lam, P, 1.0)
    rows = np.array([0, 5, 17, 41])
    np.testing.assert_array_equal(rwir_probabilities(g, Q, lam, P, 1.0, rows=rows), U[rows])
    Qn, Y = rwir_coefficients(g, Q, lam, P, 1.0)
    np.testing.assert_allclose(Qn @ Y, np.sqrt(g.degree())[:, None] * U, rtol=1e-13, atol=1e-15)


def test_labels_take_the_first_of_equal_maxima():
    k, p = rwir_labels(np.array([[0.2, 0.5, 0.5], [0.9, 0.05, 0.05], [0.1, 0.1, 0.8]]))
    assert list(k) == [1, 0, 2]
    np.testing.assert_array_equal(p, [0.5, 0.9, 0.8])


def test_displacement_priors():
    lab = rwsynth.displacement_labels((5, 5, 3))
    assert lab.shape == (75, 3) and lab[0].tolist() == [-2, -2, -1] and lab[7].tolist() == [0, -1, -1]
    f = rwsynth.displacement_field((12, 10, 8), (5, 5, 3), 6)
    P = rwsynth.displacement_priors(f, lab, 0.7)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=1e-14)
    # each voxel's largest prior sits at the label nearest its displacement
    near = np.argmin(((f[:, None, :] - lab[None]) ** 2).sum(axis=2), axis=1)
    np.testing.assert_array_equal(P.argmax(axis=1), near)
    Pt = rwsynth.displacement_priors_torch(torch.as_tensor(f), torch.as_tensor(lab), 0.7, chunk=100)
    np.testing.assert_allclose(Pt.numpy().T, P, rtol=2e-5, atol=1e-7)
