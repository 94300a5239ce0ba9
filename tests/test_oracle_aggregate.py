"""Pins of the oracle's vertex aggregation (Sec. III-C): the aggregated graph is the Galerkin product P^T L P,
Delta, eq. (33) and the propagation against dense brute force over eta and eta_bar, the transferred basis
orthonormal with the aggregated null vector first."""
import numpy as np
import pytest
import scipy.sparse as sp

import rwsynth
from oracle.aggregate import (aggregate_basis, aggregate_graph, blocks, coarse_seeds, delta, prolong,
                              transfer_basis)
from oracle.eigen import dense_eigpairs
from oracle.graph import Graph

CASES = [((9, 7, 1), 4, 2), ((10, 8, 1), 8, 3), ((7, 5, 4), 6, 2), ((11, 9, 1), 8, 2)]


def _graph(dims, conn):
    w = rwsynth.small("ta", dims, conn, C=2, seeds_per_label=2, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    return Graph(J, dims, conn, beta=25.0), J, rid, w


def _eta(g, s):
    b, cdims = blocks(g.dims, s)
    Nc = cdims[0] * cdims[1] * cdims[2]
    eta = np.zeros((g.N, Nc))
    eta[np.arange(g.N), b] = 1.0
    eta_bar = eta / eta.sum(axis=0, keepdims=True)
    return eta, eta_bar


@pytest.mark.parametrize("dims,conn,s", CASES)
def test_aggregated_laplacian_is_the_galerkin_product(dims, conn, s):
    g, _, _, _ = _graph(dims, conn)
    c = aggregate_graph(g, s)
    eta, _ = _eta(g, s)
    P = sp.csr_matrix(eta)
    np.testing.assert_allclose(c.L().toarray(), (P.T @ g.L() @ P).toarray(), atol=1e-12)


@pytest.mark.parametrize("dims,conn,s", CASES)
def test_delta_and_eq33_by_brute_force(dims, conn, s):
    g, _, _, _ = _graph(dims, conn)
    eta, eta_bar = _eta(g, s)
    adj = np.zeros((g.N, g.N), dtype=bool)
    adj[g.tail[g.present], g.head[g.present]] = True
    adj |= adj.T
    ref = np.array([sum(np.abs(eta[x] - eta[xp]).sum() for xp in np.flatnonzero(adj[x])) for x in range(g.N)])
    np.testing.assert_allclose(delta(g, s), ref)
    Q = np.random.default_rng(2).standard_normal((g.N, 5))
    np.testing.assert_allclose(aggregate_basis(g, Q, s), eta_bar.T @ (ref[:, None] * Q), atol=1e-12)
    Ub = np.random.default_rng(3).uniform(size=(eta.shape[1], 3))
    np.testing.assert_allclose(prolong(g, s, Ub), eta @ Ub)


@pytest.mark.parametrize("dims,conn,s", CASES[:2])
def test_transfer_is_orthonormal_with_the_aggregated_null_vector(dims, conn, s):
    g, _, _, _ = _graph(dims, conn)
    lam, Q = dense_eigpairs(g, 12)
    c, Qn, lb = transfer_basis(g, Q, s)
    np.testing.assert_allclose(Qn.T @ Qn, np.eye(12), atol=1e-12)
    np.testing.assert_allclose(np.abs(Qn[:, 0]), np.abs(c.ghat()), atol=1e-14)
    np.testing.assert_allclose(lb[1:], np.einsum("ij,ij->j", Qn, c.M() @ Qn)[1:], rtol=1e-12)
    assert lb[0] == 0.0 and np.all(lb[1:] > 0)


def test_coarse_seeds_merge_and_conflict():
    g, _, _, _ = _graph((9, 7, 1), 4)
    ys, ls = coarse_seeds(g, 3, [0, 1, 30], [1, 1, 0])          # 0 and 1 share block 0
    assert list(ys) == [0, 4] and list(ls) == [1, 0]
    with pytest.raises(ValueError):
        coarse_seeds(g, 3, [0, 1], [0, 1])
