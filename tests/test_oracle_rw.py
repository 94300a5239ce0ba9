"""Pins of the oracle's exact and fast random walker: closed forms on path graphs (the random walker
on a path is a series-resistor voltage divider), brute-force dense solves, the maximum principle,
and the identity that the fast random walker with the full eigenbasis equals the exact one."""
import numpy as np
import pytest

import rwsynth
from oracle.eigen import dense_eigpairs
from oracle.exact_rw import exact_rw
from oracle.fast_rw import fast_rw, fast_rw_prior
from oracle.graph import Graph


def test_path_graph_closed_form():
    """Seeds at both ends of a path: u_1(i) = sum_{j<i} 1/w_j / sum_j 1/w_j (Kirchhoff)."""
    n = 11
    J = np.random.default_rng(3).uniform(0, 1, n)
    g = Graph(J, (n, 1, 1), 4, beta=2.5)
    w = g.w                      # edges j -> j+1 in order
    r = np.concatenate([[0.0], np.cumsum(1.0 / w)])
    expect = r / r[-1]
    for method in ("cg", "direct", "dense"):
        U = exact_rw(g, [0, n - 1], [0, 1], 2, method=method, tol=1e-14)
        np.testing.assert_allclose(U[:, 1], expect, atol=1e-13)
        np.testing.assert_allclose(U[:, 0], 1 - expect, atol=1e-13)


def test_exact_rw_properties():
    w = rwsynth.small("t", (9, 8), 8, C=3, seeds_per_label=2, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (9, 8, 1), 8, beta=30.0)
    Ud = exact_rw(g, node, lab, 3, method="dense")
    Uc = exact_rw(g, node, lab, 3, method="cg", tol=1e-13)
    np.testing.assert_allclose(Uc, Ud, atol=1e-11)
    np.testing.assert_allclose(Ud.sum(axis=1), 1.0, atol=1e-13)
    assert Ud.min() >= -1e-13 and Ud.max() <= 1 + 1e-13
    np.testing.assert_array_equal(Ud[node, lab], 1.0)
    # brute force: dense solve of the full (N x N) system with Dirichlet rows replaced
    L = g.L().toarray()
    A = L.copy()
    b = np.zeros((g.N, 3))
    A[node] = 0.0
    A[node, node] = 1.0
    b[node, lab] = 1.0
    np.testing.assert_allclose(np.linalg.solve(A, b), Ud, atol=1e-12)
    # a label without seeds gets probability 0 everywhere
    U4 = exact_rw(g, node, lab, 4, method="dense")
    np.testing.assert_allclose(U4[:, 3], 0.0, atol=0)


@pytest.mark.parametrize("normalized", [True, False])
@pytest.mark.parametrize("conn,dims", [(4, (9, 9, 1)), (8, (7, 6, 1)), (6, (4, 4, 3))])
def test_fast_rw_full_basis_is_exact(normalized, conn, dims):
    """With all N eigenpairs E is the (pseudo-)inverse, eq. (14) is an identity, and the fast random
    walker reproduces eq. (5)."""
    w = rwsynth.small("t", dims, conn, C=3, seeds_per_label=2, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, dims, conn, beta=20.0, normalized=normalized)
    lam, Q = dense_eigpairs(g, g.N)
    Uf = fast_rw(g, Q, lam, node, lab, 3)
    Ue = exact_rw(g, node, lab, 3, method="dense")
    np.testing.assert_allclose(Uf, Ue, atol=1e-10)


def test_fast_rw_truncated_rows_sum_to_one():
    w = rwsynth.small("t", (12, 11), 4, C=3, seeds_per_label=3, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (12, 11, 1), 4, beta=90.0)
    lam, Q = dense_eigpairs(g, 40)
    for m in (2, 5, 17, 40):
        U = fast_rw(g, Q, lam, node, lab, 3, m=m)
        np.testing.assert_allclose(U.sum(axis=1), 1.0, atol=1e-12)
        np.testing.assert_array_equal(U[node, lab], 1.0)
        # row subset gives the same rows
        rows = np.array([0, 7, 50, 131])
        np.testing.assert_allclose(fast_rw(g, Q, lam, node, lab, 3, m=m, rows=rows), U[rows], atol=1e-14)


def test_fast_rw_prior_full_basis():
    """gamma > 0, unnormalized Laplacian: eqs. (15) and (17) with the full basis reproduce eq. (5)."""
    w = rwsynth.small("t", (8, 7), 4, C=2, seeds_per_label=2)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (8, 7, 1), 4, beta=20.0, normalized=False)
    rng = np.random.default_rng(5)
    P = rng.uniform(size=(g.N, 2))
    P /= P.sum(axis=1, keepdims=True)
    w_, V = np.linalg.eigh(g.L().toarray())
    Uf = fast_rw_prior(g, V, w_, node, lab, 2, gamma=0.3, prior=P)
    Ue = exact_rw(g, node, lab, 2, method="dense", gamma=0.3, prior=P)
    np.testing.assert_allclose(Uf, Ue, atol=1e-10)


def test_fast_rw_ignores_null_components_of_stored_basis():
    """Reading of the gamma = 0 case: only the part of each stored eigenvector orthogonal to the null
    vector enters E; adding null-vector components to the stored columns changes nothing."""
    w = rwsynth.small("t", (10, 9), 8, C=2, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (10, 9, 1), 8, beta=90.0)
    lam, Q = dense_eigpairs(g, 12)
    Q2 = Q.copy()
    Q2[:, 1:] += np.outer(g.ghat(), np.linspace(0.01, 0.05, 11))
    Q2[:, 1:] /= np.linalg.norm(Q2[:, 1:], axis=0)
    np.testing.assert_allclose(fast_rw(g, Q2, lam, node, lab, 2), fast_rw(g, Q, lam, node, lab, 2), atol=1e-12)


def test_exact_mode_agrees_and_survives_near_null_eigenvalues():
    """Exact rational evaluation of the bordered system equals the FP64 one on a well-conditioned
    basis, and keeps the rows stochastic where weakly coupled regions give eigenvalues ~1e-13."""
    w = rwsynth.small("t", (12, 11), 4, C=3, seeds_per_label=3, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (12, 11, 1), 4, beta=10.0)          # low contrast: well separated spectrum
    lam, Q = dense_eigpairs(g, 20)
    assert lam[1] > 1e-4
    np.testing.assert_allclose(fast_rw(g, Q, lam, node, lab, 3, exact=True), fast_rw(g, Q, lam, node, lab, 3),
                               atol=1e-13)
    w = rwsynth.small("s1", (23, 19), 4, m=40, C=3, seeds_per_label=4, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, w.dims, 4, beta=90.0)
    lam, Q = dense_eigpairs(g, 10)
    assert lam[1] < 1e-9                              # weakly coupled region
    U = fast_rw(g, Q, lam, node, lab, 3, exact=True)
    np.testing.assert_allclose(U.sum(axis=1), 1.0, atol=1e-13)


def test_decimal_exact_mode_equals_rational_mode():
    """The exact mode's 100-digit decimal evaluation of the bordered system gives the same FP64 results as
    the rational evaluation, on weakly coupled phantoms (second eigenvalue 7e-14 and -1.3e-16, condition
    near 1e15) with FP64 and FP32-rounded bases."""
    cases = [(rwsynth.Workload("b5", 505, (129, 7, 1), 4, 90.0, 8, 3, 5, 0.05, 4, "cycle", 0.0, "f64"), 3),
             (rwsynth.Workload("b1", 501, (64, 48, 1), 4, 90.0, 30, 2, 5, 0.05, 4, "cycle", 0.0, "f64"), 2)]
    for w, per in cases:
        J, rid = rwsynth.phantom(w, 0)
        node, lab = rwsynth.seeds(w, rid, 0, per_label=per, stream_offset=3)
        g = Graph(J, w.dims, w.conn, w.beta)
        lam, Q = dense_eigpairs(g, w.m)
        assert np.min(np.abs(lam[1:])) < 1e-12
        for Qx in (Q, Q.astype(np.float32).astype(np.float64)):
            Ur = fast_rw(g, Qx, lam, node, lab, w.C, exact="rational")
            Ud = fast_rw(g, Qx, lam, node, lab, w.C, exact=True)
            np.testing.assert_allclose(Ud, Ur, rtol=0, atol=1e-15)
