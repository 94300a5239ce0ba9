"""Pins of the oracle's online parts: the constrained least-squares fit that chooses m (KKT
conditions, an independent constrained optimizer, monotonicity), the eigenvector updates (identity on an
unchanged graph, the exact pairs from a full basis, Rayleigh-Ritz a function of the span only) and the
adjoint gradients (central finite differences)."""
import numpy as np
import pytest
import scipy.optimize as so

import rwsynth
from oracle.adjoint import adjoint_grads, ce_grad, ce_loss, loss_of
from oracle.choose_m import choose_m, f_values, lsqi
from oracle.eigen import certify, dense_eigpairs, principal_angle_sines
from oracle.exact_rw import exact_rw
from oracle.graph import Graph
from oracle.update import bank_select, diag_rq, rayleigh_ritz


@pytest.mark.parametrize("shape,rho", [((8, 3), 0.5), ((8, 3), 50.0), ((4, 7), 0.8), ((4, 7), 100.0),
                                       ((6, 6), 1.3)])
def test_lsqi_kkt_and_optimizer(shape, rho):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    b = rng.standard_normal(shape[0])
    f, mu, alpha = lsqi(A, b, rho)
    # KKT: alpha = (A^T A + mu I)^{-1} A^T b, mu >= 0, ||alpha|| <= rho, mu (||alpha|| - rho) = 0
    assert mu >= 0
    assert np.linalg.norm(alpha) <= rho * (1 + 1e-10)
    if mu > 0:
        np.testing.assert_allclose(np.linalg.norm(alpha), rho, rtol=1e-10)
        np.testing.assert_allclose((A.T @ A + mu * np.eye(shape[1])) @ alpha, A.T @ b, atol=1e-9)
    np.testing.assert_allclose(f, np.sum((A @ alpha - b) ** 2), rtol=1e-10, atol=1e-12)
    # an independent constrained optimizer reaches no lower value
    cons = {"type": "ineq", "fun": lambda a: rho * rho - a @ a}
    best = np.inf
    for x0 in (np.zeros(shape[1]), alpha * 0.5):
        r = so.minimize(lambda a: np.sum((A @ a - b) ** 2), x0, constraints=[cons], method="SLSQP",
                        options={"ftol": 1e-14, "maxiter": 500})
        best = min(best, r.fun)
    assert f <= best + 1e-8


def test_lsqi_exact_fit_is_zero():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((5, 8))
    a = rng.standard_normal(8)
    f, mu, _ = lsqi(A, A @ a, rho=2 * np.linalg.norm(a))
    assert mu == 0.0 and f < 1e-24


def test_choose_m_monotone_and_threshold():
    w = rwsynth.small("t", (14, 12), 4, C=3, seeds_per_label=4, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    g = Graph(J, (14, 12, 1), 4, beta=90.0)
    lam, Q = dense_eigpairs(g, 40)
    fs = np.array([f_values(g, Q, node, lab, 3, m) for m in range(1, 41)])
    assert np.all(np.diff(fs, axis=0) <= 1e-10 * (1 + fs[:-1]))
    m, fmax, f = choose_m(g, Q, node, lab, 3, eps=0.1)
    assert f.max() <= fmax
    if m > 2:
        assert fs[m - 2].max() > fmax       # m-1 does not qualify


def test_diag_rq_identity_on_unchanged_graph():
    w = rwsynth.small("t", (10, 9), 8, n_shapes=3)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (10, 9, 1), 8, beta=90.0)
    lam, Q = dense_eigpairs(g, 15)
    Q2, lam2 = diag_rq(g, Q)
    np.testing.assert_allclose(lam2, lam, atol=1e-13)
    Q3, lam3 = rayleigh_ritz(g, Q)
    np.testing.assert_allclose(lam3, lam, atol=1e-13)
    assert principal_angle_sines(Q3, Q).max() < 1e-7


def test_rr_full_basis_gives_new_eigenpairs():
    w = rwsynth.small("t", (7, 6), 4, n_shapes=3)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (7, 6, 1), 4, beta=90.0)
    lam, Q = dense_eigpairs(g, g.N)
    g2 = g.copy()
    g2.set_beta(150.0)
    g2.remove_edges(g2.edge_id[[3, 10]])
    Qr, lr = rayleigh_ritz(g2, Q)
    np.testing.assert_allclose(lr, np.linalg.eigvalsh(g2.M().toarray()), atol=1e-12)
    res, orth = certify(g2, Qr, lr)
    assert res.max() < 1e-12 and orth < 1e-12


def test_rr_depends_only_on_the_span():
    """Rayleigh-Ritz is a function of span([g_new, Q[:, 1:]]): a basis of the same span (columns 1..
    mixed by an invertible upper-triangular matrix, so not orthonormal) gives the same pairs."""
    w = rwsynth.small("t", (9, 8), 8, n_shapes=3)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (9, 8, 1), 8, beta=90.0)
    lam, Q = dense_eigpairs(g, 14)
    g2 = g.copy()
    g2.set_beta(150.0)
    rng = np.random.default_rng(11)
    R = np.eye(13) + 0.3 * np.triu(rng.standard_normal((13, 13)))
    Qm = Q.copy()
    Qm[:, 1:] = Q[:, 1:] @ R
    Q1, l1 = rayleigh_ritz(g2, Q)
    Q2, l2 = rayleigh_ritz(g2, Qm)
    np.testing.assert_allclose(l2, l1, atol=1e-12)
    assert principal_angle_sines(Q2, Q1).max() < 1e-7   # the sine's floor: sqrt(1 - s^2) near s = 1


def test_adjoint_matches_finite_differences():
    dims = (7, 6, 1)
    w = rwsynth.small("t", dims, 4, C=2, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    gt = rwsynth.label_map(rid, 2)
    g = Graph(J, dims, 4, beta=12.0)
    U = exact_rw(g, node, lab, 2, method="direct")
    G = ce_grad(U, gt, node)
    dw, dJ, dbeta, ds = adjoint_grads(g, node, lab, 2, G, U)
    h = 1e-6

    def L_at(J_=None, beta=None, scale=None):
        g2 = g.copy()
        if J_ is not None:
            g2.J = J_
        if beta is not None:
            g2.beta = beta
        if scale is not None:
            g2.scale = scale
        return loss_of(g2, node, lab, 2, gt)

    for i in (0, 9, 20, 41):
        Jp, Jm = g.J.copy(), g.J.copy()
        Jp[i] += h
        Jm[i] -= h
        fd = (L_at(J_=Jp) - L_at(J_=Jm)) / (2 * h)
        assert abs(fd - dJ[i]) <= 1e-6 * max(1.0, abs(fd))
    fd = (L_at(beta=g.beta + h) - L_at(beta=g.beta - h)) / (2 * h)
    assert abs(fd - dbeta) <= 1e-6 * max(1.0, abs(fd))
    for e in (0, 13, 40):
        sp_, sm_ = g.scale.copy(), g.scale.copy()
        sp_[e] += h
        sm_[e] -= h
        fd = (L_at(scale=sp_) - L_at(scale=sm_)) / (2 * h)
        assert abs(fd - ds[e]) <= 1e-6 * max(1.0, abs(fd))
    assert np.isfinite(ce_loss(U, gt, node))


@pytest.mark.parametrize("dims,conn", [((9, 8, 1), 8), ((6, 5, 4), 6)])
def test_adjoint_cg_equals_direct(dims, conn):
    """The adjoint by Jacobi-PCG (for graphs too large to factor) gives the gradients of the sparse-LU
    adjoint, which the finite-difference pin above fixes."""
    w = rwsynth.small("tc", dims, conn, C=3, seeds_per_label=3, n_shapes=3)
    J, rid = rwsynth.phantom(w)
    node, lab = rwsynth.seeds(w, rid)
    gt = rwsynth.label_map(rid, 3)
    g = Graph(J, dims, conn, beta=12.0)
    U = exact_rw(g, node, lab, 3, method="direct")
    G = ce_grad(U, gt, node)
    ref = adjoint_grads(g, node, lab, 3, G, U)
    Ucg = exact_rw(g, node, lab, 3, method="cg", tol=1e-13)
    np.testing.assert_allclose(Ucg, U, atol=1e-11)
    got = adjoint_grads(g, node, lab, 3, ce_grad(Ucg, gt, node), Ucg, method="cg", tol=1e-13)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(b).max()))


def test_bank_select_prefers_the_current_eigenbasis():
    """Ky Fan: among orthonormal bases of m columns the exact eigenbasis of the m smallest eigenvalues has the
    smallest quotient sum, so a bank holding it (beside the bases of other beta) selects it, and its sum is the
    sum of those eigenvalues."""
    w = rwsynth.small("tb", (9, 8), 4, C=2, seeds_per_label=3, n_shapes=2)
    J, rid = rwsynth.phantom(w)
    bank, betas = [], (20.0, 40.0, 80.0)
    for b in betas:
        _, Q = dense_eigpairs(Graph(J, (9, 8, 1), 4, beta=b), 12)
        bank.append(Q)
    target = Graph(J, (9, 8, 1), 4, beta=40.0)
    idx, Qn, lam, traces = bank_select(target, bank)
    assert idx == 1
    ev = np.linalg.eigvalsh(target.M().toarray())[:12]
    np.testing.assert_allclose(traces[1], ev.sum(), rtol=1e-10, atol=1e-12)
    assert traces[0] > traces[1] and traces[2] > traces[1]
    np.testing.assert_allclose(lam, diag_rq(target, bank[1])[1], rtol=1e-14)
