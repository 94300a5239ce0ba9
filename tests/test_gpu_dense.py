"""GPU parity: the dense FP64 building blocks against numpy (symmetric eigendecomposition, LU solve)."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw

from gpu_common import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,count", [(1, 1), (7, 3), (64, 2), (143, 1), (199, 2), (219, 1), (300, 1)])
def test_syev_matches_numpy(n, count):
    need_gpu()
    banner(f"syev n={n} count={count}")
    rng = np.random.default_rng(n)
    mats = []
    for b in range(count):
        X = rng.standard_normal((n, n))
        A = X + X.T
        if b == 1:                       # clustered spectrum with a repeated eigenvalue
            Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
            ev = np.concatenate([np.full(n // 3, 0.5), np.linspace(1e-8, 1, n - n // 3)])
            A = (Qm * ev) @ Qm.T
        mats.append(A)
    At = np.stack([A.T for A in mats])           # column-major storage
    w, V = rw.dense_syev(to_dev(At, torch.float64))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    for b, A in enumerate(mats):
        ev = np.linalg.eigvalsh(A)
        scale = max(1.0, np.abs(ev).max())
        np.testing.assert_allclose(w[b], ev, atol=1e-12 * scale * max(1, n / 50))
        Vb = V[b].T                               # columns = eigenvectors
        assert np.abs(A @ Vb - Vb * w[b]).max() < 1e-11 * scale * max(1, n / 50)
        assert np.abs(Vb.T @ Vb - np.eye(n)).max() < 1e-12 * max(1, n / 50)


@pytest.mark.parametrize("n", [3, 10, 64, 65, 128, 129, 150, 192, 193, 199, 200, 201, 219, 224, 225, 256])
def test_syev_tridiag_matches_numpy(n):
    """Householder + bisection + inverse iteration on matrices with separated eigenvalues (a random
    symmetric matrix, and a Rayleigh-Ritz-like one: a positive spectrum of width 1e-2 rotated by a random
    orthogonal matrix), against numpy; clustered spectra (equal eigenvalues, and gaps of 1e-9) give an
    orthonormal basis of each cluster's subspace; a cluster of more than 32 is refused."""
    need_gpu()
    banner(f"syev tridiag n={n}")
    rng = np.random.default_rng(100 + n)
    X = rng.standard_normal((n, n))
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev_rr = np.sort(1.4e-3 + 1.1e-2 * rng.random(n))
    for A in (X + X.T, (Qm * ev_rr) @ Qm.T):
        A = 0.5 * (A + A.T)
        ev = np.linalg.eigvalsh(A)
        if np.min(np.diff(ev)) < 1e-6 * np.abs(ev).max() * 4:
            continue                                   # the random draw happened to cluster: not this test
        w, V = rw.dense_syev_tridiag(to_dev(A.T, torch.float64))
        w, V = w.cpu().numpy(), V.cpu().numpy().T      # columns = eigenvectors
        scale = np.abs(ev).max()
        np.testing.assert_allclose(w, ev, atol=1e-13 * scale * max(1, n / 20))
        assert np.abs(A @ V - V * w).max() < 1e-12 * scale * max(1, n / 20)
        assert np.abs(V.T @ V - np.eye(n)).max() < 1e-11 * max(1, n / 50)
    if n >= 10:
        for ev in (np.concatenate([np.full(3, 0.5), np.linspace(1.0, 2.0, n - 3)]),
                   np.concatenate([0.5 + 1e-9 * np.arange(4), np.linspace(1.0, 2.0, n - 4)])):
            A = (Qm * ev) @ Qm.T
            A = 0.5 * (A + A.T)
            w, V = rw.dense_syev_tridiag(to_dev(A.T, torch.float64))
            w, V = w.cpu().numpy(), V.cpu().numpy().T
            np.testing.assert_allclose(w, np.sort(ev), atol=1e-13 * max(1, n / 20))
            assert np.abs(A @ V - V * w).max() < 1e-12 * max(1, n / 20)
            assert np.abs(V.T @ V - np.eye(n)).max() < 1e-11 * max(1, n / 50)
    if n >= 40:
        ev = np.concatenate([np.full(33, 0.5), np.linspace(1.0, 2.0, n - 33)])
        A = (Qm * ev) @ Qm.T
        with pytest.raises(rw.RWError):
            rw.dense_syev_tridiag(to_dev(0.5 * (A + A.T).T, torch.float64))


@pytest.mark.parametrize("n", [40, 150, 199])
def test_syev_tridiag_already_reduced(n):
    """Inputs whose columns are already reduced, so that the reflectors are the identity (tau = 0) and the
    reduction must leave the matrix unchanged: a tridiagonal matrix, a diagonal one, and a block-diagonal
    one (two tridiagonal blocks), against numpy."""
    need_gpu()
    banner(f"syev tridiag already reduced n={n}")
    rng = np.random.default_rng(300 + n)
    d = rng.standard_normal(n)
    e = rng.uniform(0.5, 1.5, n - 1) * rng.choice([-1.0, 1.0], n - 1)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    D = np.diag(np.linspace(-1.0, 1.0, n))
    B = T.copy()
    B[n // 2, n // 2 - 1] = B[n // 2 - 1, n // 2] = 0.0
    for A in (T, D, B):
        ev = np.linalg.eigvalsh(A)
        w, V = rw.dense_syev_tridiag(to_dev(A.T, torch.float64))
        w, V = w.cpu().numpy(), V.cpu().numpy().T
        scale = np.abs(ev).max()
        np.testing.assert_allclose(w, ev, atol=1e-13 * scale * max(1, n / 20))
        assert np.abs(A @ V - V * w).max() < 1e-12 * scale * max(1, n / 20)
        assert np.abs(V.T @ V - np.eye(n)).max() < 1e-11 * max(1, n / 50)


@pytest.mark.parametrize("sizes", [[64, 7, 50], [150, 129, 192, 100]], ids=["to64", "to192"])
def test_eig_rhs_batched_other_orders(sizes):
    """The batched eigenproblem at the other register layouts (orders up to 64, and 129 to 192): ascending
    eigenvalues against numpy and the sign-free products of the rotated right-hand sides."""
    need_gpu()
    banner(f"eig rhs batched sizes={sizes}")
    rng = np.random.default_rng(sum(sizes))
    ld, nrhs = max(sizes), 2
    A = rng.standard_normal((len(sizes), ld, ld))
    R = rng.standard_normal((len(sizes), nrhs, ld))
    for b, n in enumerate(sizes):
        X = rng.standard_normal((n + 40, n))
        A[b, :n, :n] = (X.T @ X).T
    w, Rp = rw.dense_eig_rhs_batched(to_dev(A, torch.float64), sizes, to_dev(R, torch.float64))
    w, Rp = w.cpu().numpy(), Rp.cpu().numpy()
    for b, n in enumerate(sizes):
        ev, V = np.linalg.eigh(A[b, :n, :n].T)
        scale = np.abs(ev).max()
        np.testing.assert_allclose(w[b, :n], ev, atol=1e-12 * scale)
        ref = V.T @ R[b, :, :n].T
        got = Rp[b, :, :n].T
        gap = np.min(np.diff(ev))
        tol = 1e-12 * scale / gap * np.abs(R[b, :, :n]).max() ** 2 * n
        for c in range(nrhs):
            for dd in range(nrhs):
                np.testing.assert_allclose(got[:, c] * got[:, dd], ref[:, c] * ref[:, dd], atol=tol)


def test_eig_rhs_batched_matches_numpy():
    """The choice-of-m eigenproblem through the tridiagonal form: a batch of Gram matrices of different
    orders inside one leading dimension (entries beyond each order hold garbage that must not be read),
    against numpy: ascending eigenvalues, and V^T R compared through the sign-free products
    (V^T R)_ic (V^T R)_id; rows beyond each order come back zero.  A threefold eigenvalue is solved, more
    than 32 equal ones are refused."""
    need_gpu()
    banner("eig rhs batched")
    rng = np.random.default_rng(31)
    ld, nrhs = 90, 3
    sizes = [88, 60, 90, 3, 45]
    A = rng.standard_normal((len(sizes), ld, ld))            # garbage everywhere, then the leading blocks
    R = rng.standard_normal((len(sizes), nrhs, ld))
    for b, n in enumerate(sizes):
        X = rng.standard_normal((150, n))
        A[b, :n, :n] = (X.T @ X).T                           # column-major storage of a symmetric matrix
    w, Rp = rw.dense_eig_rhs_batched(to_dev(A, torch.float64), sizes, to_dev(R, torch.float64))
    w, Rp = w.cpu().numpy(), Rp.cpu().numpy()
    for b, n in enumerate(sizes):
        M = A[b, :n, :n].T
        ev, V = np.linalg.eigh(M)
        scale = np.abs(ev).max()
        np.testing.assert_allclose(w[b, :n], ev, atol=1e-12 * scale)
        assert np.all(w[b, n:] == 0.0) and np.all(Rp[b, :, n:] == 0.0)
        ref = V.T @ R[b, :, :n].T                             # (n, nrhs)
        got = Rp[b, :, :n].T
        gap = np.min(np.diff(ev)) if n > 1 else scale
        tol = 1e-12 * scale / gap * np.abs(R[b, :, :n]).max() ** 2 * n
        for c in range(nrhs):
            for d in range(nrhs):
                np.testing.assert_allclose(got[:, c] * got[:, d], ref[:, c] * ref[:, d], atol=tol)
    # a threefold eigenvalue: within the cluster the rotated rows depend on the basis chosen for its subspace,
    # so their products are compared summed over the cluster (the secular equation uses only those sums)
    Qm, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    ev = np.concatenate([np.full(3, 0.5), np.linspace(1.0, 2.0, 37)])
    C = np.zeros((1, ld, ld))
    C[0, :40, :40] = ((Qm * ev) @ Qm.T).T
    w, Rp = rw.dense_eig_rhs_batched(to_dev(C, torch.float64), [40], to_dev(R[:1], torch.float64))
    w, Rp = w.cpu().numpy()[0], Rp.cpu().numpy()[0]
    np.testing.assert_allclose(w[:40], np.sort(ev), atol=1e-13)
    ref = Qm.T @ R[0, :, :40].T
    ref = ref[np.argsort(ev, kind="stable")]
    got = Rp[:, :40].T
    for c in range(nrhs):
        for d in range(nrhs):
            np.testing.assert_allclose(got[3:, c] * got[3:, d], ref[3:, c] * ref[3:, d], atol=1e-11)
            np.testing.assert_allclose((got[:3, c] * got[:3, d]).sum(), (ref[:3, c] * ref[:3, d]).sum(), atol=1e-11)
    # more than 32 equal eigenvalues: refused (the caller uses the Jacobi solver)
    ev = np.concatenate([np.full(33, 0.5), np.linspace(1.0, 2.0, 7)])
    C[0, :40, :40] = ((Qm * ev) @ Qm.T).T
    with pytest.raises(rw.RWError):
        rw.dense_eig_rhs_batched(to_dev(C, torch.float64), [40], to_dev(R[:1], torch.float64))


@pytest.mark.parametrize("n,nrhs", [(1, 1), (2, 1), (3, 2), (50, 3), (63, 1), (64, 9), (65, 3), (80, 3), (90, 4), (100, 12), (112, 2),
                                    (128, 5), (129, 2), (150, 3), (192, 4), (193, 1), (201, 4), (200, 20), (208, 8),
                                    (209, 2), (75, 260)])
def test_lu_solve_matches_numpy(n, nrhs):
    need_gpu()
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + n * 0.01 * np.eye(n)
    B = rng.standard_normal((n, nrhs))
    X, stat = rw.dense_lu_solve(to_dev(A.T, torch.float64), to_dev(B.T, torch.float64))
    assert stat > 0
    np.testing.assert_allclose(X.cpu().numpy().T, np.linalg.solve(A, B), rtol=1e-9, atol=1e-11)
    if n < 2:
        return
    S = A.copy()
    S[:, -1] = S[:, 0]                            # singular
    _, stat = rw.dense_lu_solve(to_dev(S.T, torch.float64), to_dev(B.T, torch.float64))
    assert stat == 0.0
