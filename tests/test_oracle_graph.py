"""Pins of the oracle's graph and Laplacian against facts that do not come from the oracle itself:
brute-force neighbour enumeration, closed-form edge counts, Laplacian invariants, and the closed-form
spectrum of the beta = 0 grid (a Cartesian sum of path graphs, diagonalized by the DCT-II)."""
import itertools

import numpy as np
import pytest

import rwsynth
from oracle.graph import Graph


def brute_W(J, dims, conn, beta):
    """Weights by the definition: every pair of voxels at unit (4/6) or king (8) distance."""
    nx, ny, nz = dims
    N = nx * ny * nz
    W = np.zeros((N, N))
    for a in range(N):
        ax, ay, az = a % nx, (a // nx) % ny, a // (nx * ny)
        for b in range(N):
            if a == b:
                continue
            bx, by, bz = b % nx, (b // nx) % ny, b // (nx * ny)
            d = (abs(ax - bx), abs(ay - by), abs(az - bz))
            if conn in (4, 6):
                nb = sum(d) == 1
            else:
                nb = max(d) == 1 and az == bz
            if nb:
                W[a, b] = np.exp(-beta * (J[a] - J[b]) ** 2)
    return W


@pytest.mark.parametrize("dims,conn", [((5, 4, 1), 4), ((5, 4, 1), 8), ((3, 4, 2), 6)])
def test_weights_match_brute_force(dims, conn):
    rng = np.random.default_rng(1)
    N = dims[0] * dims[1] * dims[2]
    J = rng.uniform(0, 1, N)
    g = Graph(J, dims, conn, beta=7.0)
    Wb = brute_W(J, dims, conn, 7.0)
    np.testing.assert_allclose(g.W().toarray(), Wb, rtol=0, atol=1e-15)


def test_edge_counts_closed_form():
    for (nx, ny) in [(64, 64), (7, 3)]:
        assert Graph(np.zeros(nx * ny), (nx, ny, 1), 4, 1.0).edge_id.size == (nx - 1) * ny + nx * (ny - 1)
        assert Graph(np.zeros(nx * ny), (nx, ny, 1), 8, 1.0).edge_id.size == \
            (nx - 1) * ny + nx * (ny - 1) + 2 * (nx - 1) * (ny - 1)
    nx, ny, nz = 6, 5, 4
    assert Graph(np.zeros(nx * ny * nz), (nx, ny, nz), 6, 1.0).edge_id.size == \
        (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    # the generator's edge-id list is the same set
    for dims, conn in [((9, 7, 1), 8), ((4, 5, 3), 6)]:
        g = Graph(np.zeros(np.prod(dims)), dims, conn, 1.0)
        assert np.array_equal(np.sort(g.edge_id), np.sort(rwsynth.edge_ids_valid(dims, conn)))


@pytest.mark.parametrize("conn,dims", [(4, (9, 8, 1)), (8, (9, 8, 1)), (6, (5, 4, 3))])
def test_laplacian_invariants(conn, dims):
    w = rwsynth.small("t", dims, conn)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, dims, conn, beta=90.0)
    L = g.L().toarray()
    d = g.degree()
    assert np.abs(L.sum(axis=1)).max() <= 1e-15 * max(1.0, d.max())
    np.testing.assert_array_equal(L, L.T)
    Lh = g.Lhat().toarray()
    np.testing.assert_allclose(Lh @ np.sqrt(d), 0.0, atol=1e-14)
    ev = np.linalg.eigvalsh(Lh)
    assert ev.min() > -1e-13 and ev.max() < 2.0 + 1e-13
    assert abs(ev[0]) < 1e-13
    np.testing.assert_allclose(np.linalg.norm(g.ghat()), 1.0, rtol=1e-15)


def test_doubling_beta_squares_weights():
    """Sec. IV-C: doubling beta squares every weight."""
    w = rwsynth.small("t", (8, 8), 8)
    J, _ = rwsynth.phantom(w)
    g1 = Graph(J, (8, 8, 1), 8, beta=33.0)
    g2 = Graph(J, (8, 8, 1), 8, beta=66.0)
    np.testing.assert_allclose(g2.w, g1.w ** 2, rtol=1e-13)
    ga = Graph(J, (8, 8, 1), 8, beta=33.0, weight_form="abs")
    gb = Graph(J, (8, 8, 1), 8, beta=66.0, weight_form="abs")
    np.testing.assert_allclose(gb.w, ga.w ** 2, rtol=1e-13)


def path_eigs(n):
    k = np.arange(n)
    return 4.0 * np.sin(np.pi * k / (2 * n)) ** 2


@pytest.mark.parametrize("dims,conn", [((7, 5, 1), 4), ((4, 3, 5), 6)])
def test_beta0_spectrum_is_dct(dims, conn):
    """beta = 0, free boundary: L is the Cartesian sum of path-graph Laplacians; its eigenvalues are
    sums of 4 sin^2(pi k / 2n) and its eigenvectors products of cos(pi k (x + 1/2) / n)."""
    N = int(np.prod(dims))
    g = Graph(np.random.default_rng(0).uniform(size=N), dims, conn, beta=0.0, normalized=False)
    L = g.L().toarray()
    axes = [n for n in dims if n > 1]
    expect = np.sort([sum(c) for c in itertools.product(*[path_eigs(n) for n in axes])])
    np.testing.assert_allclose(np.linalg.eigvalsh(L), expect, atol=1e-12)
    # one eigenvector by the closed form
    nx, ny, nz = dims
    kx, ky, kz = 2, 1, min(1, nz - 1)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    v = (np.cos(np.pi * kx * (x + 0.5) / nx) * np.cos(np.pi * ky * (y + 0.5) / ny)
         * np.cos(np.pi * kz * (z + 0.5) / nz)).reshape(-1)
    lam = path_eigs(nx)[kx] + path_eigs(ny)[ky] + (path_eigs(nz)[kz] if nz > 1 else 0.0)
    np.testing.assert_allclose(L @ v, lam * v, atol=1e-12)


def test_edits():
    w = rwsynth.small("t", (10, 9), 8)
    J, _ = rwsynth.phantom(w)
    g = Graph(J, (10, 9, 1), 8, beta=90.0)
    w0 = g.w.copy()
    ids = g.box_edge_ids((2, 3, 0), (6, 7, 1))
    # both endpoints inside a 4x4 box: 3*4 + 4*3 + 2*3*3 edges
    assert ids.size == 3 * 4 + 4 * 3 + 2 * 3 * 3
    g.scale_box((2, 3, 0), (6, 7, 1), 0.1)
    sel = np.isin(g.edge_id, ids)
    np.testing.assert_allclose(g.w[sel], 0.1 * w0[sel], rtol=1e-15)
    np.testing.assert_array_equal(g.w[~sel], w0[~sel])
    g.set_beta(150.0)
    g2 = Graph(J, (10, 9, 1), 8, beta=150.0)
    np.testing.assert_allclose(g.w[sel], 0.1 * g2.w[sel], rtol=1e-15)
    rm = g.edge_id[[0, 5, 17]]
    g.remove_edges(rm)
    assert np.all(g.w[[0, 5, 17]] == 0.0)
    mb = g.mask_bits()
    for e in rm:
        d, t = divmod(int(e), g.N)
        assert not (mb[t] >> d) & 1
    with pytest.raises(ValueError):
        g.remove_edges(rm[:1])          # already removed
