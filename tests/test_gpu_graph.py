"""GPU parity: graph build, edits and the stencil operator against the oracle."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.graph import Graph as OGraph

from gpu_common import banner, dev, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("2d4_f64", rwsynth.small("a", (67, 45), 4, n_shapes=3), torch.float64),
    ("2d8_f32", rwsynth.small("b", (70, 33), 8, n_shapes=4), torch.float32),
    ("2d8_f64", rwsynth.small("c", (33, 70), 8, n_shapes=4), torch.float64),
    ("3d6_f32", rwsynth.small("d", (21, 17, 9), 6, n_shapes=3), torch.float32),
    ("3d6_f64", rwsynth.small("e", (9, 23, 13), 6, n_shapes=3), torch.float64),
]


def _rtol(dt):
    return 1e-15 if dt == torch.float64 else 0.0


def _weight_rtol(og):
    """exp(x) has condition number |x|: the argument x = -beta dJ^2 is rounded differently by the two
    sides (operation order), so the FP64 weights can differ by ~ 4 u (1 + |x|) relative."""
    diff = og.J[og.tail] - og.J[og.head]
    x = og.beta * diff * diff
    rt = np.zeros((len(og.weights_by_dir()), og.N))
    rt[og.dir, og.tail] = 4 * 2.0 ** -53 * (1 + x)
    return rt


def _check_graph(gg, og, dt):
    v = gg.view()
    np.testing.assert_array_equal(v["mask"].cpu().numpy(), og.mask_bits())
    # weights, scales and degrees are FP64 on every graph; only the operator's coefficients take its type
    w_ref = og.weights_by_dir()
    w = v["weight"].cpu().numpy()
    assert v["weight"].dtype == torch.float64 and v["scale"].dtype == torch.float64
    assert np.all(np.abs(w - w_ref) <= _weight_rtol(og) * w_ref)
    d_ref = og.degree()
    np.testing.assert_allclose(v["degree"].cpu().numpy(), d_ref, rtol=1e-14)
    # FP32 graph: coefficients and the null vector are the FP64 values rounded once (1 ulp, plus the FP64
    # sides' own rounding differences); FP32 subnormals have an absolute spacing of 2^-149
    tol, atol = (1e-13, 1e-300) if dt == torch.float64 else (1.2e-7, 2.0 ** -149)
    np.testing.assert_allclose(v["ghat"].cpu().numpy().astype(np.float64), og.ghat(), rtol=tol, atol=atol)
    dinv = og.dinv_sqrt()
    c_ref = np.zeros_like(w_ref)
    c_ref[og.dir, og.tail] = og.w * dinv[og.tail] * dinv[og.head]
    np.testing.assert_allclose(v["coef"].cpu().numpy().astype(np.float64), c_ref, rtol=tol, atol=atol)


@pytest.mark.parametrize("name,w,dt", CASES, ids=[c[0] for c in CASES])
def test_graph_build_matches_oracle(name, w, dt):
    need_gpu()
    banner(f"graph build {name}")
    J, rid, node, lab = setup_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, 90.0, dtype=dt)
    og = OGraph(J, w.dims, w.conn, 90.0)
    _check_graph(gg, og, dt)


@pytest.mark.parametrize("name,w,dt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("normalized", [True, False])
def test_stencil_matches_oracle(name, w, dt, normalized):
    need_gpu()
    banner(f"stencil {name} normalized={normalized}")
    J, rid, node, lab = setup_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, 90.0, dtype=dt, normalized=normalized)
    og = OGraph(J, w.dims, w.conn, 90.0, normalized=normalized)
    M = og.M()
    rng = np.random.default_rng(4)
    for b in (1, 3, 37):
        X = rng.standard_normal((b, og.N))
        Y = rw.apply_laplacian(gg, to_dev(X, dt)).cpu().numpy().astype(np.float64)
        Xr = X.astype(np.float32).astype(np.float64) if dt == torch.float32 else X
        Yref = (M @ Xr.T).T
        err = np.linalg.norm(Y - Yref) / np.linalg.norm(Yref)
        assert err < (1e-13 if dt == torch.float64 else 2e-6), err
    # fused form: Y = a op X + b X + c Z
    X = rng.standard_normal((5, og.N))
    Z = rng.standard_normal((5, og.N))
    Yd = torch.empty_like(to_dev(X, dt))
    rw.apply_laplacian_axpby(gg, to_dev(X, dt), Yd, to_dev(Z, dt), 0.7, -0.3, 1.9)
    Xr, Zr = (X.astype(np.float32).astype(np.float64), Z.astype(np.float32).astype(np.float64)) \
        if dt == torch.float32 else (X, Z)
    ref = 0.7 * (M @ Xr.T).T - 0.3 * Xr + 1.9 * Zr
    err = np.linalg.norm(Yd.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < (1e-13 if dt == torch.float64 else 2e-6), err
    # the timed launch: bit-identical to the plain one, with the dispatch's own interval in the events
    X = to_dev(rng.standard_normal((37, og.N)), dt)
    Yp = rw.apply_laplacian(gg, X)
    Yt = torch.empty_like(X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rw.apply_laplacian_timed(gg, X, Yt, e0, e1)
    torch.cuda.synchronize()
    assert torch.equal(Yp, Yt)
    assert e0.elapsed_time(e1) > 0.0


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_edits_match_oracle(dt):
    need_gpu()
    banner(f"edits {dt}")
    w = rwsynth.small("ed", (48, 40), 8, n_shapes=4)
    J, rid, node, lab = setup_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, 90.0, dtype=dt)
    og = OGraph(J, w.dims, w.conn, 90.0)
    rng = np.random.default_rng(11)
    valid = rwsynth.edge_ids_valid(w.dims, w.conn)
    rem = np.sort(rng.choice(valid, 60, replace=False))
    sc = np.sort(rng.choice(np.setdiff1d(valid, rem), 25, replace=False))
    edits = [rwsynth.Edit("set_beta", 150.0),
             rwsynth.Edit("scale_box", 0.1, (5, 7, 0), (21, 30, 1)),
             rwsynth.Edit("scale_edges", 3.0, edge_ids=sc),
             rwsynth.Edit("remove_edges", edge_ids=rem)]
    rw.edit_graph(gg, edits)
    for e in edits:
        og.apply_edit(e)
    _check_graph(gg, og, dt)
    # removing an edge twice is an error and leaves the graph unchanged
    with pytest.raises(rw.RWError) as ei:
        rw.edit_graph(gg, [rwsynth.Edit("remove_edges", edge_ids=rem[:2])])
    assert ei.value.status == rw.RW_EINVAL
    _check_graph(gg, og, dt)


def test_invalid_graph_arguments():
    need_gpu()
    J = to_dev(np.zeros(12), torch.float64)
    with pytest.raises(rw.RWError):
        rw.Graph(J, (4, 3), 6, 1.0)          # 6-connectivity is 3D only
    with pytest.raises(rw.RWError):
        rw.Graph(J, (4, 3), 4, -1.0)         # beta < 0


@pytest.mark.parametrize("dims,conn,dt", [((40, 31), 4, torch.float32), ((33, 29), 8, torch.float64),
                                          ((14, 12, 11), 6, torch.float32)])
def test_components_match_scipy(dims, conn, dt):
    """Components over edges with w >= 1e-30 against scipy's connected components on the oracle's edge list:
    the same partition (each node's root is its component's smallest node index)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    need_gpu()
    banner(f"components {dims} conn={conn}")
    w = rwsynth.small("cc", dims, conn, n_shapes=4, beta=90.0)
    J, rid, node, lab = setup_case(w)
    J = J.copy()
    J[rid == 1] += 12.0                    # shape 1 cut off: weights exp(-90 * 144) underflow to 0
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, 90.0, dtype=dt)
    og = OGraph(J, w.dims, w.conn, 90.0)
    keep = og.w >= 1e-30
    A = sp.coo_matrix((np.ones(keep.sum()), (og.tail[keep], og.head[keep])), shape=(og.N, og.N))
    n_ref, labels = connected_components(A, directed=False)
    n_gpu, comp = gg.components()
    comp = comp.cpu().numpy()
    assert n_gpu == n_ref
    first = np.full(n_ref, og.N)
    np.minimum.at(first, labels, np.arange(og.N))
    np.testing.assert_array_equal(comp, first[labels])


def test_unanchored_component_is_reported():
    need_gpu()
    w = rwsynth.small("ua", (20, 20), 4, n_shapes=1)
    J = np.zeros(w.N)
    box = np.zeros((20, 20), dtype=bool)
    box[6:12, 7:13] = True
    J[box.reshape(-1)] = 10.0                # exp(-90 * 100) = 0: the box is its own component
    outside = np.flatnonzero(~box.reshape(-1))
    inside = np.flatnonzero(box.reshape(-1))
    node = np.array([outside[0], outside[-1]])
    lab = np.array([0, 1], dtype=np.int32)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, 90.0, dtype=torch.float64)
    assert g.components()[0] == 2
    Q, lam, _ = rw.precompute_eig(g, 8, tol=1e-9)
    for call in (lambda n, l: rw.solve_seeds(g, Q, lam, n, l, 2), lambda n, l: rw.cg_solve(g, n, l, 2)):
        with pytest.raises(rw.RWError) as ei:
            call(node, lab)
        assert ei.value.status == rw.RW_EUNANCHORED
        call(np.append(node, inside[0]), np.append(lab, 0).astype(np.int32))   # anchored: no error
