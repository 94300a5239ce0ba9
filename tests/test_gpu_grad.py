"""GPU parity: gradients of a loss on the exact random walker (autograd Function) against the oracle's
exact adjoint and against central finite differences of the GPU forward."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.adjoint import adjoint_grads, ce_grad, ce_loss
from oracle.exact_rw import exact_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, dev, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("2d4", rwsynth.small("g1", (11, 9), 4, C=2, seeds_per_label=3, n_shapes=2, beta=12.0)),
    ("2d8", rwsynth.small("g2", (9, 10), 8, C=3, seeds_per_label=2, n_shapes=3, beta=20.0)),
    ("3d6", rwsynth.small("g3", (7, 6, 5), 6, C=2, seeds_per_label=3, n_shapes=2, beta=15.0)),
]


def torch_ce(U, gt, seed_node):
    """mean over non-seed voxels of -log max(p_{i, y_i}, 1e-12) (U: (C, N))."""
    N = U.shape[1]
    mask = torch.ones(N, dtype=torch.bool, device=U.device)
    mask[torch.as_tensor(seed_node, device=U.device)] = False
    y = torch.as_tensor(gt, device=U.device, dtype=torch.long)
    p = U.gather(0, y[None, :])[0]
    return -(torch.log(torch.clamp(p[mask], min=1e-12))).mean()


def _run(w, J, node, lab, gt, beta, scale, Q=None, lam=None):
    Jt = to_dev(J, torch.float64).requires_grad_(True)
    bt = torch.tensor(beta, dtype=torch.float64, device=dev(), requires_grad=True)
    st = scale.clone().requires_grad_(True)
    U = rw.random_walker(Jt, bt, st, w.dims, w.conn, node, lab, w.C, Q=Q, lam=lam, tol=1e-14)
    loss = torch_ce(U, gt, node)
    loss.backward()
    return U.detach(), float(loss), Jt.grad, bt.grad, st.grad


@pytest.mark.parametrize("name,w", CASES, ids=[c[0] for c in CASES])
def test_gradients_match_exact_adjoint(name, w):
    need_gpu()
    banner(f"grad {name}")
    J, rid, node, lab = setup_case(w)
    gt = rwsynth.label_map(rid, w.C)
    og = OGraph(J, w.dims, w.conn, w.beta)
    nd = {4: 2, 8: 4, 6: 3}[w.conn]
    scale = torch.ones((nd, og.N), dtype=torch.float64, device=dev())
    U, loss, dJ, db, ds = _run(w, J, node, lab, gt, w.beta, scale)
    Uo = exact_rw(og, node, lab, w.C, method="direct")
    np.testing.assert_allclose(U.cpu().numpy().T, Uo, atol=1e-10)
    assert abs(loss - ce_loss(Uo, gt, node)) < 1e-10
    G = ce_grad(Uo, gt, node)
    dw_o, dJ_o, db_o, ds_o = adjoint_grads(og, node, lab, w.C, G, Uo)
    sc = max(1.0, np.abs(dJ_o).max())
    np.testing.assert_allclose(dJ.cpu().numpy(), dJ_o, atol=1e-9 * sc)
    assert abs(float(db) - db_o) <= 1e-9 * max(1.0, abs(db_o))
    ds_g = ds.cpu().numpy()
    np.testing.assert_allclose(ds_g[og.dir, og.tail], ds_o, atol=1e-9 * max(1.0, np.abs(ds_o).max()))


@pytest.mark.parametrize("name,w", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_gradients_match_finite_differences(name, w):
    need_gpu()
    banner(f"grad fd {name}")
    J, rid, node, lab = setup_case(w)
    gt = rwsynth.label_map(rid, w.C)
    nd = {4: 2, 8: 4, 6: 3}[w.conn]
    og = OGraph(J, w.dims, w.conn, w.beta)
    scale = torch.ones((nd, og.N), dtype=torch.float64, device=dev())
    _, loss, dJ, db, ds = _run(w, J, node, lab, gt, w.beta, scale)
    h = 1e-6

    def L(J_=J, beta=w.beta, s=scale):
        with torch.no_grad():
            U = rw.random_walker(to_dev(J_, torch.float64), torch.tensor(beta, dtype=torch.float64), s, w.dims,
                                 w.conn, node, lab, w.C,
                                 tol=1e-14)
            return float(torch_ce(U, gt, node))

    for i in (0, 17, 40, og.N - 1):
        Jp, Jm = J.copy(), J.copy()
        Jp[i] += h
        Jm[i] -= h
        fd = (L(J_=Jp) - L(J_=Jm)) / (2 * h)
        assert abs(fd - float(dJ[i])) <= 2e-6 * max(1.0, abs(fd)), (i, fd, float(dJ[i]))
    fd = (L(beta=w.beta + h) - L(beta=w.beta - h)) / (2 * h)
    assert abs(fd - float(db)) <= 2e-6 * max(1.0, abs(fd))
    for e in (0, 7, 30):
        d, t = int(og.dir[e]), int(og.tail[e])
        sp, sm = scale.clone(), scale.clone()
        sp[d, t] += h
        sm[d, t] -= h
        fd = (L(s=sp) - L(s=sm)) / (2 * h)
        assert abs(fd - float(ds[d, t])) <= 2e-6 * max(1.0, abs(fd))


def test_eigenbasis_warm_starts_give_the_same_gradients():
    need_gpu()
    w = CASES[0][1]
    J, rid, node, lab = setup_case(w)
    gt = rwsynth.label_map(rid, w.C)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, _ = rw.precompute_eig(g, 12, tol=1e-10)
    scale = torch.ones((2, w.N), dtype=torch.float64, device=dev())
    U1, l1, dJ1, db1, ds1 = _run(w, J, node, lab, gt, w.beta, scale)
    U2, l2, dJ2, db2, ds2 = _run(w, J, node, lab, gt, w.beta, scale, Q=Q, lam=lam)
    assert torch.allclose(U1, U2, atol=1e-11)
    assert torch.allclose(dJ1, dJ2, atol=1e-9)
    assert abs(float(db1) - float(db2)) < 1e-9
