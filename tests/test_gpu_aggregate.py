"""GPU parity for vertex aggregation (Sec. III-C) over regular blocks: the aggregated graph's weights, the
eigenvector transfer of eq. (33) with Gram-Schmidt and the normalized-cut values, the fast walker on the
aggregated graph and the propagation back, against the oracle."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.aggregate import aggregate_graph, coarse_seeds, prolong, transfer_basis
from oracle.fast_rw import fast_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

CASES = [("2d4", (41, 33), 4, 3, 20), ("2d8", (40, 30), 8, 4, 24), ("3d6", (13, 11, 9), 6, 2, 20)]


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)], ids=["f64", "f32"])
@pytest.mark.parametrize("name,dims,conn,s,m", CASES, ids=[c[0] for c in CASES])
def test_aggregation_matches_oracle(dt, tol, name, dims, conn, s, m):
    need_gpu()
    banner(f"aggregate {name} {dt} s={s}")
    w = rwsynth.small("ag", dims, conn, m=m, C=2, seeds_per_label=4, n_shapes=3)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=dt)
    Q, lam, _ = rw.precompute_eig(g, m, tol=1e-10 if dt == torch.float64 else 1e-5, max_iter=400)
    og = OGraph(J, w.dims, w.conn, w.beta)
    # the aggregated graph
    c = rw.aggregate(g, s)
    co = aggregate_graph(og, s)
    wv = c.view()["weight"].cpu().numpy()
    np.testing.assert_allclose(wv[co.dir, co.tail], co.w, rtol=1e-13, atol=1e-300)
    # the transfer: eq. (33), Gram-Schmidt, quotients
    Qc, lamc = rw.aggregate_basis(g, c, s, Q)
    co2, Qo, lamo = transfer_basis(og, Q.double().cpu().numpy().T, s)
    gate = 1e-10 if dt == torch.float64 else 1e-4
    assert np.abs(Qc.double().cpu().numpy().T - Qo).max() <= gate * max(1.0, np.abs(Qo).max())
    np.testing.assert_allclose(lamc.cpu().numpy(), lamo, rtol=gate, atol=gate * np.abs(lamo).max())
    # the walker on the blocks and the propagation
    cn, cl = rw.aggregate_seeds(g, s, node, lab)
    cno, clo = coarse_seeds(og, s, node, lab)
    np.testing.assert_array_equal(cn, cno)
    np.testing.assert_array_equal(cl, clo)
    Uc, _ = rw.solve_seeds(c, Qc, lamc, cn, cl, w.C)
    exact = bool(np.min(np.abs(lamo[1:])) < 1e-6)
    Uco = fast_rw(co2, Qo, lamo, cno, clo, w.C, exact=exact)
    err = np.abs(Uc.double().cpu().numpy().T - Uco).max()
    print(f"  coarse {c.dims}, lambda_1 {lamo[1]:.2e}, walker err {err:.2e}", flush=True)
    assert err <= gate * max(1.0, np.abs(Uco).max()), err
    U = rw.prolong(g, s, Uc)
    np.testing.assert_array_equal(U.cpu().numpy().T, prolong(og, s, Uc.cpu().numpy().T))


def test_aggregation_rejects_conflicting_seeds():
    need_gpu()
    w = rwsynth.small("ag2", (20, 18), 4, m=8, C=2)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    with pytest.raises(rw.RWError):
        rw.aggregate_seeds(g, 4, [0, 1], [0, 1])
    with pytest.raises(rw.RWError):
        rw.aggregate(g, 100)                                     # a single block
