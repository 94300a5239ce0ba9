"""GPU parity for the bank of bases precomputed for several beta (Sec. III-B, last paragraph): for the
current operator every bank basis gets the diagonal update of eq. (27), and the basis with the smallest
quotient sum is used; against the oracle's selection, quotient sums and updated pairs."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.graph import Graph as OGraph
from oracle.update import bank_select

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

BETAS = (30.0, 60.0, 120.0)


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)], ids=["f64", "f32"])
@pytest.mark.parametrize("beta", [45.0, 60.0, 200.0])
def test_bank_selection_matches_oracle(dt, tol, beta):
    need_gpu()
    banner(f"bank {dt} beta={beta}")
    w = rwsynth.small("bk", (40, 33), 8, m=16, C=2, seeds_per_label=3, n_shapes=3)
    J, rid, node, lab = setup_case(w)
    bank = []
    for b in BETAS:
        gb = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, b, dtype=dt)
        Q, lam, _ = rw.precompute_eig(gb, w.m, tol=tol, max_iter=400)
        bank.append(Q.contiguous())
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, beta, dtype=dt)
    idx, Qg, lamg, traces = rw.bank_select(g, bank)
    og = OGraph(J, w.dims, w.conn, beta)
    idx_o, Qo, lamo, traces_o = bank_select(og, [Q.double().cpu().numpy().T for Q in bank])
    rel = 1e-10 if dt == torch.float64 else 1e-5
    np.testing.assert_allclose(traces, traces_o, rtol=rel)
    srt = np.sort(traces_o)
    if srt[1] - srt[0] > 10 * rel * abs(srt[0]):                # not a tie at this precision
        assert idx == idx_o, (idx, idx_o, traces_o)
    if beta in BETAS:                                            # Ky Fan: the basis computed for this beta
        assert idx == BETAS.index(beta)
    np.testing.assert_allclose(lamg.cpu().numpy(), lamo, rtol=rel, atol=rel * abs(lamo).max())
    err = np.abs(Qg.double().cpu().numpy().T - Qo).max()
    assert err <= (1e-10 if dt == torch.float64 else 2e-5), err
    # the bank is read only
    for b, Q in zip(BETAS, bank):
        assert torch.isfinite(Q).all()
    U, _ = rw.solve_seeds(g, Qg, lamg, node, lab, w.C)
    np.testing.assert_allclose(U.double().sum(dim=0).cpu().numpy(), 1.0, atol=1e-5)


def test_bank_rejects_bad_arguments():
    need_gpu()
    w = rwsynth.small("bk2", (20, 18), 4, m=8, C=2)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
    with pytest.raises(rw.RWError):
        rw.bank_select(g, [Q.double().contiguous()])             # another dtype than the graph's
    with pytest.raises(AssertionError):
        rw.bank_select(g, [Q, Q[:4].contiguous()])               # bases of different shapes
