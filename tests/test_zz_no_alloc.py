"""The allocation-free solve (rw_solve_seeds_noalloc) against rw_solve_seeds with the same fixed m, on two
calls in a row (the second on a smaller graph with fewer seeds, fewer labels and a smaller m, so that the
shared device array still holds the first call's larger contents), and its size limits."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.eigen import dense_eigpairs
from oracle.fast_rw import fast_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu

# (workload, graph dtype, basis dtype, gate against the oracle)
CALLS = [
    (rwsynth.small("na1", (40, 37), 8, m=60, C=4, seeds_per_label=6, n_shapes=4), torch.float32, torch.float32, 1e-4),
    (rwsynth.small("na2", (23, 19), 4, m=24, C=2, seeds_per_label=3, n_shapes=3), torch.float64, torch.float64, 1e-10),
]


def _case(w, gdt, qdt):
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    og = OGraph(J, w.dims, w.conn, w.beta)
    lam, Q = dense_eigpairs(og, w.m)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=gdt)
    return og, g, to_dev(Q.T, qdt), to_dev(lam, torch.float64), node, lab


def test_noalloc_solve_matches_solve_seeds_on_two_calls():
    need_gpu()
    for k, (w, gdt, qdt, tol) in enumerate(CALLS):
        banner(f"noalloc call {k}: {w.dims} m={w.m} C={w.C}")
        og, g, Qd, lamd, node, lab = _case(w, gdt, qdt)
        Ua, ia = rw.solve_seeds_noalloc(g, Qd, lamd, node, lab, w.C, m=w.m)
        Ub, ib = rw.solve_seeds(g, Qd, lamd, node, lab, w.C, eps=0.0, m_avail=w.m)
        torch.cuda.synchronize()
        # same kernels, same launch shapes, same inputs: the same results
        assert torch.equal(Ua, Ub), (k, (Ua.double() - Ub.double()).abs().max().item())
        assert ia["m_used"] == w.m and ia["min_pivot"] == ib["min_pivot"]
        Uo = fast_rw(og, Qd.double().cpu().numpy().T, lamd.cpu().numpy(), node, lab, w.C,
                     exact=bool(np.min(np.abs(lamd.cpu().numpy()[1:])) < 1e-6))
        err = np.abs(Ua.double().cpu().numpy().T - Uo).max()
        assert err <= tol * max(1.0, np.abs(Uo).max()), (k, err)


def test_noalloc_solve_rejects_what_exceeds_its_array():
    need_gpu()
    w, gdt, qdt, _ = CALLS[1]
    og, g, Qd, lamd, node, lab = _case(w, gdt, qdt)
    many = np.arange(16385, dtype=np.int64) % og.N
    with pytest.raises(rw.RWError) as ei:
        rw.solve_seeds_noalloc(g, Qd, lamd, many, np.zeros(many.size, np.int32), w.C, m=w.m)
    assert ei.value.status == rw.RW_EWORKSPACE
    # 16384 seeds at m = 300: the seed rows of Q and B Q alone need 2 * 16384 * 300 * 8 bytes > 64 MiB
    big = rwsynth.small("na_big", (200, 100), 4, m=300, C=2, seeds_per_label=1, n_shapes=1)
    gb = rw.Graph(torch.zeros(big.N, dtype=torch.float64, device=Qd.device), big.dims, big.conn, big.beta,
                  dtype=torch.float32)
    Qb = torch.zeros((300, big.N), dtype=torch.float32, device=Qd.device)
    lb = torch.zeros(300, dtype=torch.float64, device=Qd.device)
    seeds = np.arange(16384, dtype=np.int64)
    with pytest.raises(rw.RWError) as ei:
        rw.solve_seeds_noalloc(gb, Qb, lb, seeds, np.zeros(seeds.size, np.int32), 2, m=300)
    assert ei.value.status == rw.RW_EWORKSPACE
    # the array still serves a normal call afterwards
    Ua, _ = rw.solve_seeds_noalloc(g, Qd, lamd, node, lab, w.C, m=w.m)
    Ub, _ = rw.solve_seeds(g, Qd, lamd, node, lab, w.C, eps=0.0, m_avail=w.m)
    assert torch.equal(Ua, Ub)
