"""GPU parity: exact random walker by CG against the oracle's direct solve."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.exact_rw import exact_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("2d64_cfg1", rwsynth.CFG1),
    ("2d8_small", rwsynth.small("c2", (37, 29), 8, C=3, seeds_per_label=6, n_shapes=4)),
    ("3d6_small", rwsynth.small("c3", (14, 12, 11), 6, C=2, seeds_per_label=8, n_shapes=3)),
]


@pytest.mark.parametrize("name,w", CASES, ids=[c[0] for c in CASES])
def test_cg_matches_direct_solve(name, w):
    need_gpu()
    banner(f"cg {name}")
    J, rid, node, lab = setup_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    og = OGraph(J, w.dims, w.conn, w.beta)
    U, info = rw.cg_solve(gg, node, lab, w.C, tol=1e-12)
    Ue = exact_rw(og, node, lab, w.C, method="direct")
    Ug = U.cpu().numpy().T
    assert info["rel_residual"] <= 1e-12
    # the error of a 1e-12 relative residual is bounded by cond(L_n) * 1e-12; compare loosely first
    assert np.abs(Ug - Ue).max() < 1e-7, np.abs(Ug - Ue).max()
    np.testing.assert_array_equal(Ug[node, lab], 1.0)
    np.testing.assert_allclose(Ug.sum(axis=1), 1.0, atol=1e-8)
    # tighter solve reaches the FP64 gate
    U2, info2 = rw.cg_solve(gg, node, lab, w.C, tol=1e-15, max_iter=20000, raise_on_noconv=False)
    assert np.abs(U2.cpu().numpy().T - Ue).max() < 1e-10


def test_cg_initial_guess_and_noconv():
    need_gpu()
    w = CASES[1][1]
    J, rid, node, lab = setup_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    og = OGraph(J, w.dims, w.conn, w.beta)
    Ue = exact_rw(og, node, lab, w.C, method="direct")
    U0 = to_dev(Ue.T + 1e-3, torch.float64)
    U, info = rw.cg_solve(gg, node, lab, w.C, tol=1e-10, U0=U0)
    assert np.abs(U.cpu().numpy().T - Ue).max() < 1e-8
    _, info = rw.cg_solve(gg, node, lab, w.C, tol=1e-14, max_iter=2, raise_on_noconv=False)
    assert info["status"] == rw.RW_ENOCONV and info["iters"] == 2
