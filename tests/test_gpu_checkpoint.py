"""GPU tests of the offline-phase checkpoint (rw_eig_save / rw_eig_load): the eigenpairs come back bit for
bit, the solve from a loaded basis equals the solve from the original, and a file is refused for a graph
whose operator differs (another beta, an edit, another grid) or when it is truncated."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_checkpoint_round_trip_and_refusals(dt, tmp_path):
    need_gpu()
    banner(f"checkpoint {dt}")
    w = rwsynth.small("ck", (30, 27), 8, m=24, C=3, seeds_per_label=4, n_shapes=3)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=dt)
    Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-10 if dt == torch.float64 else 1e-5, max_iter=400)
    path = str(tmp_path / "basis.rweig")
    rw.eig_save(g, path, Q, lam, tol=1e-5)
    hd = rw.eig_read_header(path)
    assert hd["dims"] == w.dims and hd["m"] == w.m and hd["conn"] == w.conn and hd["beta"] == w.beta
    Q2, lam2, hd2 = rw.eig_load(g, path)
    assert torch.equal(Q2, Q) and torch.equal(lam2, lam) and hd2 == hd
    # a fresh graph of the same image and beta has the same operator: accepted
    g_same = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=dt)
    Q3, lam3, _ = rw.eig_load(g_same, path, m=10)
    assert torch.equal(Q3, Q[:10]) and torch.equal(lam3, lam[:10])
    U1, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    U2, _ = rw.solve_seeds(g_same, Q2, lam2, node, lab, w.C)
    assert torch.equal(U1, U2)
    # another beta, an edit, another grid, another dtype, more pairs than stored, a truncated file
    for bad in (rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta * 1.5, dtype=dt),):
        with pytest.raises(rw.RWError) as ei:
            rw.eig_load(bad, path)
        assert ei.value.status == rw.RW_EINVAL
    rw.edit_graph(g_same, [rwsynth.Edit("scale_box", 0.5, (2, 3, 0), (9, 11, 1))])
    with pytest.raises(rw.RWError):
        rw.eig_load(g_same, path)
    w2 = rwsynth.small("ck2", (27, 30), 8, m=24, C=3)
    J2, _, _, _ = setup_case(w2)
    g2 = rw.Graph(to_dev(J2, torch.float64), w2.dims, w2.conn, w2.beta, dtype=dt)
    with pytest.raises(rw.RWError):
        rw.eig_load(g2, path)
    other = torch.bfloat16 if dt == torch.float32 else torch.float32
    with pytest.raises(rw.RWError):
        rw.lib()  # the binding reads the stored type; ask the C entry point for another one directly
        lamx = torch.empty(w.m, dtype=torch.float64, device=Q.device)
        Qx = torch.empty((w.m, w.N), dtype=other, device=Q.device)
        rw._check(rw.lib().rw_eig_load(g.handle, path.encode(), rw._ptr(Qx), rw._TORCH_DT[other], rw._ptr(lamx), w.m,
                                       rw._stream(g.device), None))
    with pytest.raises(rw.RWError):
        lamx = torch.empty(w.m + 1, dtype=torch.float64, device=Q.device)
        Qx = torch.empty((w.m + 1, w.N), dtype=dt, device=Q.device)
        rw._check(rw.lib().rw_eig_load(g.handle, path.encode(), rw._ptr(Qx), rw._TORCH_DT[dt], rw._ptr(lamx), w.m + 1,
                                       rw._stream(g.device), None))
    data = open(path, "rb").read()
    short = str(tmp_path / "short.rweig")
    open(short, "wb").write(data[: len(data) - 16])
    with pytest.raises(rw.RWError):
        rw.eig_load(g, short)


def test_checkpoint_pair_form(tmp_path):
    """The pair form round-trips bit for bit, a prefix of it loads as the pair form of fewer pairs, and the
    solve from the loaded pairs equals the solve from the original."""
    need_gpu()
    banner("checkpoint pair form")
    w = rwsynth.small("ckp", (26, 24), 4, m=20, C=2, seeds_per_label=4, n_shapes=3)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
    P = rw.to_pair(Q)
    path = str(tmp_path / "pair.rweig")
    rw.eig_save(g, path, P, lam)
    assert rw.eig_read_header(path)["q_dtype"] == rw.RW_BF16_PAIR
    P2, lam2, _ = rw.eig_load(g, path)
    assert isinstance(P2, rw.PairBasis) and torch.equal(P2.data, P.data) and torch.equal(lam2, lam)
    P3, lam3, _ = rw.eig_load(g, path, m=12)
    assert torch.equal(P3.data, P.data[:rw.RW_PAIR_COLS + 12]) and torch.equal(lam3, lam[:12])
    U1, _ = rw.solve_seeds(g, P, lam, node, lab, w.C)
    U2, _ = rw.solve_seeds(g, P2, lam2, node, lab, w.C)
    assert torch.equal(U1, U2)
