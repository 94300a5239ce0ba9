"""GPU tests of the asynchronous solve (rw_solve_seeds_async) and of the capture guard on the synchronous
entry points: the asynchronous call gives the same bits as rw_solve_seeds at the same m; captured into a HIP
graph it is replayed with other seed contents, with eager work and synchronizations between the replays, and
every replay is checked; its device status word reports what rw_solve_seeds reports as an error; a
synchronous call made under capture is refused with RW_ECAPTURE before it enqueues anything."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth

from gpu_common import banner, dev, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu


def _case(gdt, qdt, dims=(40, 33), conn=4, m=20, C=3):
    w = rwsynth.small("as", dims, conn, m=m, C=C, seeds_per_label=5, n_shapes=3)
    J, rid, node, lab = setup_case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=gdt)
    Q, lam, _ = rw.precompute_eig(g, m, tol=1e-10 if gdt == torch.float64 else 1e-5, max_iter=400)
    if qdt != Q.dtype:
        Q = rw.convert_block(Q, qdt)
    g.components()
    return w, rid, g, Q, lam


def _async(g, Q, lam, node, lab, C, work=None):
    S = len(node)
    if work is None:
        work = torch.empty(rw.solve_workspace_bytes(g, Q.shape[0], S, C), dtype=torch.uint8, device=dev())
    U = torch.empty((C, g.N), dtype=g.dtype, device=dev())
    status = torch.full((1,), 99, dtype=torch.int32, device=dev())
    rw.solve_seeds_async(g, Q, lam, torch.as_tensor(np.asarray(node, np.int64)).to(dev()),
                         torch.as_tensor(np.asarray(lab, np.int32)).to(dev()), C, U, work, status)
    return U, int(status.item())


@pytest.mark.parametrize("gdt,qdt", [(torch.float64, torch.float64), (torch.float32, torch.float32),
                                     (torch.float32, torch.bfloat16)], ids=["f64", "f32", "bf16"])
def test_async_equals_sync(gdt, qdt):
    need_gpu()
    banner(f"async eager {gdt} {qdt}")
    w, rid, g, Q, lam = _case(gdt, qdt)
    node, lab = rwsynth.seeds(w, rid, 0)
    Us, info = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    assert info["m_used"] == w.m
    Ua, st = _async(g, Q, lam, node, lab, w.C)
    assert st == rw.RW_OK
    assert torch.equal(Ua, Us), (Ua.double() - Us.double()).abs().max().item()


def test_async_graph_replays_with_new_seeds():
    need_gpu()
    banner("async capture and replay")
    w, rid, g, Q, lam = _case(torch.float32, torch.float32, dims=(48, 41), m=24)
    rounds = [rwsynth.seeds(w, rid, 0, per_label=6, stream_offset=r) for r in range(5)]
    S = max(len(r[0]) for r in rounds)
    # every round is padded to S seeds with extra seeds of its own labels, so the graph's shapes stay fixed
    padded = []
    for r, (node, lab) in enumerate(rounds):
        rng = np.random.default_rng(700 + r)
        free = np.setdiff1d(np.arange(w.N), node)
        extra = np.sort(rng.choice(free, size=S - len(node), replace=False))
        lab_map = rwsynth.label_map(rid, w.C)
        n2 = np.concatenate([node, extra])
        l2 = np.concatenate([lab, lab_map[extra].astype(np.int32)])
        o = np.argsort(n2)
        padded.append((n2[o], l2[o]))
    d_node = torch.empty(S, dtype=torch.int64, device=dev())
    d_lab = torch.empty(S, dtype=torch.int32, device=dev())
    U = torch.empty((w.C, g.N), dtype=g.dtype, device=dev())
    work = torch.empty(rw.solve_workspace_bytes(g, w.m, S, w.C), dtype=torch.uint8, device=dev())
    status = torch.full((1,), 99, dtype=torch.int32, device=dev())
    d_node.copy_(torch.as_tensor(padded[0][0]))
    d_lab.copy_(torch.as_tensor(padded[0][1]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                          # warm-up on the capture's side stream
        rw.solve_seeds_async(g, Q, lam, d_node, d_lab, w.C, U, work, status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rw.solve_seeds_async(g, Q, lam, d_node, d_lab, w.C, U, work, status)
    for r, (node, lab) in enumerate(padded):
        d_node.copy_(torch.as_tensor(node))
        d_lab.copy_(torch.as_tensor(lab))
        status.fill_(99)
        graph.replay()
        junk = torch.randn(1 << 20, device=dev()).sum()        # unrelated eager work between replays
        torch.cuda.synchronize()
        ref, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C, m_avail=w.m)
        torch.cuda.synchronize()
        assert int(status.item()) == rw.RW_OK, r
        assert torch.equal(U, ref), (r, (U - ref).abs().max().item())
        del junk


def test_async_status_word_matches_sync_errors():
    need_gpu()
    banner("async status codes")
    w, rid, g, Q, lam = _case(torch.float64, torch.float64, dims=(30, 26), m=12, C=2)
    node, lab = rwsynth.seeds(w, rid, 0)
    # invalid seeds: out-of-range node, out-of-range label, not ascending, repeated node
    bad_sets = []
    n2 = node.copy(); n2[-1] = w.N; bad_sets.append((n2, lab))
    l2 = lab.copy(); l2[0] = w.C; bad_sets.append((node, l2))
    n3 = node.copy(); n3[[0, 1]] = n3[[1, 0]]; bad_sets.append((n3, lab))
    n4 = node.copy(); n4[1] = n4[0]; l4 = lab.copy(); l4[1] = l4[0]; bad_sets.append((n4, l4))
    for nb, lb in bad_sets:
        U, st = _async(g, Q, lam, nb, lb, w.C)
        assert st == rw.RW_EINVAL
    # the same solve is fine afterwards (the flags start from zero on every call)
    U, st = _async(g, Q, lam, node, lab, w.C)
    assert st == rw.RW_OK
    # a component without a seed: two halves joined by weights below 1e-30 (exp(-90) at a unit step)
    Jh = np.zeros((26, 30))
    Jh[:, 15:] = 1.0
    gh = rw.Graph(to_dev(Jh.reshape(-1), torch.float64), (30, 26, 1), 4, 90.0, dtype=torch.float64)
    gh.components()
    rng = np.random.default_rng(5)
    Qh = torch.as_tensor(np.linalg.qr(rng.standard_normal((gh.N, 6)))[0].T.copy()).to(dev())
    lamh = torch.arange(6, dtype=torch.float64, device=dev()) * 0.1
    left = np.array([30 * 3 + 2, 30 * 20 + 4], np.int64)                 # both seeds in the left half
    with pytest.raises(rw.RWError) as ei:
        rw.solve_seeds(gh, Qh, lamh, left, np.array([0, 1], np.int32), 2)
    assert ei.value.status == rw.RW_EUNANCHORED
    assert _async(gh, Qh, lamh, left, np.array([0, 1], np.int32), 2)[1] == rw.RW_EUNANCHORED
    # a singular reduced system: two equal basis columns with both eigenvalues set to 0 give two equal columns of
    # Lambda - Q_s^T B Q_n (the elimination leaves a pivot of rounding size in the second)
    Qs = Q.clone()
    Qs[3] = Qs[2]
    lams = lam.clone()
    lams[2] = 0.0
    lams[3] = 0.0
    with pytest.raises(rw.RWError) as ei:
        rw.solve_seeds(g, Qs, lams, node, lab, w.C)
    assert ei.value.status == rw.RW_ESINGULAR
    assert _async(g, Qs, lams, node, lab, w.C)[1] == rw.RW_ESINGULAR
    # a workspace too small, and components not current (after an edit): refused by the call itself
    work = torch.empty(1024, dtype=torch.uint8, device=dev())
    with pytest.raises(rw.RWError) as ei:
        _async(g, Q, lam, node, lab, w.C, work=work)
    assert ei.value.status == rw.RW_EWORKSPACE
    rw.edit_graph(g, [rwsynth.Edit("scale_box", 0.5, (2, 3, 0), (9, 11, 1))])
    with pytest.raises(rw.RWError) as ei:
        _async(g, Q, lam, node, lab, w.C)
    assert ei.value.status == rw.RW_EINVAL and "components" in str(ei.value)


def test_sync_entry_points_refuse_capture():
    need_gpu()
    banner("capture guard")
    w, rid, g, Q, lam = _case(torch.float32, torch.float32, dims=(24, 20), m=10, C=2)
    node, lab = rwsynth.seeds(w, rid, 0)
    U0, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    U = torch.empty_like(U0)
    ws = rw.SolveWorkspace()
    ws.get(rw.solve_workspace_bytes(g, w.m, len(node), w.C) * 4, g.device)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    errs = []
    with torch.cuda.graph(graph):
        U.zero_()                                          # the graph holds this fill and nothing of the library
        for call in (lambda: rw.solve_seeds(g, Q, lam, node, lab, w.C, U=U, workspace=ws), g.components):
            try:
                call()
            except rw.RWError as e:
                errs.append(e.status)
    assert errs == [rw.RW_ECAPTURE, rw.RW_ECAPTURE]
    assert "capture" in rw.lib().rw_last_error().decode()
    torch.cuda.synchronize()
    # nothing was enqueued by the refused calls, and the library still works afterwards
    U1, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    assert torch.equal(U1, U0)
