"""GPU parity at the full workload sizes, in the configuration bench.py runs: the 64 x 64 FP64 case in full
against the oracle, the 512 x 512 interactive case on sampled rows and by certification, the 128^3 and 96^3
volumes by properties that hold at any size, and the batched workload image by image against the single
solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.choose_m import choose_m, f_values
from oracle.eigen import certify, dense_eigpairs, principal_angle_sines
from oracle.exact_rw import exact_rw, seed_split
from oracle.fast_rw import fast_rw
from oracle.graph import Graph as OGraph
from oracle.update import rayleigh_ritz

from gpu_common import banner, dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _case(w, seed=0):
    J, rid = rwsynth.phantom(w, seed)
    node, lab = rwsynth.seeds(w, rid, seed)
    return J, rid, node, lab


def test_small64_full_against_oracle():
    """64 x 64, 4-connected, FP64, m = 50: eigenpairs against a dense eigendecomposition, exact RW by CG
    against a direct solve, and the eigenbasis solve against the oracle on the same basis."""
    need_gpu()
    w = rwsynth.CFG1
    banner(f"full size {w.name}")
    J, rid, node, lab = _case(w)
    og = OGraph(J, w.dims, w.conn, w.beta)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, info = rw.precompute_eig(g, w.m, tol=1e-10, max_iter=400)
    lam_o, Q_o = dense_eigpairs(og, w.m)
    Qn, ln = Q.cpu().numpy().T, lam.cpu().numpy()
    np.testing.assert_allclose(ln, lam_o, atol=1e-9)
    res, orth = certify(og, Qn, ln)
    assert res.max() <= 1e-9 and orth <= 1e-12
    gaps = np.diff(lam_o)
    mp = max([k for k in range(2, w.m) if gaps[k - 1] > 1e-6] + [2])
    assert principal_angle_sines(Qn[:, :mp], Q_o[:, :mp]).max() < 1e-6
    Ucg, cinfo = rw.cg_solve(g, node, lab, w.C, tol=1e-13)
    Ud = exact_rw(og, node, lab, w.C, method="direct")
    assert np.abs(Ucg.cpu().numpy().T - Ud).max() < 1e-10
    U, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    Uf = fast_rw(og, Qn, ln, node, lab, w.C, exact=bool(np.min(np.abs(ln[1:])) < 1e-6))
    assert np.abs(U.cpu().numpy().T - Uf).max() <= 1e-10


@pytest.fixture(scope="module")
def interactive512():
    need_gpu()
    w = rwsynth.CFG2
    J, rid, node, lab = _case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q, lam, info = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
    return w, J, node, lab, g, Q, lam, info


def test_interactive512_certified_and_sampled_rows(interactive512):
    """512 x 512, 8-connected, FP32, m = 200, in the bench's configuration: the eigenpairs certified on the
    CPU in FP64, the choice of m (eps = 0.1) against the oracle's linear scan, and 3000 sampled rows of the
    solve against the oracle's fast RW on the same (upcast) basis."""
    w, J, node, lab, g, Q, lam, info = interactive512
    banner("full size interactive512")
    og = OGraph(J, w.dims, w.conn, w.beta)
    Qn, ln = Q.to(torch.float64).cpu().numpy().T, lam.cpu().numpy()
    res, orth = certify(og, Qn, ln)
    assert res.max() <= 3e-5 + 2e-6 and orth <= 1e-5, (res.max(), orth)
    # independent FP64 spectrum (shift-invert Lanczos) for the lowest 20 pairs
    ev = spla.eigsh(og.Lhat(), k=20, sigma=-1e-3, which="LM", return_eigenvectors=False)
    np.testing.assert_allclose(np.sort(ev), ln[:20], atol=5e-5)
    U, inf = rw.solve_seeds(g, Q, lam, node, lab, w.C, eps=0.1)
    m_o, fmax, f = choose_m(og, Qn, node, lab, w.C, eps=0.1)
    if inf["m_used"] != m_o:
        fa = f_values(og, Qn, node, lab, w.C, inf["m_used"]).max()
        fb = f_values(og, Qn, node, lab, w.C, m_o).max()
        assert min(abs(fa - fmax), abs(fb - fmax)) <= 1e-6 * fmax, (inf, m_o)
    rows = np.random.default_rng(7).choice(w.N, 3000, replace=False)
    Uo = fast_rw(og, Qn, ln, node, lab, w.C, m=inf["m_used"], rows=rows)
    err = np.abs(U.cpu().numpy().T[rows].astype(np.float64) - Uo).max()
    assert err <= 1e-4, err
    np.testing.assert_allclose(U.sum(0).cpu().numpy(), 1.0, atol=1e-4)


def test_interactive512_edits_and_rayleigh_ritz(interactive512):
    """The bench's three edits in order: graph mask bit-exact, Rayleigh-Ritz eigenvalues against the oracle's
    dense Rayleigh-Ritz on the same (upcast) basis."""
    w, J, node, lab, g0, Q0, lam0, _ = interactive512
    banner("full size interactive512 edits")
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q, lam = Q0.clone(), lam0.clone()
    og = OGraph(J, w.dims, w.conn, w.beta)
    for e in rwsynth.cfg2_edits(w, 0):
        Qin = Q.to(torch.float64).cpu().numpy().T
        rw.update_eig(g, [e], Q, lam, mode=rw.RW_UPDATE_RR)
        og.apply_edit(e)
        np.testing.assert_array_equal(g.view()["mask"].cpu().numpy(), og.mask_bits())
        _, lam_o = rayleigh_ritz(og, Qin)
        np.testing.assert_allclose(lam.cpu().numpy(), lam_o, atol=2e-6, rtol=1e-5)


def test_volume128_properties():
    """128^3, 6-connected, FP32 basis and its BF16 copy: at this size the checks are properties (sampled
    eigenpair certification, rows summing to one, one-hot seeds, probabilities bounded)."""
    need_gpu()
    w = rwsynth.CFG3
    banner(f"full size {w.name}")
    J, rid, node, lab = _case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q, lam, info = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
    og = OGraph(J, w.dims, w.conn, w.beta)
    cols = np.array([0, 1, 2, 17, 50, 99])
    Qs = Q[torch.as_tensor(cols, device=dev())].to(torch.float64).cpu().numpy().T
    r = og.Lhat() @ Qs - Qs * lam.cpu().numpy()[cols]
    assert np.linalg.norm(r, axis=0).max() <= 3e-5 + 2e-6
    for qd in (torch.float32, torch.bfloat16):
        Qd = Q if qd == torch.float32 else rw.convert_block(Q, torch.bfloat16)
        U, _ = rw.solve_seeds(g, Qd, lam, node, lab, w.C)
        Un = U.to(torch.float64).cpu().numpy()
        np.testing.assert_allclose(Un.sum(0), 1.0, atol=1e-4 if qd == torch.float32 else 1e-2)
        np.testing.assert_array_equal(Un.T[node, lab], 1.0)


def test_grad96_forward_residual():
    """96^3, 6-connected, FP64 exact RW (the differentiation form's forward) warm-started from the
    eigenbasis: the oracle's sparse operator gives the relative residual of every label's system."""
    need_gpu()
    w = rwsynth.CFG5
    banner(f"full size {w.name}")
    J, rid, node, lab = _case(w)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-8, max_iter=600)
    U0, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C)
    U, cinfo = rw.cg_solve(g, node, lab, w.C, tol=1e-12, U0=U0)
    og = OGraph(J, w.dims, w.conn, w.beta)
    L = og.L().tocsr()
    s, n = seed_split(og.N, node)
    Un = U.cpu().numpy().T
    Ln, B = L[n][:, n], L[n][:, s]
    for c in range(w.C):
        rhs = -(B @ Un[s, c])
        rr = np.linalg.norm(Ln @ Un[n, c] - rhs) / np.linalg.norm(rhs)
        assert rr <= 1e-10, (c, rr)
    assert np.all(Un >= -1e-10) and np.all(Un <= 1 + 1e-10)
    np.testing.assert_allclose(Un.sum(1), 1.0, atol=1e-10)


def test_batch64_images_match_single_solves():
    """The batched workload (first 8 of its 64 images, sides up to 768, m in {50, 100, 200}) in the bench's
    launch configuration (autotuned tiles, HIP-graph replays): each image against the single-image solve."""
    need_gpu()
    banner("full size batch64 (8 images)")
    imgs = rwsynth.cfg4_images(64, 0)[:8]
    images = []
    for w in imgs:
        J, rid = rwsynth.phantom(w, 0)
        gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
        Q, lam, _ = rw.precompute_eig(gg, w.m, tol=1e-5, max_iter=400)
        rnds = [rwsynth.cfg4_round(w, rid, r, 0) for r in range(3)]
        images.append({"graph": gg, "Q": Q, "lam": lam, "rounds": rnds, "C_cap": 4,
                       "S_cap": max(len(x[1]) for x in rnds)})
    bs = rw.BatchSolver(images, use_graph=True)
    for r in range(3):
        bs.set_seeds([im["rounds"][r] for im in images])
        bs.run()
        torch.cuda.synchronize()
        for im, Ub in zip(images, bs.outputs()):
            C, node, lab = im["rounds"][r]
            Us, inf = rw.solve_seeds(im["graph"], im["Q"], im["lam"], node, lab, C)
            # different LU kernels for the reduced system: rounding amplified by its conditioning
            assert (Ub - Us).abs().max().item() <= max(1e-5, 1e-11 / max(inf["min_pivot"], 1e-300))
