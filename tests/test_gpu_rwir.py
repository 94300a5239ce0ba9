"""GPU parity for the walker driven by priors alone at registration label counts (eq. (5) with no seeds,
eq. (15) in the eigenbasis, hat variables of Sec. II-C; the choice of m of eq. (25)): probabilities and per-voxel
labels against the oracle on the same basis, for FP64, FP32 and BF16 bases (the BF16 labels come from the fused
matrix-core reconstruction, which never forms U), up to the full 21 x 21 x 9 displacement-label grid."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.graph import Graph as OGraph
from oracle.priors import choose_m_prior, g_values, sampled_labels
from oracle.rwir import rwir_labels, rwir_probabilities

from gpu_common import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu

# (name, dims, conn, label extent, m); N = 1353 is not a multiple of 8, C and m are not multiples of 16
CASES = [("2d4", (41, 33), 4, (9, 9), 24), ("2d8", (40, 30), 8, (11, 11), 30), ("3d6", (20, 18, 16), 6, (7, 7, 5), 40)]


def _case(dims, conn, extent, m, config_id=60):
    w = rwsynth.small("rwir", dims, conn, beta=50.0, m=m, C=2, n_shapes=4, intensity="uniform",
                      config_id=config_id)
    J, _ = rwsynth.phantom(w)
    lab = rwsynth.displacement_labels(extent)
    field = rwsynth.displacement_field(w.dims, extent, config_id)
    P = rwsynth.displacement_priors(field, lab)                      # N x C
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, _ = rw.precompute_eig(g, m, tol=1e-10, max_iter=600)
    return w, J, P, g, Q, lam


def _check_labels(Uo, lab, prob, tol):
    """The label chosen is a largest oracle probability up to tol, and prob is the oracle's value there."""
    lab = lab.cpu().numpy()
    prob = prob.double().cpu().numpy()
    rows = np.arange(Uo.shape[0])
    top = Uo.max(axis=1)
    at = Uo[rows, lab]
    assert np.all(at >= top - tol), (at - top).min()
    assert np.abs(prob - at).max() <= tol, np.abs(prob - at).max()
    k, _ = rwir_labels(Uo)
    return float(np.mean(k == lab))


@pytest.mark.parametrize("gamma", [1.0, 0.3])
@pytest.mark.parametrize("name,dims,conn,extent,m", CASES, ids=[c[0] for c in CASES])
def test_fp64_matches_oracle(name, dims, conn, extent, m, gamma):
    need_gpu()
    banner(f"rwir fp64 {name} gamma={gamma}")
    w, J, P, g, Q, lam = _case(dims, conn, extent, m)
    og = OGraph(J, w.dims, w.conn, w.beta)
    Pd = to_dev(P.T, torch.float64)
    U, lab, prob, info = rw.solve_priors(g, Q, lam, Pd, gamma, want_labels=True)
    Uo = rwir_probabilities(og, Q.cpu().numpy().T, lam.cpu().numpy(), P, gamma)
    err = np.abs(U.cpu().numpy().T - Uo).max()
    assert err <= 1e-10, err
    # the labels use the same arithmetic as U: exactly its arg max (first of equal maxima)
    Ug = U.cpu().numpy().T
    np.testing.assert_array_equal(lab.cpu().numpy(), np.argmax(Ug, axis=1))
    np.testing.assert_array_equal(prob.cpu().numpy(), Ug.max(axis=1))
    agree = _check_labels(Uo, lab, prob, 1e-10)
    print(f"  C={P.shape[1]} m={info['m_used']} max|dU|={err:.1e} labels agree {agree:.4f}", flush=True)
    np.testing.assert_allclose(Ug.sum(axis=1), 1.0, atol=1e-10)


@pytest.mark.parametrize("name,dims,conn,extent,m", CASES, ids=[c[0] for c in CASES])
def test_choice_of_m_matches_oracle(name, dims, conn, extent, m):
    need_gpu()
    banner(f"rwir choice of m {name}")
    w, J, P, g, Q, lam = _case(dims, conn, extent, m)
    og = OGraph(J, w.dims, w.conn, w.beta)
    Qn = Q.cpu().numpy().T
    r = 2
    ks = sampled_labels(P.shape[1], r, og.ndim)
    # eps between the thresholds that select m/2 and m/2 - 1, so that the choice sits mid-range
    gw = [g_values(og, Qn, P, ks, mm).max() for mm in (m // 2 - 1, m // 2)]
    scale = og.degree().sum()
    eps = float(np.sqrt(np.sqrt(gw[0] * gw[1]) / scale))
    m_o, gmax_o, g_o = choose_m_prior(og, Qn, P, eps=eps, r=r)
    U, _, _, info = rw.solve_priors(g, Q, lam, to_dev(P.T, torch.float64), 1.0, eps=eps, r=r)
    print(f"  eps={eps:.3e}: m {info['m_used']} (oracle {m_o})", flush=True)
    assert info["m_used"] == m_o
    np.testing.assert_allclose(info["g_max"], gmax_o, rtol=1e-12)
    np.testing.assert_allclose(info["g_worst"], g_o.max(), rtol=1e-8, atol=1e-12 * gmax_o)
    Uo = rwir_probabilities(og, Qn, lam.cpu().numpy(), P, 1.0, m=m_o)
    assert np.abs(U.cpu().numpy().T - Uo).max() <= 1e-10


@pytest.mark.parametrize("name,dims,conn,extent,m", CASES, ids=[c[0] for c in CASES])
def test_fp32_matches_oracle(name, dims, conn, extent, m):
    need_gpu()
    banner(f"rwir fp32 {name}")
    w, J, P, g64, Q, lam = _case(dims, conn, extent, m)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Q32 = Q.float()
    og = OGraph(J, w.dims, w.conn, w.beta)
    P32 = P.astype(np.float32)
    U, lab, prob, _ = rw.solve_priors(g, Q32, lam, to_dev(P32.T, torch.float32), 1.0, want_labels=True)
    Uo = rwir_probabilities(og, Q32.double().cpu().numpy().T, lam.cpu().numpy(), P32.astype(np.float64), 1.0)
    err = np.abs(U.double().cpu().numpy().T - Uo).max()
    assert err <= 1e-4, err
    agree = _check_labels(Uo, lab, prob, 1e-4)
    print(f"  max|dU|={err:.1e} labels agree {agree:.4f}", flush=True)


@pytest.mark.parametrize("pdt", [torch.bfloat16, torch.float32], ids=["pbf16", "pf32"])
@pytest.mark.parametrize("name,dims,conn,extent,m", CASES, ids=[c[0] for c in CASES])
def test_bf16_matches_oracle(name, dims, conn, extent, m, pdt):
    need_gpu()
    banner(f"rwir bf16 {name} priors {pdt}")
    w, J, P, g64, Q, lam = _case(dims, conn, extent, m)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Qb = rw.convert_block(Q.float(), torch.bfloat16)
    og = OGraph(J, w.dims, w.conn, w.beta)
    Pd = to_dev(P.T, torch.float32).to(pdt).contiguous()
    Pin = Pd.double().cpu().numpy().T                       # the priors as the call receives them
    U, lab, prob, _ = rw.solve_priors(g, Qb, lam, Pd, 1.0, want_labels=True)
    Uo = rwir_probabilities(og, Qb.double().cpu().numpy().T, lam.cpu().numpy(), Pin, 1.0)
    err = np.abs(U.double().cpu().numpy().T - Uo).max()
    assert err <= 1e-2, err
    agree = _check_labels(Uo, lab, prob, 1e-2)
    # the fused labels pick a largest value of the U the same call reconstructs, up to the BF16 rounding
    Ug = U.double().cpu().numpy().T
    at = Ug[np.arange(Ug.shape[0]), lab.cpu().numpy()]
    assert np.all(at >= Ug.max(axis=1) - 1e-2)
    print(f"  max|dU|={err:.1e} labels agree with the oracle's arg max {agree:.4f}", flush=True)


@pytest.mark.parametrize("qdt", [torch.bfloat16, torch.float32], ids=["bf16", "fp32"])
def test_full_displacement_grid(qdt):
    """C = 21 x 21 x 9 = 3969 labels on a 24 x 24 x 20 volume, m = 60."""
    need_gpu()
    banner(f"rwir full label grid {qdt}")
    extent = rwsynth.CFG6_EXTENT
    w, J, P, g64, Q, lam = _case((24, 24, 20), 6, extent, 60, config_id=61)
    g = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Qc = rw.convert_block(Q.float(), torch.bfloat16) if qdt == torch.bfloat16 else Q.float()
    pdt = torch.bfloat16 if qdt == torch.bfloat16 else torch.float32
    Pd = to_dev(P.T, torch.float32).to(pdt).contiguous()
    og = OGraph(J, w.dims, w.conn, w.beta)
    U, lab, prob, _ = rw.solve_priors(g, Qc, lam, Pd, rwsynth.CFG6_GAMMA, want_labels=True)
    Uo = rwir_probabilities(og, Qc.double().cpu().numpy().T, lam.cpu().numpy(), Pd.double().cpu().numpy().T,
                            rwsynth.CFG6_GAMMA)
    tol = 1e-2 if qdt == torch.bfloat16 else 1e-4
    err = np.abs(U.double().cpu().numpy().T - Uo).max()
    assert err <= tol, err
    agree = _check_labels(Uo, lab, prob, tol)
    print(f"  C={P.shape[1]} max|dU|={err:.1e} labels agree {agree:.4f}", flush=True)
    # labels only (the path that never forms U) give the same labels
    _, lab2, prob2, _ = rw.solve_priors(g, Qc, lam, Pd, rwsynth.CFG6_GAMMA, want_U=False, want_labels=True)
    assert torch.equal(lab, lab2) and torch.equal(prob, prob2)


def test_invalid_arguments():
    need_gpu()
    w, J, P, g, Q, lam = _case((20, 18), 4, (5, 5), 12)
    Pd = to_dev(P.T, torch.float64)
    with pytest.raises(rw.RWError):
        rw.solve_priors(g, Q, lam, Pd, 0.0)                                  # gamma must be > 0
    with pytest.raises(rw.RWError):
        rw.solve_priors(g, Q, lam, Pd, 1.0, want_U=False)                    # nothing asked for
    with pytest.raises(rw.RWError):
        rw.solve_priors(g, rw.convert_block(Q.float(), torch.bfloat16), lam, Pd, 1.0)   # FP64 priors, BF16 basis
