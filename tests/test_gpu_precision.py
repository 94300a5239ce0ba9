"""GPU parity for the precision form: BF16 matrix-core contractions with the eigenbasis, and the FP32 /
BF16 paths against the FP64 path on the same (upcast or rounded) basis."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.eigen import certify, principal_angle_sines
from oracle.fast_rw import fast_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, dev, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64 (test-side reference of the storage)."""
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("N,m,C", [(1000, 37, 3), (1001, 16, 8), (4096, 100, 4), (777, 5, 1)])
def test_project_basis_bf16_matches_reference(N, m, C):
    need_gpu()
    banner(f"project N={N} m={m} C={C}")
    rng = np.random.default_rng(N + m)
    Q = rng.standard_normal((m, N)) / np.sqrt(N)
    X = rng.uniform(0, 1, (C, N)).astype(np.float32)
    Qb = to_dev(Q, torch.float32).to(torch.bfloat16)
    P = rw.project_basis(Qb, to_dev(X, torch.float32)).cpu().numpy()          # (C, m)
    ref = (bf16_round(Q) @ X.astype(np.float64).T).T                         # same BF16 basis, exact X
    scale = np.abs(bf16_round(Q)) @ np.abs(X.astype(np.float64)).T
    # X keeps ~16 bits through its two BF16 parts; FP32 accumulation over N terms
    assert np.all(np.abs(P - ref) <= 1e-5 * scale.T + 1e-12), np.abs(P - ref).max()
    P32 = rw.project_basis(to_dev(Q, torch.float32), to_dev(X, torch.float32)).cpu().numpy()
    ref32 = (Q.astype(np.float32).astype(np.float64) @ X.astype(np.float64).T).T
    np.testing.assert_allclose(P32, ref32, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dims,conn,C,m", [((30, 26), 8, 3, 45), ((31, 29), 4, 8, 33), ((12, 11, 9), 6, 4, 40)])
def test_reconstruction_bf16_matrix_cores(dims, conn, C, m):
    """BF16 basis through the matrix cores against the oracle on the same rounded basis (1e-2 gate) and
    against the FP32 VALU path on that basis (the difference is the BF16 rounding of Y only)."""
    need_gpu()
    banner(f"reconstruct bf16 {dims} C={C}")
    w = rwsynth.small("p", dims, conn, m=m, C=C, seeds_per_label=4, n_shapes=5)
    J, rid, node, lab = setup_case(w)
    g64 = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, info = rw.precompute_eig(g64, m, tol=1e-10)
    g32 = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    Qb = rw.convert_block(Q, torch.bfloat16)
    Ub, _ = rw.solve_seeds(g32, Qb, lam, node, lab, C)
    Qb64 = Qb.to(torch.float64)
    U32, _ = rw.solve_seeds(g32, Qb64.to(torch.float32), lam, node, lab, C)      # VALU path, same values
    og = OGraph(J, w.dims, w.conn, w.beta)
    Uo = fast_rw(og, Qb64.cpu().numpy().T, lam.cpu().numpy(), node, lab, C, exact=True)
    err = np.abs(Ub.cpu().numpy().T.astype(np.float64) - Uo).max()
    assert err <= 1e-2, err
    assert (Ub - U32).abs().max().item() <= 1e-3
    np.testing.assert_array_equal(Ub.cpu().numpy().T[node, lab], 1.0)


def test_mixed_precision_against_fp64_path():
    """3D phantom (6-connected, beta 120, intensities uniform in [0, 1]): FP32 eigensolver vs FP64
    eigensolver per eigenpair, and probability maps from the FP64 basis evaluated in FP64, FP32 and BF16."""
    need_gpu()
    banner("mixed precision 3D")
    w = rwsynth.Workload("mixed_small", 3, (28, 26, 24), 6, 120.0, 40, 4, 30, 0.03, 8, "uniform", 0.0, "mixed")
    J, rid, node, lab = setup_case(w)
    Jd = to_dev(J, torch.float64)
    g64 = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float64)
    g32 = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float32)
    Q64, lam64, i64 = rw.precompute_eig(g64, w.m, tol=1e-10, max_iter=400)
    Q32, lam32, i32 = rw.precompute_eig(g32, w.m, tol=1e-5, max_iter=400)
    og = OGraph(J, w.dims, w.conn, w.beta)
    res, orth = certify(og, Q32.to(torch.float64).cpu().numpy().T, lam32.cpu().numpy())
    assert res.max() < 5e-5 and orth < 5e-6
    dl = np.abs(lam32.cpu().numpy() - lam64.cpu().numpy())
    assert dl.max() < 1e-4, dl.max()
    ev = lam64.cpu().numpy()
    mp = max([k for k in range(2, w.m) if ev[k] - ev[k - 1] > 1e-3] + [2])
    sines = principal_angle_sines(Q32.to(torch.float64).cpu().numpy().T[:, :mp], Q64.cpu().numpy().T[:, :mp])
    assert sines.max() < 1e-2, sines.max()
    U64, _ = rw.solve_seeds(g64, Q64, lam64, node, lab, w.C)
    U32, _ = rw.solve_seeds(g32, Q64.to(torch.float32), lam64, node, lab, w.C)
    Ub, _ = rw.solve_seeds(g32, rw.convert_block(Q64, torch.bfloat16), lam64, node, lab, w.C)
    e32 = (U32.double() - U64).abs().max().item()
    e16 = (Ub.double() - U64).abs().max().item()
    assert e32 <= 1e-4, e32
    assert e16 <= 1e-2, e16


@pytest.mark.parametrize("dims,conn,C,m", [((30, 26), 8, 3, 45), ((12, 11, 9), 6, 4, 40), ((31, 29), 4, 10, 33),
                                           ((20, 18), 4, 2, 6)])
def test_pair_form_against_oracle_and_fp64_path(dims, conn, C, m):
    """The BF16 pair form: its plain block equals rw_convert_block's BF16 copy and its remainder columns
    hold q_j - hi_j to BF16 (zero beyond m - 1); the solve matches the oracle on the basis the pair
    represents (hi + lo) at 1e-4, through the matrix cores (C <= 8) and the vector units (C = 10); against
    the FP64 path its error is below the plain BF16 copy's."""
    need_gpu()
    banner(f"pair form {dims} conn={conn} C={C} m={m}")
    w = rwsynth.small("pp", dims, conn, m=m, C=C, seeds_per_label=4, n_shapes=5)
    J, rid, node, lab = setup_case(w)
    g64 = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, _ = rw.precompute_eig(g64, m, tol=1e-10)
    g32 = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float32)
    P = rw.to_pair(Q)
    Qb = rw.convert_block(Q, torch.bfloat16)
    assert torch.equal(P.plain(), Qb)
    lo = P.data[:rw.RW_PAIR_COLS].double()
    k = min(rw.RW_PAIR_COLS, m - 1)
    ref_lo = (Q[1:1 + k] - Qb[1:1 + k].double()).float().to(torch.bfloat16).double()
    assert torch.equal(lo[:k], ref_lo) and torch.all(lo[k:] == 0)
    Qv = P.value()
    assert (Qv[1:1 + k] - Q[1:1 + k]).abs().max().item() <= 2.0 ** -15 * Q[1:1 + k].abs().max().item()
    Up, _ = rw.solve_seeds(g32, P, lam, node, lab, C)
    og = OGraph(J, w.dims, w.conn, w.beta)
    Uo = fast_rw(og, Qv.cpu().numpy().T, lam.cpu().numpy(), node, lab, C, exact=True)
    err_o = np.abs(Up.cpu().numpy().T.astype(np.float64) - Uo).max()
    U64, _ = rw.solve_seeds(g64, Q, lam, node, lab, C)
    Ub, _ = rw.solve_seeds(g32, Qb, lam, node, lab, C)
    e_pair = (Up.double() - U64).abs().max().item()
    e_bf16 = (Ub.double() - U64).abs().max().item()
    print(f"  vs oracle on the pair's basis {err_o:.2e}; vs FP64 path: pair {e_pair:.2e}, plain BF16 {e_bf16:.2e}",
          flush=True)
    assert err_o <= 1e-4, err_o
    assert e_pair <= 1e-2 and e_pair <= e_bf16, (e_pair, e_bf16)
    np.testing.assert_array_equal(Up.cpu().numpy().T[node, lab], 1.0)
