"""GPU parity: the online eigenbasis solve and the choice of m against the oracle, on the same basis."""
import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.choose_m import choose_m, f_values
from oracle.eigen import dense_eigpairs
from oracle.exact_rw import exact_rw
from oracle.fast_rw import fast_rw
from oracle.graph import Graph as OGraph

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu

# (name, workload, graph dtype, Q dtype, tolerance, tolerance kind)
CASES = [
    ("2d4_f64", rwsynth.small("s1", (23, 19), 4, m=40, C=3, seeds_per_label=4, n_shapes=3), torch.float64,
     torch.float64, 1e-10, "rel"),
    ("2d8_f64_m", rwsynth.small("s2", (20, 21), 8, m=60, C=2, seeds_per_label=30, n_shapes=3), torch.float64,
     torch.float64, 1e-10, "rel"),
    ("3d6_f64", rwsynth.small("s3", (8, 9, 7), 6, m=30, C=4, seeds_per_label=3, n_shapes=4), torch.float64,
     torch.float64, 1e-10, "rel"),
    ("2d8_f32", rwsynth.small("s4", (30, 26), 8, m=45, C=3, seeds_per_label=5, n_shapes=4), torch.float32,
     torch.float32, 1e-4, "abs"),
    ("2d4_bf16", rwsynth.small("s5", (26, 30), 4, m=45, C=2, seeds_per_label=5, n_shapes=3), torch.float32,
     torch.bfloat16, 1e-2, "abs"),
]


def _oracle_case(w):
    J, rid, node, lab = setup_case(w)
    og = OGraph(J, w.dims, w.conn, w.beta)
    lam, Q = dense_eigpairs(og, w.m)
    return J, node, lab, og, lam, Q


def _needs_exact(lam):
    """The oracle's FP64 bordered system divides by the non-null eigenvalues; below 1e-6 its own
    rounding exceeds the FP64 gate, so the oracle evaluates that system in extended precision instead."""
    return np.min(np.abs(lam[1:])) < 1e-6


@pytest.mark.parametrize("name,w,gdt,qdt,tol,kind", CASES, ids=[c[0] for c in CASES])
def test_solve_matches_oracle(name, w, gdt, qdt, tol, kind):
    need_gpu()
    banner(f"solve {name}")
    J, node, lab, og, lam, Q = _oracle_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=gdt)
    Qd = to_dev(Q.T, qdt)                          # (m, N): column-major N x m
    lamd = to_dev(lam, torch.float64)
    # the oracle runs on the basis the GPU sees (upcast)
    Qseen = Qd.to(torch.float64).cpu().numpy().T
    for m in (2, w.m // 2, w.m):
        U, info = rw.solve_seeds(gg, Qd, lamd, node, lab, w.C, m_avail=m)
        Ug = U.to(torch.float64).cpu().numpy().T
        Uo = fast_rw(og, Qseen, lam, node, lab, w.C, m=m, exact=_needs_exact(lam[:m]))
        err = np.abs(Ug - Uo).max()
        if kind == "rel":
            assert err <= tol * max(1.0, np.abs(Uo).max()), (m, err)
        else:
            assert err <= tol, (m, err)
        assert info["m_used"] == m
        np.testing.assert_array_equal(Ug[node, lab], 1.0)
    # full basis (tiny case) reproduces exact random walker
    if w.N <= 500 and qdt == torch.float64:
        lamf, Qf = dense_eigpairs(og, og.N)
        U, _ = rw.solve_seeds(gg, to_dev(Qf.T, qdt), to_dev(lamf, torch.float64), node, lab, w.C)
        Ue = exact_rw(og, node, lab, w.C, method="direct")
        assert np.abs(U.cpu().numpy().T - Ue).max() < 1e-9


# weakly coupled phantoms: a region joined to the rest by weights near exp(-90 * 0.36); the second eigenvalue
# is 7e-14 (64 x 48) and -1.3e-16 (the 129 x 7 strip), and the reduced system's condition number ~1e15
WEAK = [("strip129x7", rwsynth.Workload("b5", 505, (129, 7, 1), 4, 90.0, 8, 3, 5, 0.05, 4, "cycle", 0.0, "f64")),
        ("img64x48", rwsynth.Workload("b1", 501, (64, 48, 1), 4, 90.0, 30, 3, 5, 0.05, 4, "cycle", 0.0, "f64"))]


@pytest.mark.parametrize("name,w", WEAK, ids=[c[0] for c in WEAK])
@pytest.mark.parametrize("gdt,qdt,tol", [(torch.float64, torch.float64, 1e-10), (torch.float32, torch.float32, 1e-4),
                                         (torch.float32, torch.bfloat16, 1e-2)], ids=["f64", "f32", "bf16"])
def test_solve_weakly_coupled_matches_exact_oracle(name, w, gdt, qdt, tol):
    """The FP32 graph's coefficients and the stored low-precision null vector would decide the solution of
    this system; the solve forms its seed rows from FP64 weights and takes the basis in FP64 around the exact
    null vector, and matches the oracle's exact evaluation of the bordered system on the same basis."""
    need_gpu()
    banner(f"solve weakly coupled {name} {gdt} {qdt}")
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0, per_label=5, stream_offset=3)
    og = OGraph(J, w.dims, w.conn, w.beta)
    lam, Q = dense_eigpairs(og, w.m)
    assert np.min(np.abs(lam[1:])) < 1e-12
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=gdt)
    Qd = to_dev(Q.T, qdt)
    Qseen = Qd.to(torch.float64).cpu().numpy().T
    U, info = rw.solve_seeds(gg, Qd, to_dev(lam, torch.float64), node, lab, w.C)
    Uo = fast_rw(og, Qseen, lam, node, lab, w.C, exact=True)
    err = np.abs(U.to(torch.float64).cpu().numpy().T - Uo).max()
    print(f"  S={node.size} min_pivot={info['min_pivot']:.1e} err={err:.2e}", flush=True)
    bound = tol * max(1.0, np.abs(Uo).max()) if gdt == torch.float64 else tol
    assert err <= bound, err


def test_solve_rows_sum_to_one_and_seed_validation():
    need_gpu()
    w = CASES[0][1]
    J, node, lab, og, lam, Q = _oracle_case(w)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    Qd, lamd = to_dev(Q.T, torch.float64), to_dev(lam, torch.float64)
    # unsorted input with an exact duplicate gives the same answer
    perm = np.random.default_rng(0).permutation(node.size)
    n2 = np.concatenate([node[perm], node[:1]])
    l2 = np.concatenate([lab[perm], lab[:1]])
    U1, _ = rw.solve_seeds(gg, Qd, lamd, node, lab, w.C)
    U2, _ = rw.solve_seeds(gg, Qd, lamd, n2, l2, w.C)
    assert torch.equal(U1, U2)
    np.testing.assert_allclose(U1.sum(0).cpu().numpy(), 1.0, atol=1e-12)
    # conflicting duplicate, out-of-range node and label
    for bad_n, bad_l in ((np.concatenate([node, node[:1]]), np.concatenate([lab, (lab[:1] + 1) % w.C])),
                         (np.concatenate([node, [og.N]]), np.concatenate([lab, [0]])),
                         (node, np.where(np.arange(node.size) == 0, w.C, lab))):
        with pytest.raises(rw.RWError) as ei:
            rw.solve_seeds(gg, Qd, lamd, bad_n, bad_l, w.C)
        assert ei.value.status == rw.RW_EINVAL


@pytest.mark.parametrize("seed,per,m", [(0, 5, 48), (1, 5, 48), (2, 5, 48), (3, 30, 60), (4, 40, 70)])
def test_choice_of_m_matches_oracle(seed, per, m):
    """Few seeds (the chosen m exceeds S: decided by the per-candidate eigendecompositions) and many
    seeds (the chosen m is below S: decided by the Cholesky screen)."""
    need_gpu()
    banner(f"choice of m seed={seed} per={per} m={m}")
    w = rwsynth.small("cm", (24, 22), 4, m=m, C=3, seeds_per_label=per, n_shapes=3, config_id=200 + seed)
    J, rid, node, lab = setup_case(w, seed)
    og = OGraph(J, w.dims, w.conn, w.beta)
    lam, Q = dense_eigpairs(og, w.m)
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, w.beta, dtype=torch.float64)
    for eps in (0.1, 0.05, 0.2):
        U, info = rw.solve_seeds(gg, to_dev(Q.T, torch.float64), to_dev(lam, torch.float64), node, lab, w.C, eps=eps)
        m_o, fmax, f = choose_m(og, Q, node, lab, w.C, eps=eps)
        if info["m_used"] != m_o:
            # only acceptable when the decision is borderline in FP64
            fa = f_values(og, Q, node, lab, w.C, info["m_used"]).max()
            fb = f_values(og, Q, node, lab, w.C, m_o).max()
            assert min(abs(fa - fmax), abs(fb - fmax)) <= 1e-9 * fmax, (eps, info, m_o)
        else:
            np.testing.assert_allclose(info["f_worst"], f.max(), rtol=1e-8, atol=1e-12)
        mu = info["m_used"]
        Uo = fast_rw(og, Q, lam, node, lab, w.C, m=mu, exact=_needs_exact(lam[:mu]))
        assert np.abs(U.cpu().numpy().T - Uo).max() < 1e-10
