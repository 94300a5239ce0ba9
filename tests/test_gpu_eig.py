"""GPU parity: offline eigenpairs and their online updates against the oracle."""
import itertools

import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth
from oracle.eigen import certify, dense_eigpairs, full_spectrum, principal_angle_sines
from oracle.graph import Graph as OGraph
from oracle.update import diag_rq, rayleigh_ritz

from gpu_common import banner, need_gpu, setup_case, to_dev

pytestmark = pytest.mark.gpu


def gap_index(ev, m, tol):
    """Largest m' <= m with a clear gap after it (the span of the first m' pairs is well defined)."""
    for mp in range(m, 1, -1):
        if ev[mp] - ev[mp - 1] > 100 * tol:
            return mp
    return 1


def _gpu_eig(w, dt, tol, m, beta=None, normalized=True, **kw):
    J, rid, node, lab = setup_case(w)
    beta = w.beta if beta is None else beta
    gg = rw.Graph(to_dev(J, torch.float64), w.dims, w.conn, beta, dtype=dt, normalized=normalized)
    og = OGraph(J, w.dims, w.conn, beta, normalized=normalized)
    Q, lam, info = rw.precompute_eig(gg, m, tol=tol, **kw)
    return gg, og, Q.to(torch.float64).cpu().numpy().T, lam.cpu().numpy(), info


EIG_CASES = [
    ("2d4_f64", rwsynth.small("e1", (24, 22), 4, n_shapes=3), torch.float64, 1e-10, 20),
    ("2d8_f64", rwsynth.small("e2", (19, 23), 8, n_shapes=3), torch.float64, 1e-10, 31),
    ("3d6_f64", rwsynth.small("e3", (9, 8, 7), 6, n_shapes=3), torch.float64, 1e-10, 16),
    ("2d8_f32", rwsynth.small("e4", (26, 24), 8, n_shapes=4), torch.float32, 1e-5, 30),
    ("3d6_f32", rwsynth.small("e5", (10, 9, 8), 6, n_shapes=3), torch.float32, 1e-5, 20),
    # blocks wide enough for the matrix-core Gram (X^T X and the symmetric X^T op X) and, at m = 190, for
    # the global-memory Jacobi variant of the Rayleigh-Ritz step
    ("2d8_f64_m110", rwsynth.small("e6", (30, 28), 8, n_shapes=4), torch.float64, 1e-10, 110),
    ("2d4_f32_m190", rwsynth.small("e7", (36, 34), 4, n_shapes=4), torch.float32, 1e-5, 190),
]


@pytest.mark.parametrize("name,w,dt,tol,m", EIG_CASES, ids=[c[0] for c in EIG_CASES])
def test_eigenpairs_match_dense_oracle(name, w, dt, tol, m):
    need_gpu()
    banner(f"eig {name}")
    gg, og, Q, lam, info = _gpu_eig(w, dt, tol, m)
    assert info["status"] == rw.RW_OK and info["n_converged"] == m
    # certification in FP64 on the CPU: residuals and orthonormality
    res, orth = certify(og, Q, lam)
    slack = 1.0 if dt == torch.float64 else 3.0   # FP32 storage of the returned vectors
    assert res.max() <= slack * tol + (2e-6 if dt == torch.float32 else 0.0), res.max()
    assert orth <= (1e-12 if dt == torch.float64 else 2e-6), orth
    # eigenvalues against the dense spectrum: each Ritz value within its residual of an eigenvalue
    ev = full_spectrum(og)
    np.testing.assert_allclose(lam, ev[:m], atol=max(10 * tol, 1e-12) if dt == torch.float64 else 5e-5)
    # the span of the first m' pairs (up to a clear gap) agrees with the dense eigenvectors
    mp = gap_index(ev, m, tol)
    lam_o, Q_o = dense_eigpairs(og, mp)
    assert principal_angle_sines(Q[:, :mp], Q_o).max() < (1e-6 if dt == torch.float64 else 3e-3)
    np.testing.assert_allclose(Q[:, 0], og.ghat(), atol=1e-15 if dt == torch.float64 else 1e-6)


def test_beta0_spectrum_closed_form_at_larger_size():
    """beta = 0, unnormalized L of a 4-connected 96 x 80 grid: eigenvalues are the sums of path-graph
    eigenvalues 4 sin^2(pi k / 2n) (exact, no dense oracle needed)."""
    need_gpu()
    banner("eig beta=0 closed form")
    nx, ny, m = 96, 80, 24
    J = np.zeros(nx * ny)
    gg = rw.Graph(to_dev(J, torch.float64), (nx, ny), 4, 0.0, dtype=torch.float64, normalized=False)
    Q, lam, info = rw.precompute_eig(gg, m, tol=1e-9)
    pe = lambda n: 4 * np.sin(np.pi * np.arange(n) / (2 * n)) ** 2
    expect = np.sort([a + b for a, b in itertools.product(pe(nx)[:20], pe(ny)[:20])])[:m]
    np.testing.assert_allclose(lam.cpu().numpy(), expect, atol=1e-9)


def test_noconvergence_is_reported_and_deterministic():
    need_gpu()
    w = EIG_CASES[0][1]
    gg, og, Q, lam, info = _gpu_eig(w, torch.float64, 1e-12, 20, max_iter=1, raise_on_noconv=False)
    assert info["status"] == rw.RW_ENOCONV and info["iters"] == 1
    _, _, Q2, lam2, info2 = _gpu_eig(w, torch.float64, 1e-12, 20, max_iter=1, raise_on_noconv=False)
    assert np.array_equal(Q, Q2) and np.array_equal(lam, lam2)       # bitwise reproducible
    with pytest.raises(rw.RWError) as ei:
        _gpu_eig(w, torch.float64, 1e-12, 20, max_iter=1)
    assert ei.value.status == rw.RW_ENOCONV


UPD_CASES = [
    ("2d8_f64", rwsynth.small("u1", (22, 20), 8, n_shapes=3), torch.float64, 1e-10, 24),
    ("2d8_f32", rwsynth.small("u2", (24, 22), 8, n_shapes=3), torch.float32, 1e-5, 24),
]


def _edits(w, og):
    rng = np.random.default_rng(3)
    valid = rwsynth.edge_ids_valid(w.dims, w.conn)
    rem = np.sort(rng.choice(valid, 15, replace=False))
    return [rwsynth.Edit("set_beta", 150.0), rwsynth.Edit("scale_box", 0.1, (3, 4, 0), (11, 12, 1)),
            rwsynth.Edit("remove_edges", edge_ids=rem)]


@pytest.mark.parametrize("dims,m", [((24, 22), 24), ((40, 36), 40)], ids=["small", "fold"])
def test_update_rr_on_a_perturbed_basis(dims, m):
    """Rayleigh-Ritz on a stored FP32 basis whose Gram is far from I (max |G - I| about 4e-3): the series for
    G^{-1/2} does not apply, so the step forms the projected matrix again with Cholesky QR.  The result is
    the Rayleigh-Ritz pairs of the same span (the second case takes the folded, in-place rotation)."""
    need_gpu()
    banner(f"update on a perturbed basis {dims}")
    w = rwsynth.small("up", dims, 8, n_shapes=3)
    dt, tol = torch.float32, 1e-5
    gg, og, Q0, lam0, info = _gpu_eig(w, dt, tol, m)
    Qp = Q0.copy()
    Qp[:, 1:] *= 1.0 + 2e-3 * (1.0 + np.arange(1, m) / m)   # same span, columns 1.. longer by 0.2-0.4 %
    edits = [rwsynth.Edit("set_beta", 150.0)]
    og2 = og.copy()
    og2.apply_edit(edits[0])
    g2 = rw.Graph(to_dev(og.J, torch.float64), w.dims, w.conn, w.beta, dtype=dt)
    Qd, lamd = to_dev(Qp.T, dt), to_dev(lam0, torch.float64)
    rw.update_eig(g2, edits, Qd, lamd, mode=rw.RW_UPDATE_RR, tol=tol)
    Qo, lo = rayleigh_ritz(og2, Qp.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(lamd.cpu().numpy(), lo, atol=2e-4)
    assert principal_angle_sines(Qd.to(torch.float64).cpu().numpy().T, Qo).max() < 1e-3


@pytest.mark.parametrize("name,w,dt,tol,m", UPD_CASES, ids=[c[0] for c in UPD_CASES])
def test_update_modes_match_oracle(name, w, dt, tol, m):
    need_gpu()
    banner(f"update {name}")
    vtol = 1e-10 if dt == torch.float64 else 2e-4
    gg, og, Q0, lam0, info = _gpu_eig(w, dt, tol, m)
    edits = _edits(w, og)
    og2 = og.copy()
    for e in edits:
        og2.apply_edit(e)
    # no edit: the paper's update returns the same eigenvalues
    for mode in (rw.RW_UPDATE_DIAG_RQ, rw.RW_UPDATE_RR):
        Qd, lamd = to_dev(Q0.T, dt), to_dev(lam0, torch.float64)
        rw.update_eig(gg, [], Qd, lamd, mode=mode, tol=tol)
        np.testing.assert_allclose(lamd.cpu().numpy(), lam0, atol=3 * tol)
    results = {}
    for mode in (rw.RW_UPDATE_DIAG_RQ, rw.RW_UPDATE_RR, rw.RW_UPDATE_RR_REFINE):
        g2 = rw.Graph(to_dev(og.J, torch.float64), w.dims, w.conn, w.beta, dtype=dt)
        Qd, lamd = to_dev(Q0.T, dt), to_dev(lam0, torch.float64)
        info = rw.update_eig(g2, edits, Qd, lamd, mode=mode, tol=tol)
        results[mode] = (Qd.to(torch.float64).cpu().numpy().T, lamd.cpu().numpy(), info)
    Qin = Q0.astype(np.float32).astype(np.float64) if dt == torch.float32 else Q0
    # mode 0: Gram-Schmidt in order + Rayleigh quotients (the paper's update)
    Qo, lo = diag_rq(og2, Qin)
    Qg, lg, _ = results[rw.RW_UPDATE_DIAG_RQ]
    np.testing.assert_allclose(lg, lo, atol=vtol)
    assert np.abs(Qg - Qo).max() < (1e-9 if dt == torch.float64 else 1e-3)
    # mode 1: Rayleigh-Ritz on the same span
    Qo, lo = rayleigh_ritz(og2, Qin)
    Qg, lg, _ = results[rw.RW_UPDATE_RR]
    np.testing.assert_allclose(lg, lo, atol=vtol)
    assert principal_angle_sines(Qg, Qo).max() < (1e-7 if dt == torch.float64 else 1e-3)
    # mode 2: refined to tol on the new graph; agrees with a cold recompute on the span
    Qg, lg, info = results[rw.RW_UPDATE_RR_REFINE]
    assert info["status"] == rw.RW_OK
    res, orth = certify(og2, Qg, lg)
    assert res.max() <= 3 * tol + (2e-6 if dt == torch.float32 else 0.0)
    ev = full_spectrum(og2)
    np.testing.assert_allclose(lg, ev[:m], atol=max(10 * tol, 1e-12) if dt == torch.float64 else 5e-5)
