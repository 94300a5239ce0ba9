"""Full-size gradient check on the differentiation workload: a 96^3 phantom (5 ellipsoids, noise sigma
0.05), 6-connected, beta 120, C = 2, 100 seeds per label, m = 80 eigenpairs for the warm starts; loss =
mean cross-entropy of the exact random walker probabilities against the phantom's mask.

The forward and adjoint gradients (dl/dJ, dl/dbeta, dl/ds) through the autograd Function are compared
with the oracle's exact adjoint (stored in tests/golden/grad96.json: 64 sampled intensities, 64 sampled
edges, beta, one random direction, U at 1000 voxels) and with central finite differences of the GPU
forward (h = 1e-6, FP64) on the same entries.  The finite differences carry an absolute noise of about
1e-9 (two forward solves to a relative residual of 1e-13, divided by 2h); the gate is 1e-5 relative plus
5e-9 absolute."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1607_04174_amd as rw
import rwsynth

from gpu_common import banner, need_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad96.json")
H = 1e-6


def test_grad96_against_oracle_adjoint_and_finite_differences():
    need_gpu()
    gold = json.load(open(GOLDEN))
    w = rwsynth.CFG5
    banner(f"grad96 {w.dims} C={w.C}")
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    gt = rwsynth.label_map(rid, w.C)
    assert gold["N"] == w.N
    dev = torch.device("cuda", 0)
    Jd = torch.as_tensor(J, device=dev, dtype=torch.float64)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float64)
    Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-8, max_iter=600)
    scale = torch.ones((3, w.N), dtype=torch.float64, device=dev)
    mask = torch.ones(w.N, dtype=torch.bool, device=dev)
    mask[torch.as_tensor(node, device=dev)] = False
    y = torch.as_tensor(gt, device=dev, dtype=torch.long)

    def loss_of(U):
        p = U.gather(0, y[None, :])[0]
        return -(torch.log(torch.clamp(p[mask], min=1e-12))).mean()

    Jt = Jd.clone().requires_grad_(True)
    bt = torch.tensor(w.beta, dtype=torch.float64, device=dev, requires_grad=True)
    st = scale.clone().requires_grad_(True)
    U = rw.random_walker(Jt, bt, st, w.dims, w.conn, node, lab, w.C, Q=Q, lam=lam, tol=1e-12)
    L = loss_of(U)
    L.backward()
    dJ, db, ds = Jt.grad.cpu().numpy(), float(bt.grad), st.grad.cpu().numpy()
    Ud = U.detach()

    # against the oracle
    un = np.asarray(gold["U_nodes"])
    e_u = np.abs(Ud[:, torch.as_tensor(un, device=dev)].T.cpu().numpy() - np.asarray(gold["U_values"])).max()
    e_l = abs(float(L.detach()) - gold["loss"])
    ji, jv = np.asarray(gold["dJ_index"]), np.asarray(gold["dJ_value"])
    ed, et, ev = np.asarray(gold["ds_dir"]), np.asarray(gold["ds_tail"]), np.asarray(gold["ds_value"])
    d = torch.as_tensor(np.random.default_rng(gold["direction_seed"]).standard_normal(w.N), device=dev)
    dirv = float((Jt.grad * d).sum())
    print(f"  vs oracle: U {e_u:.1e}, loss {e_l:.1e}, dJ {np.abs(dJ[ji] - jv).max():.1e} "
          f"(max |dJ| {gold['dJ_absmax']:.1e}), ds {np.abs(ds[ed, et] - ev).max():.1e}, "
          f"dbeta {abs(db - gold['dbeta']):.1e}, direction {abs(dirv - gold['direction_value']):.1e}", flush=True)
    assert e_u <= 1e-9 and e_l <= 1e-12
    np.testing.assert_allclose(dJ[ji], jv, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(ds[ed, et], ev, rtol=1e-7, atol=1e-12)
    assert abs(db - gold["dbeta"]) <= 1e-7 * abs(gold["dbeta"])
    assert abs(dirv - gold["direction_value"]) <= 1e-7 * abs(gold["direction_value"])

    # central finite differences of the GPU forward
    def fwd(J_=None, beta=w.beta, s=scale):
        with torch.no_grad():
            Uf = rw.random_walker(Jd if J_ is None else J_, torch.tensor(beta, dtype=torch.float64), s, w.dims,
                                  w.conn, node, lab, w.C, Q=Q, lam=lam, tol=1e-13)
            return float(loss_of(Uf))

    def check(fd, adj, what):
        assert abs(fd - adj) <= 1e-5 * abs(adj) + 5e-9, (what, fd, adj)

    worst = 0.0
    for i in ji:
        Jp, Jm = Jd.clone(), Jd.clone()
        Jp[int(i)] += H
        Jm[int(i)] -= H
        fd = (fwd(J_=Jp) - fwd(J_=Jm)) / (2 * H)
        check(fd, float(dJ[i]), f"J[{i}]")
        worst = max(worst, abs(fd - dJ[i]))
    for dd, tt in zip(ed, et):
        sp, sm = scale.clone(), scale.clone()
        sp[int(dd), int(tt)] += H
        sm[int(dd), int(tt)] -= H
        fd = (fwd(s=sp) - fwd(s=sm)) / (2 * H)
        check(fd, float(ds[dd, tt]), f"s[{dd}, {tt}]")
        worst = max(worst, abs(fd - ds[dd, tt]))
    fd = (fwd(beta=w.beta + H) - fwd(beta=w.beta - H)) / (2 * H)
    check(fd, db, "beta")
    fd = (fwd(J_=Jd + H * d) - fwd(J_=Jd - H * d)) / (2 * H)
    check(fd, dirv, "direction")
    print(f"  finite differences: worst absolute difference {worst:.1e}", flush=True)
