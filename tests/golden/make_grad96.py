"""Writes grad96.json: oracle values for the full-size gradient test of the differentiation workload
(96^3 phantom of 5 ellipsoids, noise sigma 0.05, 6-connected, beta 120, C = 2, 100 seeds per label; loss =
mean cross-entropy of the exact random walker probabilities against the phantom's mask over non-seed
voxels).  Exact random walker (Sec. II-A eq. (5), gamma = 0) and its adjoint by the oracle's
Jacobi-PCG to a relative residual of 1e-12.  Stored: the loss, U at 1000 seeded random voxels, dl/dJ at
the 32 largest-magnitude and 32 seeded random voxels, dl/ds at the 32 largest-magnitude and 32 seeded
random edges, dl/dbeta, and the directional derivative along a seeded standard-normal direction over J.

    python tests/golden/make_grad96.py        (about two minutes on one core)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import rwsynth  # noqa: E402
from oracle.adjoint import adjoint_grads, ce_grad, ce_loss  # noqa: E402
from oracle.exact_rw import exact_rw  # noqa: E402
from oracle.graph import Graph  # noqa: E402

DIRECTION_SEED = 7     # d = default_rng(7).standard_normal(N)
SAMPLE_SEED = 11


def main():
    w = rwsynth.CFG5
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    gt = rwsynth.label_map(rid, w.C)
    g = Graph(J, w.dims, w.conn, w.beta)
    U = exact_rw(g, node, lab, w.C, method="cg", tol=1e-12)
    G = ce_grad(U, gt, node)
    _, dJ, db, ds = adjoint_grads(g, node, lab, w.C, G, U, method="cg", tol=1e-12)
    rng = np.random.default_rng(SAMPLE_SEED)
    un = np.sort(rng.choice(g.N, 1000, replace=False))
    top = np.argsort(-np.abs(dJ), kind="stable")[:32]
    rest = np.setdiff1d(np.arange(g.N), top)
    ji = np.concatenate([top, np.sort(rng.choice(rest, 32, replace=False))])
    etop = np.argsort(-np.abs(ds), kind="stable")[:32]
    erest = np.setdiff1d(np.arange(ds.size), etop)
    ek = np.concatenate([etop, np.sort(rng.choice(erest, 32, replace=False))])
    d = np.random.default_rng(DIRECTION_SEED).standard_normal(g.N)
    out = {
        "source": "oracle: exact random walker and adjoint by Jacobi-PCG (tol 1e-12), Sec. II-A eq. (5); "
                  "written by tests/golden/make_grad96.py",
        "workload": w.name, "N": int(g.N), "loss": ce_loss(U, gt, node),
        "U_nodes": un.tolist(), "U_values": U[un].tolist(),
        "dJ_index": ji.tolist(), "dJ_value": dJ[ji].tolist(),
        "ds_dir": g.dir[ek].astype(int).tolist(), "ds_tail": g.tail[ek].astype(int).tolist(),
        "ds_value": ds[ek].tolist(), "dbeta": float(db),
        "direction_seed": DIRECTION_SEED, "direction_value": float(dJ @ d),
        "dJ_absmax": float(np.abs(dJ).max()), "ds_absmax": float(np.abs(ds).max()),
    }
    with open(os.path.join(HERE, "grad96.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
