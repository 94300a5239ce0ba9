"""Vertex aggregation and the transfer of the eigenbasis to the aggregated graph (oracle; test
infrastructure only).

Sec. III-C: a coarser vertex set of super-vertices y, a projection function eta(x, y) (the influence of
super-vertex y on vertex x) and an aggregation function eta_bar(x, y) (the influence of vertex x on
super-vertex y), normalized so that sum_y eta(x, y) = 1 and sum_x eta_bar(x, y) = 1.  The walker is solved
on the aggregated graph and propagated back by U_x = sum_y eta(x, y) U_bar_y.  The stored eigenvectors
are carried to the super-vertices by

    Delta(x) = sum_{x' in N(x)} sum_y |eta(x, y) - eta(x', y)|
    q_bar_y  = sum_x Delta(x) eta_bar(x, y) q_x

(eq. (33); Delta removes vertices whose edges are all consumed inside one super-vertex), then made
orthonormal by Gram-Schmidt and given their normalized-cut values (Rayleigh quotients) on the aggregated
graph, after which the fast walker runs there unchanged.

Readings:
  * the super-vertices: regular blocks of s x s (x s) voxels, the last ones clipped at the image border
    (the paper aggregates by prior probabilities and proximity; the transfer itself does not depend on how
    the vertices are grouped); eta(x, y) = 1 for the block y holding x, eta_bar(x, y) = 1 / |y| for x in y;
  * the aggregated graph: the same connectivity on the grid of blocks, the weight between two blocks the sum
    of the weights of the edges joining them, so that its Laplacian is P^T L P for the 0/1 assignment
    matrix P (edges inside a block cancel);
  * N(x): the vertices joined to x by an edge of the graph (present, whatever its weight);
  * eq. (33) acts on the stored columns as they are (the variables of the operator: hat variables under
    L_hat), and the result is read as in the beta update: the aggregated graph's null vector replaces the
    first column, the others are orthonormalized against it in order, and the quotients use the aggregated
    operator (update.diag_rq);
  * seeds move to their blocks; two seeds with different labels in one block are an error.
"""
from __future__ import annotations

import numpy as np

from .graph import Graph
from .update import diag_rq


def blocks(dims, s):
    """(block index of every vertex, block grid dims)."""
    nx, ny, nz = dims
    cx, cy = -(-nx // s), -(-ny // s)
    cz = -(-nz // s) if nz > 1 else 1
    i = np.arange(nx * ny * nz)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    return (x // s) + cx * ((y // s) + cy * (z // s if nz > 1 else 0)), (cx, cy, cz)


def _coords(idx, dims):
    nx, ny, _ = dims
    return np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=-1)


def aggregate_graph(graph, s):
    """The aggregated graph: a Graph on the block grid, same connectivity, intensities 0 (base weights 1)
    and per-edge scales = summed weights of the fine edges joining the two blocks."""
    b, cdims = blocks(graph.dims, s)
    coarse = Graph(np.zeros(cdims[0] * cdims[1] * cdims[2]), cdims, graph.conn, graph.beta,
                   weight_form=graph.weight_form, normalized=graph.normalized)
    w = graph.w
    bt, bh = b[graph.tail], b[graph.head]
    cross = (bt != bh) & (w != 0.0)
    ct, ch = _coords(bt[cross], cdims), _coords(bh[cross], cdims)
    off = ch - ct
    # coarse forward directions and their offsets
    dirs = {}
    for e, t, h, d in zip(coarse.edge_id, coarse.tail, coarse.head, coarse.dir):
        o = tuple(_coords(np.array([h]), cdims)[0] - _coords(np.array([t]), cdims)[0])
        dirs.setdefault(int(d), o)
    scale = np.zeros(coarse.edge_id.size)
    Nc = coarse.N
    for k, (tb, hb, o, wk) in enumerate(zip(bt[cross], bh[cross], off, w[cross])):
        o = tuple(int(v) for v in o)
        eid = None
        for d, od in dirs.items():
            if od == o:
                eid = d * Nc + int(tb)
            elif od == tuple(-v for v in o):
                eid = d * Nc + int(hb)
        if eid is None:
            raise ValueError(f"blocks joined by offset {o} have no edge in the aggregated connectivity")
        scale[coarse._pos[eid]] += wk
    coarse.scale = scale
    return coarse


def delta(graph, s):
    """Delta(x) = sum over the edge neighbours x' of sum_y |eta(x, y) - eta(x', y)| (2 per neighbour in
    another block)."""
    b, _ = blocks(graph.dims, s)
    t, h = graph.tail[graph.present], graph.head[graph.present]
    diff = (b[t] != b[h]).astype(np.float64) * 2.0
    out = np.zeros(graph.N)
    np.add.at(out, t, diff)
    np.add.at(out, h, diff)
    return out


def aggregate_basis(graph, Q, s):
    """eq. (33): q_bar_y = sum_x Delta(x) eta_bar(x, y) q_x for every column of Q (N x m)."""
    b, cdims = blocks(graph.dims, s)
    Nc = cdims[0] * cdims[1] * cdims[2]
    size = np.bincount(b, minlength=Nc).astype(np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    out = np.zeros((Nc, Q.shape[1]))
    np.add.at(out, b, delta(graph, s)[:, None] * Q)
    return out / size[:, None]


def transfer_basis(graph, Q, s):
    """(aggregated graph, Q_bar (orthonormalized, null vector first), lambda_bar (quotients))."""
    coarse = aggregate_graph(graph, s)
    Qn, lam = diag_rq(coarse, aggregate_basis(graph, Q, s))
    return coarse, Qn, lam


def coarse_seeds(graph, s, seed_node, seed_label):
    """Seeds moved to their blocks (sorted, distinct); conflicting labels in one block raise ValueError."""
    b, _ = blocks(graph.dims, s)
    lab = {}
    for v, l in zip(np.asarray(seed_node), np.asarray(seed_label)):
        y = int(b[int(v)])
        if lab.setdefault(y, int(l)) != int(l):
            raise ValueError(f"block {y} holds seeds of labels {lab[y]} and {int(l)}")
    ys = np.array(sorted(lab), dtype=np.int64)
    return ys, np.array([lab[int(y)] for y in ys], dtype=np.int32)


def prolong(graph, s, Ubar):
    """U_x = sum_y eta(x, y) U_bar_y = U_bar of x's block (Ubar: N_bar x C)."""
    b, _ = blocks(graph.dims, s)
    return np.asarray(Ubar)[b]
