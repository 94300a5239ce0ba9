"""Image graph and Laplacian (oracle; test infrastructure only).

Sec. II-A, eq. (2): w_xy = exp(-beta |J(x) - J(y)|) for neighbouring voxels, 0 otherwise; D is the
diagonal of row sums of W and L = D - W.  Sec. II-C: the normalized Laplacian
L_hat = D^{-1/2} L D^{-1/2}, with U_hat = D^{1/2} U.

Readings (the paper is silent or differs from the benchmark statement):
  * weight form: the default is the squared difference exp(-beta (J_x - J_y)^2) that the
    benchmark statement fixes; the paper's absolute difference is kept as weight_form="abs".
    Both give w(2 beta) = w(beta)^2, the property quoted in Sec. IV-C.
  * neighbourhood: 4- or 8-connected in 2D, 6-connected in 3D; diagonal edges use the same formula
    with no distance factor; free boundary, no wrap-around.
  * per-edge scale s_e (default 1): w_e = s_e * exp(...), so that edits can scale or remove edges
    (s_e = 0 and the edge marked absent) and a later beta change keeps them.
  * a node with d = 0 gets D^{-1/2} := 0, so its row of L_hat is zero.
  * the null vector (Sec. II-B, after eq. (6)): g = 1/sqrt(N) for L; for L_hat it is
    D^{1/2} 1 / ||D^{1/2} 1||.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def forward_offsets(ndim: int, conn: int):
    """Forward neighbour offsets (dx, dy, dz), one per stored edge direction."""
    if ndim == 2 and conn == 4:
        return [(1, 0, 0), (0, 1, 0)]
    if ndim == 2 and conn == 8:
        return [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0)]
    if ndim == 3 and conn == 6:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    raise ValueError(f"unsupported connectivity {conn} for {ndim}D")


def grid_edges(dims, conn):
    """Every edge of the grid graph as (edge_id, tail, head, dir); edge_id = dir*N + tail."""
    nx, ny, nz = dims
    ndim = 2 if nz == 1 else 3
    N = nx * ny * nz
    ids, tails, heads, dirs = [], [], [], []
    for d, (dx, dy, dz) in enumerate(forward_offsets(ndim, conn)):
        for z in range(nz):
            for y in range(ny):
                x = np.arange(nx)
                xh, yh, zh = x + dx, y + dy, z + dz
                ok = (xh >= 0) & (xh < nx) & (0 <= yh < ny) & (0 <= zh < nz)
                t = x[ok] + nx * (y + ny * z)
                h = xh[ok] + nx * (yh + ny * zh)
                ids.append(d * N + t)
                tails.append(t)
                heads.append(h)
                dirs.append(np.full(t.size, d))
    return (np.concatenate(ids).astype(np.int64), np.concatenate(tails).astype(np.int64),
            np.concatenate(heads).astype(np.int64), np.concatenate(dirs).astype(np.int64))


class Graph:
    """Weighted image graph with its Laplacians, all in FP64."""

    def __init__(self, J, dims, conn, beta, weight_form="squared", normalized=True):
        self.J = np.asarray(J, dtype=np.float64).reshape(-1)
        self.dims = tuple(int(v) for v in dims)
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        assert self.J.size == self.N
        self.ndim = 2 if self.dims[2] == 1 else 3
        self.conn = conn
        self.beta = float(beta)
        self.weight_form = weight_form
        self.normalized = normalized
        self.edge_id, self.tail, self.head, self.dir = grid_edges(self.dims, conn)
        self.scale = np.ones(self.edge_id.size)
        self.present = np.ones(self.edge_id.size, dtype=bool)
        self._pos = {int(e): k for k, e in enumerate(self.edge_id)}

    # ---- weights (Sec. II-A eq. (2)) ----
    def base_weight(self):
        diff = self.J[self.tail] - self.J[self.head]
        if self.weight_form == "squared":
            return np.exp(-self.beta * diff * diff)
        return np.exp(-self.beta * np.abs(diff))

    @property
    def w(self):
        return np.where(self.present, self.scale * self.base_weight(), 0.0)

    def W(self):
        w = self.w
        A = sp.coo_matrix((np.concatenate([w, w]),
                           (np.concatenate([self.tail, self.head]), np.concatenate([self.head, self.tail]))),
                          shape=(self.N, self.N))
        return A.tocsr()

    def degree(self):
        d = np.zeros(self.N)
        np.add.at(d, self.tail, self.w)
        np.add.at(d, self.head, self.w)
        return d

    def dinv_sqrt(self):
        d = self.degree()
        out = np.zeros(self.N)
        pos = d > 0
        out[pos] = 1.0 / np.sqrt(d[pos])
        return out

    def L(self):
        """L = D - W (sparse CSR)."""
        return (sp.diags(self.degree()) - self.W()).tocsr()

    def Lhat(self):
        """L_hat = D^{-1/2} L D^{-1/2} (Sec. II-C); zero rows/columns where d = 0."""
        Dm = sp.diags(self.dinv_sqrt())
        return (Dm @ self.L() @ Dm).tocsr()

    def M(self):
        """The operator the method works with: L_hat (default) or L."""
        return self.Lhat() if self.normalized else self.L()

    def ghat(self):
        """Unit null vector of M: D^{1/2} 1 / ||D^{1/2} 1|| (normalized) or 1/sqrt(N)."""
        if self.normalized:
            v = np.sqrt(self.degree())
        else:
            v = np.ones(self.N)
        return v / np.linalg.norm(v)

    def hat_scale(self):
        """Per-node factor s with U_hat = s * U: D^{1/2} (normalized) or 1."""
        return np.sqrt(self.degree()) if self.normalized else np.ones(self.N)

    # ---- edits ----
    def set_beta(self, beta):
        self.beta = float(beta)

    def scale_edges(self, edge_ids, factor):
        for e in np.asarray(edge_ids).reshape(-1):
            k = self._pos.get(int(e))
            if k is None or not self.present[k]:
                raise ValueError(f"edge {int(e)} is not present")
            self.scale[k] *= factor

    def box_edge_ids(self, lo, hi):
        """Ids of the present edges with both endpoints inside the box [lo, hi) (x, y, z)."""
        nx, ny, _ = self.dims
        def inside(i):
            x = i % nx
            y = (i // nx) % ny
            z = i // (nx * ny)
            return ((x >= lo[0]) & (x < hi[0]) & (y >= lo[1]) & (y < hi[1]) & (z >= lo[2]) & (z < hi[2]))
        sel = inside(self.tail) & inside(self.head) & self.present
        return self.edge_id[sel]

    def scale_box(self, lo, hi, factor):
        self.scale_edges(self.box_edge_ids(lo, hi), factor)

    def remove_edges(self, edge_ids):
        for e in np.asarray(edge_ids).reshape(-1):
            k = self._pos.get(int(e))
            if k is None or not self.present[k]:
                raise ValueError(f"edge {int(e)} is not present")
            self.present[k] = False
            self.scale[k] = 0.0

    def apply_edit(self, edit):
        """Apply one rwsynth.Edit-like object (kind, value, box_lo, box_hi, edge_ids)."""
        if edit.kind == "set_beta":
            self.set_beta(edit.value)
        elif edit.kind == "scale_box":
            self.scale_box(edit.box_lo, edit.box_hi, edit.value)
        elif edit.kind == "scale_edges":
            self.scale_edges(edit.edge_ids, edit.value)
        elif edit.kind == "remove_edges":
            self.remove_edges(edit.edge_ids)
        else:
            raise ValueError(edit.kind)

    def copy(self):
        g = Graph(self.J, self.dims, self.conn, self.beta, self.weight_form, self.normalized)
        g.scale = self.scale.copy()
        g.present = self.present.copy()
        return g

    def mask_bits(self):
        """uint8 per node: bit d set iff the forward edge in direction d exists (present)."""
        m = np.zeros(self.N, dtype=np.uint8)
        for d in range(len(forward_offsets(self.ndim, self.conn))):
            sel = (self.dir == d) & self.present
            m[self.tail[sel]] |= np.uint8(1 << d)
        return m

    def weights_by_dir(self):
        """Dense [ndir][N] array of forward-edge weights (0 where the edge is absent or off-grid)."""
        nd = len(forward_offsets(self.ndim, self.conn))
        out = np.zeros((nd, self.N))
        out[self.dir, self.tail] = self.w
        return out
