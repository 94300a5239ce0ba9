"""Seeded synthetic inputs for random-walker segmentation: phantoms, seeds and graph edits.

This module generates *inputs only*.  It holds none of the method's arithmetic (no edge weights,
no Laplacian, no solve): it draws images, label maps, seed sets and edit lists, and both the CPU
oracle and the GPU path consume what it returns.

The paper evaluates on clinical images (2D cardiac CT and blood-cell slices, 3D thigh MR and brain
MR; Section IV-A, "Setup") that are not available here.  Piecewise-constant ellipse / ellipsoid
phantoms with Gaussian noise stand in for them: they have the same structure (a few regions with
distinct mean intensity separated by sharp edges), 2-5 labels, and tens to hundreds of seeds per
label, as in the paper's seed protocol (Section IV-A).

Layout conventions shared by every consumer:
  * an image of dims (nx, ny[, nz]) is a flat array of N = nx*ny*nz values, x fastest, then y, then z
    (node id  i = x + nx*(y + ny*z));
  * seeds are (node id int64, label int32) pairs sorted by node id;
  * an edge is named by  e = dir*N + tail, where the edge joins `tail` and `tail + offset(dir)`
    and the forward directions are, in order,
        2D 4-connected: +x, +y
        2D 8-connected: +x, +y, +x+y, +x-y
        3D 6-connected: +x, +y, +z
    (this numbering is an interface, documented beside the C header's edit structure).

Random streams: numpy PCG64 seeded with SeedSequence([config_id, seed, stream]), one stream each
for the phantom geometry (0), the noise (1), the seeds (2) and the edits (3).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.ndimage as ndi

STREAM_PHANTOM, STREAM_NOISE, STREAM_SEEDS, STREAM_EDITS = 0, 1, 2, 3

# forward stencil offsets (dx, dy, dz) per direction; the edge-id interface above
FORWARD_DIRS = {
    (2, 4): ((1, 0, 0), (0, 1, 0)),
    (2, 8): ((1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0)),
    (3, 6): ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
}


def rng_for(config_id: int, seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, seed, stream])))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload (image + labels + method parameters)."""
    name: str
    config_id: int
    dims: Tuple[int, int, int]          # (nx, ny, nz); nz = 1 for 2D
    conn: int                           # 4 or 8 (2D), 6 (3D)
    beta: float
    m: int                              # number of precomputed eigenpairs (null pair included)
    C: int                              # number of labels
    seeds_per_label: int
    sigma: float                        # noise standard deviation
    n_shapes: int
    intensity: str                      # "cycle" ({0.2,0.5,0.8}[j mod 3]) or "uniform" (U[0,1])
    ramp: float = 0.0                   # + ramp * x/(nx-1)
    dtype: str = "f64"                  # arithmetic type of the path for this workload

    @property
    def ndim(self) -> int:
        return 2 if self.dims[2] == 1 else 3

    @property
    def N(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]


# The five workloads of the benchmark plan, plus tiny ones for oracle/parity tests.
CFG1 = Workload("2d64_4conn_m50", 1, (64, 64, 1), 4, 90.0, 50, 2, 20, 0.05, 3, "cycle", 0.0, "f64")
CFG2 = Workload("2d512_8conn_m200", 2, (512, 512, 1), 8, 90.0, 200, 3, 50, 0.05, 6, "cycle", 0.2, "f32")
CFG3 = Workload("3d128_6conn_m100", 3, (128, 128, 128), 6, 120.0, 100, 4, 200, 0.03, 8, "uniform", 0.0,
                "mixed")
CFG5 = Workload("3d96_6conn_m80_grad", 5, (96, 96, 96), 6, 120.0, 80, 2, 100, 0.05, 5, "cycle", 0.0, "f64")

# cfg2 online edits (applied cumulatively, in this order)
CFG2_EDIT_BETA = 150.0
CFG2_EDIT_BOX = 32
CFG2_EDIT_BOX_SCALE = 0.1
CFG2_EDIT_REMOVE = 500

CYCLE = (0.2, 0.5, 0.8)


def small(name: str, dims, conn, beta=90.0, m=12, C=2, seeds_per_label=3, sigma=0.05, n_shapes=2,
          intensity="cycle", ramp=0.0, config_id=100, dtype="f64") -> Workload:
    """A small workload for tests (same generator, other sizes)."""
    d = tuple(dims) + (1,) * (3 - len(dims))
    return Workload(name, config_id, d, conn, beta, m, C, seeds_per_label, sigma, n_shapes, intensity,
                    ramp, dtype)


# ----------------------------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------------------------

def _rotation3(rng: np.random.Generator) -> np.ndarray:
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 2] = -q[:, 2]
    return q


def phantom(w: Workload, seed: int = 0):
    """Return (J, region_id): J float64 flat intensities, region_id int32 flat (0 = background,
    j+1 = shape j after painter's-order overwriting)."""
    nx, ny, nz = w.dims
    rng = rng_for(w.config_id, seed, STREAM_PHANTOM)
    side = float(min(nx, ny) if nz == 1 else min(nx, ny, nz))
    if nz == 1:
        yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                             indexing="ij")
        coords = [xx, yy]
    else:
        zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                                 np.arange(nx, dtype=np.float64), indexing="ij")
        coords = [xx, yy, zz]
    ndim = len(coords)
    sizes = [nx, ny, nz][:ndim]
    J = np.zeros(coords[0].shape, dtype=np.float64)
    rid = np.zeros(coords[0].shape, dtype=np.int32)
    for j in range(w.n_shapes):
        c = np.array([rng.uniform(0.15, 0.85) * s for s in sizes])
        a = rng.uniform(0.08, 0.30, size=ndim) * side
        if ndim == 2:
            th = rng.uniform(0.0, np.pi)
            R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        else:
            R = _rotation3(rng)
        val = CYCLE[j % 3] if w.intensity == "cycle" else rng.uniform(0.0, 1.0)
        d = [coords[k] - c[k] for k in range(ndim)]
        # coordinates in the shape frame: R^T d
        acc = np.zeros_like(J)
        for r in range(ndim):
            u = sum(R[k, r] * d[k] for k in range(ndim))
            acc += (u / a[r]) ** 2
        inside = acc <= 1.0
        J[inside] = val
        rid[inside] = j + 1
    if w.ramp:
        J = J + w.ramp * coords[0] / (nx - 1)
    noise = rng_for(w.config_id, seed, STREAM_NOISE).standard_normal(J.shape)
    J = J + w.sigma * noise
    return J.reshape(-1), rid.reshape(-1)


def label_map(region_id: np.ndarray, C: int) -> np.ndarray:
    """0 = background; shape j -> 1 + (j mod (C-1)).  region_id = j+1 for shape j."""
    lab = np.zeros_like(region_id)
    fg = region_id > 0
    if C > 1:
        lab[fg] = 1 + (region_id[fg] - 1) % (C - 1)
    return lab.astype(np.int32)


def _structure(ndim: int, conn: int):
    if ndim == 2 and conn == 8:
        return np.ones((3, 3), dtype=bool)
    return ndi.generate_binary_structure(ndim, 1)


def seeds(w: Workload, region_id: np.ndarray, seed: int = 0, C: Optional[int] = None,
          per_label: Optional[int] = None, stream_offset: int = 0):
    """Seed set: for every label, one seed in each connected component of each of its regions,
    then the rest uniformly without replacement among the label's pixels, up to `per_label`
    (more if the mandatory ones exceed it).  Returns (node int64 sorted, label int32)."""
    C = w.C if C is None else C
    per_label = w.seeds_per_label if per_label is None else per_label
    nx, ny, nz = w.dims
    shape = (ny, nx) if nz == 1 else (nz, ny, nx)
    lab = label_map(region_id, C)
    rng = rng_for(w.config_id, seed, STREAM_SEEDS + 16 * stream_offset)
    st = _structure(w.ndim, w.conn)
    nodes: List[np.ndarray] = []
    labels: List[np.ndarray] = []
    for k in range(C):
        pix = np.flatnonzero(lab == k)
        if pix.size == 0:
            continue
        chosen = []
        for r in np.unique(region_id[pix]):
            comp, ncomp = ndi.label((region_id == r).reshape(shape), structure=st)
            comp = comp.reshape(-1)
            for ci in range(1, ncomp + 1):
                members = np.flatnonzero(comp == ci)
                chosen.append(int(members[rng.integers(members.size)]))
        chosen = np.array(sorted(set(chosen)), dtype=np.int64)
        rest = np.setdiff1d(pix, chosen, assume_unique=False)
        extra = max(0, per_label - chosen.size)
        extra = min(extra, rest.size)
        if extra:
            chosen = np.concatenate([chosen, rng.choice(rest, size=extra, replace=False)])
        nodes.append(chosen.astype(np.int64))
        labels.append(np.full(chosen.size, k, dtype=np.int32))
    node = np.concatenate(nodes)
    label = np.concatenate(labels)
    order = np.argsort(node, kind="stable")
    return node[order], label[order]


# ----------------------------------------------------------------------------------------------
# edge ids and edits
# ----------------------------------------------------------------------------------------------

def edge_ids_valid(dims, conn) -> np.ndarray:
    """All edge ids e = dir*N + tail whose head lies inside the grid (free boundary)."""
    nx, ny, nz = dims
    ndim = 2 if nz == 1 else 3
    N = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    out = []
    for d, (dx, dy, dz) in enumerate(FORWARD_DIRS[(ndim, conn)]):
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        out.append(d * N + np.flatnonzero(ok))
    return np.concatenate(out).astype(np.int64)


@dataclasses.dataclass
class Edit:
    kind: str                      # "set_beta" | "scale_box" | "scale_edges" | "remove_edges"
    value: float = 0.0
    box_lo: Tuple[int, int, int] = (0, 0, 0)
    box_hi: Tuple[int, int, int] = (0, 0, 0)   # exclusive
    edge_ids: Optional[np.ndarray] = None


def cfg2_edits(w: Workload, seed: int = 0) -> List[Edit]:
    """The three online edits of the 512x512 workload, cumulative, in order: beta 90 -> 150; the
    edges with both endpoints in a random 32x32 block scaled by 0.1; 500 random edges removed
    (uniform without replacement over the edges present after the first two edits)."""
    rng = rng_for(w.config_id, seed, STREAM_EDITS)
    nx, ny, _ = w.dims
    b = CFG2_EDIT_BOX
    x0 = int(rng.integers(0, nx - b + 1))
    y0 = int(rng.integers(0, ny - b + 1))
    box = Edit("scale_box", CFG2_EDIT_BOX_SCALE, (x0, y0, 0), (x0 + b, y0 + b, 1))
    present = edge_ids_valid(w.dims, w.conn)
    rem = np.sort(rng.choice(present, size=CFG2_EDIT_REMOVE, replace=False)).astype(np.int64)
    return [Edit("set_beta", CFG2_EDIT_BETA), box, Edit("remove_edges", 0.0, edge_ids=rem)]


# ----------------------------------------------------------------------------------------------
# batched workload: 64 ragged 2D phantoms, 8 interaction rounds each
# ----------------------------------------------------------------------------------------------

CFG4_ID = 4


def cfg4_images(n_images: int = 64, seed: int = 0, side_lo: int = 128, side_hi: int = 768):
    """Per image: a Workload (4 ellipses, sigma 0.05, 4-connected, beta 90) with side lengths drawn
    uniformly in [side_lo, side_hi] and m drawn from {50, 100, 200}."""
    rng = rng_for(CFG4_ID, seed, STREAM_PHANTOM + 100)
    out = []
    for i in range(n_images):
        nx = int(rng.integers(side_lo, side_hi + 1))
        ny = int(rng.integers(side_lo, side_hi + 1))
        m = int(rng.choice([50, 100, 200]))
        out.append(Workload(f"batch{i}", 1000 + i, (nx, ny, 1), 4, 90.0, m, 2, 10, 0.05, 4, "cycle", 0.0,
                            "f32"))
    return out


def cfg4_round(img: Workload, region_id: np.ndarray, rnd: int, seed: int = 0):
    """Seed-set interaction `rnd` for one batched image: C ~ U{2,3,4}, seeds per label ~ U{10..100}."""
    rng = rng_for(img.config_id, seed, 1000 + rnd)
    C = int(rng.integers(2, 5))
    per = int(rng.integers(10, 101))
    node, label = seeds(img, region_id, seed=seed, C=C, per_label=per, stream_offset=rnd + 1)
    return C, node, label


# ----------------------------------------------------------------------------------------------
# registration-style priors (displacement labels)
# ----------------------------------------------------------------------------------------------
# In registration the labels are displacement vectors on a regular grid (Sec. IV-A: 21 x 21 x 9 or
# 31 x 31 x 13 of them) and the prior of label k at voxel x comes from comparing the patch around x
# with the patch around x + v_k in the other image, normalized over the labels.  The image pairs are
# not available; the stand-in keeps the structure such priors have: at each voxel a peak around the
# best-matching displacement, that displacement varying smoothly over the volume, with per-voxel
# jitter for the noise of the patch comparison.
STREAM_DISPLACEMENT = 4

CFG6_ID = 6
CFG6 = Workload("3d96_6conn_rwir", CFG6_ID, (96, 96, 96), 6, 50.0, 200, 21 * 21 * 9, 0, 0.03, 8, "uniform",
                0.0, "mixed")
CFG6_EXTENT = (21, 21, 9)        # displacement labels per axis: C = 3969
CFG6_GAMMA = 1.0
CFG6_SIGMA = 0.7                 # width of a voxel's prior peak, in label spacings
CFG6_JITTER = 0.5                # per-voxel jitter of the best displacement (voxels)


def displacement_labels(extent) -> np.ndarray:
    """C x 3 displacement vectors of the label grid (ex x ey x ez, centred at 0); label k = ix + ex*(iy +
    ey*iz), as the node numbering."""
    ex, ey, ez = (tuple(extent) + (1,) * 3)[:3]
    k = np.arange(ex * ey * ez)
    return np.stack([k % ex - ex // 2, (k // ex) % ey - ey // 2, k // (ex * ey) - ez // 2],
                    axis=1).astype(np.float64)


def displacement_field(dims, extent, config_id: int, seed: int = 0, n_bumps: int = 4,
                       jitter: float = CFG6_JITTER) -> np.ndarray:
    """N x 3 best-matching displacement per voxel: a sum of Gaussian bumps (centres uniform in the volume,
    widths 15-35 % of the smallest side, amplitudes up to 0.8 of the label range per axis) plus Gaussian
    jitter of standard deviation `jitter` per voxel and axis.  Axes without labels (extent 1) stay 0."""
    nx, ny, nz = dims
    ext = (tuple(extent) + (1,) * 3)[:3]
    rng = rng_for(config_id, seed, STREAM_DISPLACEMENT)
    i = np.arange(nx * ny * nz)
    xyz = np.stack([i % nx, (i // nx) % ny, i // (nx * ny)], axis=1).astype(np.float64)
    side = float(min(s for s in dims if s > 1))
    field = np.zeros((i.size, 3))
    for _ in range(n_bumps):
        c = rng.uniform(0.0, 1.0, size=3) * np.array(dims, dtype=np.float64)
        width = rng.uniform(0.15, 0.35) * side
        amp = rng.uniform(-0.8, 0.8, size=3) * np.array([e // 2 for e in ext], dtype=np.float64)
        r2 = (((xyz - c) * (np.array(dims) > 1)) ** 2).sum(axis=1)
        field += np.exp(-0.5 * r2 / width ** 2)[:, None] * amp[None, :]
    field += jitter * rng.standard_normal(field.shape) * (np.array(ext) > 1)[None, :]
    return field


def displacement_priors(field: np.ndarray, labels: np.ndarray, sigma: float = CFG6_SIGMA,
                        rows=None) -> np.ndarray:
    """N x C (or len(rows) x C) priors: at voxel x, p_k proportional to exp(-|v_k - d(x)|^2 / (2 sigma^2)),
    normalized over the labels (the largest exponent subtracted first)."""
    f = field if rows is None else field[np.asarray(rows)]
    e = -((f[:, None, :] - labels[None, :, :]) ** 2).sum(axis=2) / (2.0 * sigma * sigma)
    e -= e.max(axis=1, keepdims=True)
    p = np.exp(e)
    return p / p.sum(axis=1, keepdims=True)


def displacement_priors_torch(field, labels, sigma: float = CFG6_SIGMA, dtype=None, chunk: int = 16384):
    """The same priors computed with torch on the tensors' device, returned label-major (C, N) in `dtype`
    (FP32 arithmetic, so equal to displacement_priors up to FP32 rounding)."""
    import torch
    N, C = field.shape[0], labels.shape[0]
    out = torch.empty((C, N), dtype=dtype or torch.float32, device=field.device)
    f32, l32 = field.float(), labels.float()
    for a in range(0, N, chunk):
        f = f32[a:a + chunk]
        e = -((f[:, None, :] - l32[None, :, :]) ** 2).sum(dim=2) / (2.0 * sigma * sigma)
        out[:, a:a + chunk] = torch.softmax(e, dim=1).t().to(out.dtype)
    return out
