"""Python binding of librw (include/rw.h): precomputed-eigenvector random-walker segmentation on
MI355X (gfx950).

This module only marshals arguments: every step of the computation runs in the HIP library.
PyTorch provides device memory (torch tensors on a ROCm device) and the current HIP stream.
The library must have been built (python -m paper_1607_04174_amd.build); importing the binding
without it raises immediately - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librw.so")

RW_OK, RW_EINVAL, RW_ENOCONV, RW_EUNANCHORED, RW_ESINGULAR, RW_EWORKSPACE, RW_EHIP, RW_ECAPTURE = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "RW_OK", -1: "RW_EINVAL", -2: "RW_ENOCONV", -3: "RW_EUNANCHORED", -4: "RW_ESINGULAR",
                -5: "RW_EWORKSPACE", -6: "RW_EHIP", -7: "RW_ECAPTURE"}
RW_F64, RW_F32, RW_BF16, RW_BF16_PAIR = 0, 1, 2, 3
RW_PAIR_COLS = 8
RW_EDIT_SET_BETA, RW_EDIT_SCALE_EDGES, RW_EDIT_SCALE_BOX, RW_EDIT_REMOVE_EDGES = 0, 1, 2, 3
RW_UPDATE_DIAG_RQ, RW_UPDATE_RR, RW_UPDATE_RR_REFINE = 0, 1, 2

_TORCH_DT = {torch.float64: RW_F64, torch.float32: RW_F32, torch.bfloat16: RW_BF16}
_DT_TORCH = {v: k for k, v in _TORCH_DT.items()}


class RWError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class rw_graph_desc(ct.Structure):
    _fields_ = [("ndim", ct.c_int32), ("dims", ct.c_int64 * 3), ("conn", ct.c_int32), ("dtype", ct.c_int32),
                ("weight_form", ct.c_int32), ("normalized", ct.c_int32)]


class rw_graph_view(ct.Structure):
    _fields_ = [("N", ct.c_int64), ("ndir", ct.c_int32), ("dtype", ct.c_int32), ("beta", ct.c_double),
                ("J", ct.c_void_p), ("weight", ct.c_void_p), ("scale", ct.c_void_p), ("coef", ct.c_void_p),
                ("diag", ct.c_void_p), ("dinv", ct.c_void_p), ("ghat", ct.c_void_p), ("degree", ct.c_void_p),
                ("mask", ct.c_void_p), ("comp", ct.c_void_p)]


class rw_edit(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("value", ct.c_double), ("edge_ids", ct.c_void_p), ("n", ct.c_int64),
                ("box_lo", ct.c_int64 * 3), ("box_hi", ct.c_int64 * 3)]


class rw_eig_opts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("max_iter", ct.c_int32), ("degree", ct.c_int32), ("guard", ct.c_int32),
                ("seed", ct.c_uint64), ("warm", ct.c_int32), ("q_dtype", ct.c_int32)]


class rw_eig_header(ct.Structure):
    _fields_ = [("magic", ct.c_char * 8), ("version", ct.c_int32), ("ndim", ct.c_int32), ("conn", ct.c_int32),
                ("graph_dtype", ct.c_int32), ("weight_form", ct.c_int32), ("normalized", ct.c_int32),
                ("dims", ct.c_int64 * 3), ("beta", ct.c_double), ("m", ct.c_int32), ("q_dtype", ct.c_int32),
                ("tol", ct.c_double), ("weight_hash", ct.c_uint64), ("q_bytes", ct.c_uint64),
                ("lambda_bytes", ct.c_uint64), ("reserved", ct.c_int32 * 6)]


class rw_eig_info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("n_converged", ct.c_int32), ("spmm_columns", ct.c_int64),
                ("max_residual", ct.c_double), ("seconds", ct.c_double)]


class rw_solve_info(ct.Structure):
    _fields_ = [("m_used", ct.c_int32), ("f_max", ct.c_double), ("f_worst", ct.c_double),
                ("min_pivot", ct.c_double), ("eig_probes", ct.c_int32)]


class rw_batch_image(ct.Structure):
    _fields_ = [("g", ct.c_void_p), ("Q", ct.c_void_p), ("q_dtype", ct.c_int32), ("lambda_", ct.c_void_p),
                ("m", ct.c_int32), ("S_cap", ct.c_int64), ("C_cap", ct.c_int32), ("U", ct.c_void_p)]


class rw_cg_info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("rel_residual", ct.c_double)]


_lib = None

_SIGS = {
    "rw_last_error": (ct.c_char_p, []),
    "rw_version": (ct.c_int, []),
    "rw_graph_bytes": (ct.c_int, [ct.POINTER(rw_graph_desc), ct.POINTER(ct.c_size_t)]),
    "rw_build_graph": (ct.c_int, [ct.POINTER(rw_graph_desc), ct.c_void_p, ct.c_int, ct.c_double, ct.c_void_p,
                                  ct.c_size_t, ct.c_void_p, ct.POINTER(ct.c_void_p)]),
    "rw_graph_destroy": (ct.c_int, [ct.c_void_p]),
    "rw_graph_get_view": (ct.c_int, [ct.c_void_p, ct.POINTER(rw_graph_view)]),
    "rw_graph_components": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.c_void_p]),
    "rw_edit_graph": (ct.c_int, [ct.c_void_p, ct.POINTER(rw_edit), ct.c_int, ct.c_void_p]),
    "rw_apply_laplacian": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p]),
    "rw_apply_laplacian_timed": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p,
                                            ct.c_void_p, ct.c_void_p]),
    "rw_apply_laplacian_axpby": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                            ct.c_double, ct.c_double, ct.c_double, ct.c_void_p]),
    "rw_eig_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rw_eig_opts), ct.POINTER(ct.c_size_t)]),
    "rw_precompute_eig": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rw_eig_opts), ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.POINTER(rw_eig_info)]),
    "rw_update_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rw_eig_opts),
                                             ct.POINTER(ct.c_size_t)]),
    "rw_update_eig": (ct.c_int, [ct.c_void_p, ct.POINTER(rw_edit), ct.c_int, ct.c_int, ct.POINTER(rw_eig_opts),
                                 ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                 ct.POINTER(rw_eig_info)]),
    "rw_solve_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int64, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_solve_seeds": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                                  ct.c_void_p, ct.c_int64, ct.c_int, ct.c_double, ct.c_void_p, ct.c_void_p,
                                  ct.c_size_t, ct.c_void_p, ct.POINTER(rw_solve_info)]),
    "rw_solve_seeds_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                                          ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_void_p,
                                          ct.POINTER(rw_solve_info)]),
    "rw_solve_seeds_async": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                                        ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                                        ct.c_void_p, ct.c_void_p]),
    "rw_solve_prior_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int64, ct.c_int,
                                                  ct.POINTER(ct.c_size_t)]),
    "rw_solve_seeds_prior": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                                        ct.c_void_p, ct.c_int64, ct.c_int, ct.c_double, ct.c_void_p, ct.c_int,
                                        ct.c_double, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                        ct.POINTER(rw_solve_info)]),
    "rw_priors_workspace_bytes": (ct.c_int, [ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_solve_priors_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                                   ct.POINTER(ct.c_size_t)]),
    "rw_solve_priors": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int,
                                   ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.c_void_p, ct.c_void_p,
                                   ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.POINTER(rw_solve_info)]),
    "rw_priors_from_seeds": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p,
                                        ct.c_int, ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p]),
    "rw_bank_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rw_eig_opts), ct.POINTER(ct.c_size_t)]),
    "rw_bank_select": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_void_p), ct.c_int, ct.POINTER(rw_eig_opts), ct.c_int,
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                  ct.POINTER(ct.c_int), ct.c_void_p]),
    "rw_aggregate_desc": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rw_graph_desc)]),
    "rw_aggregate_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_aggregate_graph": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_size_t,
                                      ct.c_void_p, ct.POINTER(ct.c_void_p)]),
    "rw_aggregate_basis": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p,
                                      ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "rw_aggregate_seeds": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p,
                                      ct.c_void_p, ct.POINTER(ct.c_int64)]),
    "rw_prolong": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p]),
    "rw_dense_syev_workspace_bytes": (ct.c_int, [ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_dense_syev": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_size_t,
                                 ct.c_void_p]),
    "rw_dense_syev_tridiag_workspace_bytes": (ct.c_int, [ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_dense_eig_rhs_batched_workspace_bytes": (ct.c_int, [ct.c_int, ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_dense_eig_rhs_batched": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int,
                                            ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "rw_dense_syev_tridiag": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_size_t,
                                         ct.c_void_p]),
    "rw_dense_lu_solve": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p]),
    "rw_eig_save": (ct.c_int, [ct.c_void_p, ct.c_char_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_double,
                               ct.c_void_p]),
    "rw_eig_read_header": (ct.c_int, [ct.c_char_p, ct.c_void_p]),
    "rw_eig_load": (ct.c_int, [ct.c_void_p, ct.c_char_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                               ct.c_void_p]),
    "rw_cg_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_convert_block": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int64, ct.c_int, ct.c_void_p]),
    "rw_project_workspace_bytes": (ct.c_int, [ct.c_int64, ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_project_basis": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_int, ct.c_void_p,
                                    ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "rw_cg_solve_rhs": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_double,
                                   ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                   ct.POINTER(rw_cg_info)]),
    "rw_graph_set_scale": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "rw_grad_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_size_t)]),
    "rw_grad_edges": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "rw_spectral_workspace_bytes": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_spectral_apply": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int,
                                     ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "rw_batch_workspace_bytes": (ct.c_int, [ct.POINTER(rw_batch_image), ct.c_int, ct.POINTER(ct.c_size_t)]),
    "rw_batch_create": (ct.c_int, [ct.POINTER(rw_batch_image), ct.c_int, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                   ct.POINTER(ct.c_void_p)]),
    "rw_batch_destroy": (ct.c_int, [ct.c_void_p]),
    "rw_batch_info": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                                 ct.POINTER(ct.c_double)]),
    "rw_batch_set_seeds": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "rw_batch_enqueue": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "rw_batch_status": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double), ct.c_void_p]),
    "rw_cg_solve": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_double, ct.c_int,
                               ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                               ct.POINTER(rw_cg_info)]),
}


def lib():
    """The loaded librw (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1607_04174_amd.build`")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGS)


def _check(status: int):
    if status != RW_OK:
        raise RWError(status, lib().rw_last_error().decode(errors="replace"))


def _stream(device=None):
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(0)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------------------------
# graph
# ---------------------------------------------------------------------------------------------
class Graph:
    """Weighted image graph (Sec. II-A eq. (2)) living in a device buffer owned by this object."""

    def __init__(self, J: torch.Tensor, dims: Sequence[int], conn: int, beta: float, dtype=torch.float32,
                 weight_form: str = "squared", normalized: bool = True):
        dims = tuple(int(v) for v in dims) + (1,) * (3 - len(dims))
        self.dims = dims
        self.ndim = 2 if dims[2] == 1 else 3
        self.N = dims[0] * dims[1] * dims[2]
        self.conn = conn
        self.dtype = dtype
        self.normalized = normalized
        self.device = J.device
        d = rw_graph_desc()
        d.ndim = self.ndim
        for k in range(3):
            d.dims[k] = dims[k]
        d.conn = conn
        d.dtype = _TORCH_DT[dtype]
        d.weight_form = 0 if weight_form == "squared" else 1
        d.normalized = 1 if normalized else 0
        self._desc = d
        nb = ct.c_size_t()
        _check(lib().rw_graph_bytes(ct.byref(d), ct.byref(nb)))
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=J.device)
        J = J.contiguous()
        if J.numel() != self.N or J.dtype not in (torch.float32, torch.float64):
            raise ValueError("J must hold N float32/float64 values")
        self._J = J
        h = ct.c_void_p()
        _check(lib().rw_build_graph(ct.byref(d), _ptr(J), _TORCH_DT[J.dtype], float(beta), _ptr(self.buf), nb.value,
                                    _stream(J.device), ct.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rw_graph_destroy(h)
            self.handle = None

    def view(self):
        """dict of torch tensors aliasing the graph's device arrays."""
        v = rw_graph_view()
        _check(lib().rw_graph_get_view(self.handle, ct.byref(v)))
        base = self.buf.data_ptr()
        N, nd = v.N, v.ndir
        tdt = _DT_TORCH[v.dtype]
        es = torch.empty((), dtype=tdt).element_size()

        def sl(ptr, count, dt, esz):
            off = ptr - base
            return self.buf[off: off + count * esz].view(dt)

        return {"beta": v.beta, "J": sl(v.J, N, torch.float64, 8),
                "weight": sl(v.weight, nd * N, torch.float64, 8).view(nd, N),
                "scale": sl(v.scale, nd * N, torch.float64, 8).view(nd, N),
                "coef": sl(v.coef, nd * N, tdt, es).view(nd, N), "diag": sl(v.diag, N, tdt, es),
                "dinv": sl(v.dinv, N, tdt, es), "ghat": sl(v.ghat, N, tdt, es),
                "degree": sl(v.degree, N, torch.float64, 8), "mask": sl(v.mask, N, torch.uint8, 1),
                "comp": sl(v.comp, N, torch.int64, 8)}

    def components(self):
        """(number of components, (N,) int64 tensor of component roots) over edges with w >= 1e-30."""
        nc = ct.c_int64()
        _check(lib().rw_graph_components(self.handle, ct.byref(nc), _stream(self.device)))
        return nc.value, self.view()["comp"]


def build_graph(J, dims, conn, beta, dtype=torch.float32, weight_form="squared", normalized=True) -> Graph:
    return Graph(J, dims, conn, beta, dtype, weight_form, normalized)


def _edits(edits):
    arr = (rw_edit * max(1, len(edits)))()
    keep = []
    for k, e in enumerate(edits):
        kind = {"set_beta": RW_EDIT_SET_BETA, "scale_edges": RW_EDIT_SCALE_EDGES, "scale_box": RW_EDIT_SCALE_BOX,
                "remove_edges": RW_EDIT_REMOVE_EDGES}[e.kind]
        arr[k].kind = kind
        arr[k].value = float(e.value)
        if e.edge_ids is not None:
            ids = np.ascontiguousarray(np.asarray(e.edge_ids, dtype=np.int64))
            keep.append(ids)
            arr[k].edge_ids = ids.ctypes.data
            arr[k].n = ids.size
        lo = tuple(e.box_lo) + (0,) * (3 - len(e.box_lo))
        hi = tuple(e.box_hi) + (1,) * (3 - len(e.box_hi))
        for q in range(3):
            arr[k].box_lo[q] = int(lo[q])
            arr[k].box_hi[q] = int(hi[q])
    return arr, keep


def edit_graph(g: Graph, edits) -> None:
    """Apply edits (objects with kind, value, box_lo, box_hi, edge_ids) in order."""
    arr, keep = _edits(edits)
    _check(lib().rw_edit_graph(g.handle, arr, len(edits), _stream(g.device)))


def apply_laplacian(g: Graph, X: torch.Tensor, Y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Y = op X for X of shape (b, N) (each row one vector, i.e. column-major N x b)."""
    X = X.contiguous()
    b = X.numel() // g.N
    if Y is None:
        Y = torch.empty_like(X)
    _check(lib().rw_apply_laplacian(g.handle, _ptr(X), _ptr(Y), b, _stream(g.device)))
    return Y


def apply_laplacian_timed(g: Graph, X: torch.Tensor, Y: torch.Tensor, start, stop) -> torch.Tensor:
    """apply_laplacian with the operator kernel's own start and end recorded into two torch.cuda.Event
    objects (enable_timing=True); start.elapsed_time(stop) is then that dispatch's duration."""
    b = X.numel() // g.N
    for e in (start, stop):
        if not e.cuda_event:                       # torch creates its events lazily, on the first record
            e.record(torch.cuda.current_stream(g.device))
    _check(lib().rw_apply_laplacian_timed(g.handle, _ptr(X), _ptr(Y), b, _stream(g.device),
                                          ct.c_void_p(start.cuda_event), ct.c_void_p(stop.cuda_event)))
    return Y


def apply_laplacian_axpby(g: Graph, X, Y, Z, alpha, beta, gamma):
    b = X.numel() // g.N
    _check(lib().rw_apply_laplacian_axpby(g.handle, _ptr(X), _ptr(Y), _ptr(Z), b, float(alpha), float(beta),
                                          float(gamma), _stream(g.device)))
    return Y


# ---------------------------------------------------------------------------------------------
# eigenpairs and updates
# ---------------------------------------------------------------------------------------------
def _eig_opts(tol, max_iter, degree, guard, seed, warm, q_dtype):
    o = rw_eig_opts()
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.degree = int(degree)
    o.guard = int(guard)
    o.seed = int(seed)
    o.warm = int(warm)
    o.q_dtype = _TORCH_DT[q_dtype]
    return o


def precompute_eig(g: Graph, m: int, tol: float = 1e-5, max_iter: int = 200, degree: int = 0, guard: int = 0,
                   seed: int = 0, q_dtype=None, Q: Optional[torch.Tensor] = None, warm: bool = False,
                   raise_on_noconv: bool = True):
    """The m smallest eigenpairs.  Returns (Q (m, N) tensor, lambda (m,) float64 tensor, info dict)."""
    q_dtype = q_dtype or g.dtype
    o = _eig_opts(tol, max_iter, degree, guard, seed, warm, q_dtype)
    if Q is None:
        Q = torch.empty((m, g.N), dtype=q_dtype, device=g.device)
    lam = torch.empty(m, dtype=torch.float64, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_eig_workspace_bytes(g.handle, m, ct.byref(o), ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    info = rw_eig_info()
    st = lib().rw_precompute_eig(g.handle, m, ct.byref(o), _ptr(Q), _ptr(lam), _ptr(work), nb.value,
                                 _stream(g.device), ct.byref(info))
    if st != RW_OK and not (st == RW_ENOCONV and not raise_on_noconv):
        _check(st)
    return Q, lam, {"iters": info.iters, "n_converged": info.n_converged, "spmm_columns": info.spmm_columns,
                    "max_residual": info.max_residual, "seconds": info.seconds, "status": st}


def update_eig(g: Graph, edits, Q: torch.Tensor, lam: torch.Tensor, mode: int = RW_UPDATE_RR, tol: float = 1e-5,
               max_iter: int = 200, degree: int = 0, guard: int = 0, raise_on_noconv: bool = True):
    """Apply edits to g and update (Q, lam) in place by `mode`.  Returns the info dict."""
    m = Q.shape[0]
    o = _eig_opts(tol, max_iter, degree, guard, 0, 1, Q.dtype)
    nb = ct.c_size_t()
    _check(lib().rw_update_workspace_bytes(g.handle, m, ct.byref(o), ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    arr, keep = _edits(edits)
    info = rw_eig_info()
    st = lib().rw_update_eig(g.handle, arr, len(edits), int(mode), ct.byref(o), _ptr(Q), _ptr(lam), m, _ptr(work),
                             nb.value, _stream(g.device), ct.byref(info))
    if st != RW_OK and not (st == RW_ENOCONV and not raise_on_noconv):
        _check(st)
    return {"iters": info.iters, "n_converged": info.n_converged, "spmm_columns": info.spmm_columns,
            "max_residual": info.max_residual, "seconds": info.seconds, "status": st}


def aggregate(g: Graph, s: int) -> Graph:
    """The graph of s x s (x s) blocks of g (rw_aggregate_graph): same connectivity, summed crossing weights."""
    d = rw_graph_desc()
    _check(lib().rw_aggregate_desc(g.handle, int(s), ct.byref(d)))
    nb, nw = ct.c_size_t(), ct.c_size_t()
    _check(lib().rw_graph_bytes(ct.byref(d), ct.byref(nb)))
    _check(lib().rw_aggregate_workspace_bytes(g.handle, int(s), ct.byref(nw)))
    c = Graph.__new__(Graph)
    c.dims = tuple(int(d.dims[k]) for k in range(3))
    c.ndim, c.N, c.conn, c.dtype, c.normalized, c.device = g.ndim, c.dims[0] * c.dims[1] * c.dims[2], g.conn, \
        g.dtype, g.normalized, g.device
    c._desc = d
    c.buf = torch.empty(nb.value, dtype=torch.uint8, device=g.device)
    c._work = torch.empty(nw.value, dtype=torch.uint8, device=g.device)
    h = ct.c_void_p()
    _check(lib().rw_aggregate_graph(g.handle, int(s), _ptr(c.buf), nb.value, _ptr(c._work), nw.value,
                                    _stream(g.device), ct.byref(h)))
    c.handle = h
    return c


def aggregate_basis(g: Graph, coarse: Graph, s: int, Q: torch.Tensor, lam_out: bool = True, tol: float = 1e-5):
    """Eq. (33) transfer of Q (m, N) to the blocks, then the diagonal update on the aggregated graph
    (Gram-Schmidt in order against its null vector, normalized-cut values).  Returns (Q_bar (m, N_bar), lambda)."""
    m = Q.shape[0]
    Q = Q.contiguous()
    Qc = torch.empty((m, coarse.N), dtype=Q.dtype, device=Q.device)
    nw = ct.c_size_t()
    _check(lib().rw_aggregate_workspace_bytes(g.handle, int(s), ct.byref(nw)))
    work = _workspace(nw.value, g.device)
    _check(lib().rw_aggregate_basis(g.handle, int(s), _ptr(Q), _TORCH_DT[Q.dtype], m, _ptr(Qc), _ptr(work),
                                    nw.value, _stream(g.device)))
    lam = torch.empty(m, dtype=torch.float64, device=Q.device)
    update_eig(coarse, [], Qc, lam, mode=RW_UPDATE_DIAG_RQ, tol=tol)
    return Qc, lam


def aggregate_seeds(g: Graph, s: int, seed_node, seed_label):
    """Seeds moved to their blocks (sorted, distinct; conflicting labels in a block raise RWError)."""
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    on = np.empty(max(1, nodes.size), np.int64)
    ol = np.empty(max(1, nodes.size), np.int32)
    n = ct.c_int64()
    _check(lib().rw_aggregate_seeds(g.handle, int(s), ct.c_void_p(nodes.ctypes.data), ct.c_void_p(labels.ctypes.data),
                                    nodes.size, ct.c_void_p(on.ctypes.data), ct.c_void_p(ol.ctypes.data), ct.byref(n)))
    return on[:n.value].copy(), ol[:n.value].copy()


def prolong(g: Graph, s: int, Uc: torch.Tensor) -> torch.Tensor:
    """U_x = U_bar of x's block (Uc: (C, N_bar) of g's dtype) -> (C, N)."""
    C = Uc.shape[0]
    U = torch.empty((C, g.N), dtype=Uc.dtype, device=Uc.device)
    _check(lib().rw_prolong(g.handle, int(s), _ptr(Uc.contiguous()), C, _ptr(U), _stream(g.device)))
    return U


def bank_select(g: Graph, bank, tol: float = 1e-5):
    """Choose among bases (a list of (m, N) tensors of the graph's dtype) for g's current operator.
    Returns (index, Q (m, N) updated copy, lambda_hat (m,), quotient sums per basis)."""
    m = bank[0].shape[0]
    dt = bank[0].dtype
    for Q in bank:
        assert Q.shape == bank[0].shape and Q.dtype == dt and Q.is_contiguous()
    o = _eig_opts(tol, 1, 0, 0, 0, 1, dt)
    nb = ct.c_size_t()
    _check(lib().rw_bank_workspace_bytes(g.handle, m, ct.byref(o), ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    ptrs = (ct.c_void_p * len(bank))(*[Q.data_ptr() for Q in bank])
    Q_out = torch.empty_like(bank[0])
    lam = torch.empty(m, dtype=torch.float64, device=g.device)
    chosen = ct.c_int(-1)
    traces = (ct.c_double * len(bank))()
    _check(lib().rw_bank_select(g.handle, ptrs, len(bank), ct.byref(o), m, _ptr(Q_out), _ptr(lam), _ptr(work),
                                nb.value, _stream(g.device), ct.byref(chosen), traces))
    return chosen.value, Q_out, lam, list(traces)


# ---------------------------------------------------------------------------------------------
# online solve
# ---------------------------------------------------------------------------------------------
class SolveWorkspace:
    """Reusable device workspace for solve_seeds (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = _workspace(nbytes, device)
        return self.buf


def solve_seeds(g: Graph, Q: torch.Tensor, lam: torch.Tensor, seed_node, seed_label, C: int, eps: float = 0.0,
                m_avail: Optional[int] = None, U: Optional[torch.Tensor] = None,
                workspace: Optional[SolveWorkspace] = None):
    """Label probabilities (C, N) in the graph's dtype from the eigenbasis.  Returns (U, info dict)."""
    m_avail = Q.shape[0] if m_avail is None else int(m_avail)
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    S = nodes.size
    if U is None:
        U = torch.empty((C, g.N), dtype=g.dtype, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_solve_workspace_bytes(g.handle, m_avail, max(S, 1), C, ct.byref(nb)))
    work = (workspace or SolveWorkspace()).get(nb.value, g.device)
    info = rw_solve_info()
    _check(lib().rw_solve_seeds(g.handle, *_qarg(Q), _ptr(lam), m_avail,
                                ct.c_void_p(nodes.ctypes.data), ct.c_void_p(labels.ctypes.data), S, C, float(eps),
                                _ptr(U), _ptr(work), work.numel(), _stream(g.device), ct.byref(info)))
    return U, {"m_used": info.m_used, "f_max": info.f_max, "f_worst": info.f_worst, "min_pivot": info.min_pivot,
               "eig_probes": info.eig_probes}


def _header_dict(h: rw_eig_header) -> dict:
    return {"version": h.version, "ndim": h.ndim, "conn": h.conn, "graph_dtype": h.graph_dtype,
            "weight_form": h.weight_form, "normalized": h.normalized, "dims": tuple(h.dims), "beta": h.beta,
            "m": h.m, "q_dtype": h.q_dtype, "tol": h.tol, "weight_hash": h.weight_hash}


def eig_save(g: Graph, path: str, Q: torch.Tensor, lam: torch.Tensor, tol: float = 0.0) -> None:
    """Write the eigenpairs (Q: (m, N) = column-major N x m, or a PairBasis; lam: (m,) float64) of graph g
    to `path`."""
    if not isinstance(Q, PairBasis):
        Q = Q.contiguous()
    lam = lam.to(torch.float64).contiguous()
    _check(lib().rw_eig_save(g.handle, os.fsencode(path), *_qarg(Q), _ptr(lam), Q.shape[0], float(tol),
                             _stream(g.device)))


def eig_read_header(path: str) -> dict:
    """The header of a checkpoint (host only)."""
    h = rw_eig_header()
    _check(lib().rw_eig_read_header(os.fsencode(path), ct.byref(h)))
    return _header_dict(h)


def eig_load(g: Graph, path: str, m: Optional[int] = None):
    """Load the first m pairs (all by default) of a checkpoint written for g's current operator.
    Returns (Q (m, N) tensor, or a PairBasis for the pair form; lam (m,); header dict)."""
    hd = eig_read_header(path)
    m = hd["m"] if m is None else int(m)
    pair = hd["q_dtype"] == RW_BF16_PAIR
    if pair:
        Q = PairBasis(torch.empty((RW_PAIR_COLS + m, g.N), dtype=torch.bfloat16, device=g.device))
    else:
        Q = torch.empty((m, g.N), dtype=_DT_TORCH[hd["q_dtype"]], device=g.device)
    lam = torch.empty(m, dtype=torch.float64, device=g.device)
    h = rw_eig_header()
    _check(lib().rw_eig_load(g.handle, os.fsencode(path), _qarg(Q)[0], hd["q_dtype"], _ptr(lam), m,
                             _stream(g.device), ct.byref(h)))
    return Q, lam, _header_dict(h)


def solve_seeds_noalloc(g: Graph, Q: torch.Tensor, lam: torch.Tensor, seed_node, seed_label, C: int,
                        m: Optional[int] = None, U: Optional[torch.Tensor] = None):
    """solve_seeds with a fixed m through rw_solve_seeds_noalloc, whose workspace is the library's own device
    array (the call allocates nothing; U is allocated here only when not given).  Returns (U, info dict)."""
    m = Q.shape[0] if m is None else int(m)
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    if U is None:
        U = torch.empty((C, g.N), dtype=g.dtype, device=g.device)
    info = rw_solve_info()
    _check(lib().rw_solve_seeds_noalloc(g.handle, *_qarg(Q), _ptr(lam), m,
                                        ct.c_void_p(nodes.ctypes.data), ct.c_void_p(labels.ctypes.data), nodes.size,
                                        C, _ptr(U), _stream(g.device), ct.byref(info)))
    return U, {"m_used": info.m_used, "min_pivot": info.min_pivot}


def solve_seeds_prior(g: Graph, Q, lam: torch.Tensor, seed_node, seed_label, C: int, gamma: float,
                      prior: torch.Tensor, eps: float = 0.0, r: int = 4, m_avail: Optional[int] = None,
                      U: Optional[torch.Tensor] = None, workspace: Optional[SolveWorkspace] = None):
    """Label probabilities (C, N) with priors (C, N) (float64 or float32) and weight gamma > 0; eps > 0 chooses m
    from the priors (one label in every r^d).  Returns (U, info dict)."""
    m_avail = Q.shape[0] if m_avail is None else int(m_avail)
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    prior = prior.contiguous()
    assert tuple(prior.shape) == (C, g.N) and prior.dtype in (torch.float64, torch.float32)
    if U is None:
        U = torch.empty((C, g.N), dtype=g.dtype, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_solve_prior_workspace_bytes(g.handle, m_avail, max(nodes.size, 1), C, ct.byref(nb)))
    work = (workspace or SolveWorkspace()).get(nb.value, g.device)
    info = rw_solve_info()
    _check(lib().rw_solve_seeds_prior(g.handle, *_qarg(Q), _ptr(lam), m_avail, ct.c_void_p(nodes.ctypes.data),
                                      ct.c_void_p(labels.ctypes.data), nodes.size, C, float(gamma), _ptr(prior),
                                      _TORCH_DT[prior.dtype], float(eps), int(r), _ptr(U), _ptr(work), work.numel(),
                                      _stream(g.device), ct.byref(info)))
    return U, {"m_used": info.m_used, "g_max": info.f_max, "g_worst": info.f_worst, "min_pivot": info.min_pivot}


def solve_priors(g: Graph, Q: torch.Tensor, lam: torch.Tensor, prior: torch.Tensor, gamma: float,
                 eps: float = 0.0, r: int = 4, m_avail: Optional[int] = None, want_U: bool = True,
                 want_labels: bool = False, U: Optional[torch.Tensor] = None,
                 workspace: Optional[SolveWorkspace] = None):
    """The walker driven by priors alone (no seeds), for label counts up to thousands: prior (C, N) of float64 /
    float32 (FP64 or FP32 basis) or bfloat16 / float32 (BF16 basis).  Returns (U or None, labels or None,
    prob or None, info dict); labels (N,) int32 are the smallest labels of largest probability per voxel."""
    m_avail = Q.shape[0] if m_avail is None else int(m_avail)
    prior = prior.contiguous()
    C = prior.shape[0]
    assert prior.shape[1] == g.N and Q.dtype in _TORCH_DT and prior.dtype in _TORCH_DT
    if want_U and U is None:
        U = torch.empty((C, g.N), dtype=g.dtype, device=g.device)
    lab = torch.empty(g.N, dtype=torch.int32, device=g.device) if want_labels else None
    prob = torch.empty(g.N, dtype=g.dtype, device=g.device) if want_labels else None
    nb = ct.c_size_t()
    _check(lib().rw_solve_priors_workspace_bytes(g.handle, _TORCH_DT[Q.dtype], m_avail, C, int(r),
                                                 int(want_labels), ct.byref(nb)))
    work = (workspace or SolveWorkspace()).get(nb.value, g.device)
    info = rw_solve_info()
    _check(lib().rw_solve_priors(g.handle, _ptr(Q.contiguous()), _TORCH_DT[Q.dtype], _ptr(lam), m_avail, _ptr(prior),
                                 _TORCH_DT[prior.dtype], C, float(gamma), float(eps), int(r),
                                 _ptr(U if want_U else None), _ptr(lab), _ptr(prob), _ptr(work), work.numel(),
                                 _stream(g.device),
                                 ct.byref(info)))
    return (U if want_U else None), lab, prob, {"m_used": info.m_used, "g_max": info.f_max, "g_worst": info.f_worst}


def priors_from_seeds(g: Graph, seed_node, seed_label, C: int, dtype=torch.float32) -> torch.Tensor:
    """(C, N) Gaussian-fit priors from the seeds' intensities (rw_priors_from_seeds)."""
    nodes = torch.as_tensor(np.asarray(seed_node, dtype=np.int64)).to(g.device)
    labels = torch.as_tensor(np.asarray(seed_label, dtype=np.int32)).to(g.device)
    out = torch.empty((C, g.N), dtype=dtype, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_priors_workspace_bytes(C, ct.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device=g.device)
    status = torch.full((1,), 99, dtype=torch.int32, device=g.device)
    _check(lib().rw_priors_from_seeds(g.handle, _ptr(nodes), _ptr(labels), nodes.numel(), C, _ptr(out),
                                      _TORCH_DT[dtype], _ptr(work), work.numel(), _ptr(status), _stream(g.device)))
    st = int(status.item())
    if st != RW_OK:
        raise RWError(st, "a seed is out of range")
    return out


def solve_workspace_bytes(g: Graph, m: int, S: int, C: int) -> int:
    nb = ct.c_size_t()
    _check(lib().rw_solve_workspace_bytes(g.handle, int(m), max(int(S), 1), int(C), ct.byref(nb)))
    return nb.value


def solve_seeds_async(g: Graph, Q: torch.Tensor, lam: torch.Tensor, seed_node: torch.Tensor,
                      seed_label: torch.Tensor, C: int, U: torch.Tensor, work: torch.Tensor, status: torch.Tensor,
                      m: Optional[int] = None, stream=None) -> None:
    """rw_solve_seeds_async: enqueue a fixed-m solve whose seeds (int64 nodes, ascending and distinct, and
    int32 labels) are device tensors; nothing is read back and nothing waits, so the call can be captured
    into a HIP graph.  status (a device int32 tensor) receives RW_OK or an RW_E* code when the work runs;
    work is a byte tensor of at least solve_workspace_bytes(g, m, S, C)."""
    m = Q.shape[0] if m is None else int(m)
    assert seed_node.dtype == torch.int64 and seed_label.dtype == torch.int32 and status.dtype == torch.int32
    assert seed_node.is_contiguous() and seed_label.is_contiguous() and U.is_contiguous() and work.is_contiguous()
    assert seed_node.numel() == seed_label.numel() and U.dtype == g.dtype and tuple(U.shape) == (C, g.N)
    s = _stream(g.device) if stream is None else ct.c_void_p(stream.cuda_stream)
    _check(lib().rw_solve_seeds_async(g.handle, *_qarg(Q), _ptr(lam), m, _ptr(seed_node),
                                      _ptr(seed_label), seed_node.numel(), int(C), _ptr(U), _ptr(work),
                                      work.numel() * work.element_size(), _ptr(status), s))


def cg_solve(g: Graph, seed_node, seed_label, C: int, tol: float = 1e-12, max_iter: int = 100000,
             U0: Optional[torch.Tensor] = None, raise_on_noconv: bool = True):
    """Exact random walker by FP64 CG.  Returns (U (C, N) float64, info dict)."""
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    if U0 is not None:
        U = U0.to(torch.float64).contiguous().clone()
    else:
        U = torch.empty((C, g.N), dtype=torch.float64, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_cg_workspace_bytes(g.handle, C, ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    info = rw_cg_info()
    st = lib().rw_cg_solve(g.handle, ct.c_void_p(nodes.ctypes.data), ct.c_void_p(labels.ctypes.data), nodes.size, C,
                           float(tol), int(max_iter), 1 if U0 is not None else 0, _ptr(U), _ptr(work), nb.value,
                           _stream(g.device), ct.byref(info))
    if st != RW_OK and not (st == RW_ENOCONV and not raise_on_noconv):
        _check(st)
    return U, {"iters": info.iters, "rel_residual": info.rel_residual, "status": st}


# ---------------------------------------------------------------------------------------------
# dense building blocks
# ---------------------------------------------------------------------------------------------
def dense_syev(A: torch.Tensor, vectors: bool = True):
    """Eigenpairs of a batch of symmetric FP64 matrices A (count, n, n) (each read as column-major).
    Returns (w (count, n), V (count, n, n) with V[b, j] the j-th eigenvector, or None)."""
    A = A.contiguous()
    count, n = A.shape[0], A.shape[1]
    w = torch.empty((count, n), dtype=torch.float64, device=A.device)
    V = torch.empty((count, n, n), dtype=torch.float64, device=A.device) if vectors else None
    nb = ct.c_size_t()
    _check(lib().rw_dense_syev_workspace_bytes(n, count, ct.byref(nb)))
    work = _workspace(nb.value, A.device)
    _check(lib().rw_dense_syev(_ptr(A), _ptr(w), _ptr(V), n, count, _ptr(work), nb.value, _stream(A.device)))
    return w, V


def dense_syev_tridiag(A: torch.Tensor):
    """Eigenpairs of one symmetric FP64 matrix A (n, n) (read as column-major) through its tridiagonal form
    (3 <= n <= 199).  Returns (w (n,), V (n, n) with V[j] the j-th eigenvector).  Raises RWError with
    RW_ENOCONV when eigenvalues are too close for inverse iteration."""
    A = A.contiguous()
    n = A.shape[0]
    w = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty((n, n), dtype=torch.float64, device=A.device)
    nb = ct.c_size_t()
    _check(lib().rw_dense_syev_tridiag_workspace_bytes(n, ct.byref(nb)))
    work = _workspace(nb.value, A.device)
    _check(lib().rw_dense_syev_tridiag(_ptr(A), _ptr(w), _ptr(V), n, _ptr(work), nb.value, _stream(A.device)))
    return w, V


def dense_eig_rhs_batched(A: torch.Tensor, sizes, R: torch.Tensor):
    """Eigenvalues and rotated right-hand sides of a batch of symmetric FP64 matrices A (count, ld, ld),
    each read column-major with order sizes[b], right-hand sides R (count, nrhs, ld) (column-major ld x nrhs
    per matrix).  Returns (w (count, ld), R' (count, nrhs, ld)) with R'_b = V_b^T R_b and zero rows beyond
    sizes[b].  Raises RWError with RW_ENOCONV when some matrix has clustered eigenvalues."""
    A = A.contiguous()
    count, ld = A.shape[0], A.shape[1]
    nrhs = R.shape[1]
    Rout = R.clone().contiguous()
    w = torch.empty((count, ld), dtype=torch.float64, device=A.device)
    sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    nb = ct.c_size_t()
    _check(lib().rw_dense_eig_rhs_batched_workspace_bytes(int(sz.max()), count, nrhs, ct.byref(nb)))
    work = _workspace(nb.value, A.device)
    _check(lib().rw_dense_eig_rhs_batched(_ptr(A), ld, ct.c_void_p(sz.ctypes.data), count, _ptr(Rout), nrhs, _ptr(w),
                                          _ptr(work), nb.value, _stream(A.device)))
    return w, Rout


def dense_lu_solve(A: torch.Tensor, B: torch.Tensor):
    """Solve A X = B (A (n, n), B (nrhs, n): both column-major views).  Returns (X, stat)."""
    A = A.clone().contiguous()
    X = B.clone().contiguous()
    n = A.shape[0]
    nrhs = X.numel() // n
    stat = torch.empty(1, dtype=torch.float64, device=A.device)
    _check(lib().rw_dense_lu_solve(_ptr(A), n, _ptr(X), nrhs, _ptr(stat), _stream(A.device)))
    return X, float(stat.item())


# ---------------------------------------------------------------------------------------------
# differentiation of the exact random walker
# ---------------------------------------------------------------------------------------------
def cg_solve_rhs(g: Graph, seed_node, seed_label, C: int, B: torch.Tensor, tol: float = 1e-12,
                 max_iter: int = 100000, X0: Optional[torch.Tensor] = None, raise_on_noconv: bool = True):
    """Solve L_n X_n = B_n (X zero on seeds).  B, X: (C, N) float64.  Returns (X, info)."""
    nodes = np.ascontiguousarray(np.asarray(seed_node, dtype=np.int64))
    labels = np.ascontiguousarray(np.asarray(seed_label, dtype=np.int32))
    B = B.to(torch.float64).contiguous()
    X = X0.to(torch.float64).contiguous().clone() if X0 is not None else torch.empty_like(B)
    nb = ct.c_size_t()
    _check(lib().rw_cg_workspace_bytes(g.handle, C, ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    info = rw_cg_info()
    st = lib().rw_cg_solve_rhs(g.handle, ct.c_void_p(nodes.ctypes.data), ct.c_void_p(labels.ctypes.data), nodes.size,
                               C, _ptr(B), float(tol), int(max_iter), 1 if X0 is not None else 0, _ptr(X), _ptr(work),
                               nb.value, _stream(g.device), ct.byref(info))
    if st != RW_OK and not (st == RW_ENOCONV and not raise_on_noconv):
        _check(st)
    return X, {"iters": info.iters, "rel_residual": info.rel_residual, "status": st}


def graph_set_scale(g: Graph, scale: torch.Tensor) -> None:
    scale = scale.to(torch.float64).contiguous()
    _check(lib().rw_graph_set_scale(g.handle, _ptr(scale), _stream(g.device)))


def grad_edges(g: Graph, U: torch.Tensor, A: torch.Tensor):
    """(dw (ndir, N), dJ (N,), dbeta (scalar tensor), ds (ndir, N)) for the exact solution U and adjoint A."""
    C = U.shape[0]
    nd = {(2, 4): 2, (2, 8): 4, (3, 6): 3}[(g.ndim, g.conn)]
    dw = torch.empty((nd, g.N), dtype=torch.float64, device=g.device)
    ds = torch.empty_like(dw)
    dJ = torch.empty(g.N, dtype=torch.float64, device=g.device)
    db = torch.empty((), dtype=torch.float64, device=g.device)
    nb = ct.c_size_t()
    _check(lib().rw_grad_workspace_bytes(g.handle, ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    _check(lib().rw_grad_edges(g.handle, _ptr(U.contiguous()), _ptr(A.contiguous()), C, _ptr(dw), _ptr(dJ), _ptr(db),
                               _ptr(ds), _ptr(work), nb.value, _stream(g.device)))
    return dw, dJ, db, ds


def spectral_apply(g: Graph, Q: torch.Tensor, lam: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """X = S Q' Lambda'^{-1} Q'^T S B (truncated pseudo-inverse through the eigenbasis)."""
    m = Q.shape[0]
    C = B.shape[0]
    B = B.to(torch.float64).contiguous()
    X = torch.empty_like(B)
    nb = ct.c_size_t()
    _check(lib().rw_spectral_workspace_bytes(g.handle, m, C, ct.byref(nb)))
    work = _workspace(nb.value, g.device)
    _check(lib().rw_spectral_apply(g.handle, _ptr(Q.contiguous()), _ptr(lam), m, _ptr(B), C, _ptr(X), _ptr(work),
                                   nb.value, _stream(g.device)))
    return X


class RandomWalkerFn(torch.autograd.Function):
    """U = exact random walker probabilities (C, N) as a function of the intensities J (N,), beta (scalar
    tensor) and per-edge scales s (ndir, N).  Forward: FP64 CG started from the fast (eigenbasis) solution
    when (Q, lam) are given.  Backward: the adjoint system L_n A = dl/dU by CG started from the spectral
    pseudo-inverse through the same eigenbasis, then the edge-gradient kernel.  Only U is kept for the
    backward pass (no CG iterates)."""

    @staticmethod
    def forward(ctx, J, beta, scale, dims, conn, seed_node, seed_label, C, Q=None, lam=None, tol=1e-12,
                normalized=True):
        g = Graph(J.detach().to(torch.float64), dims, conn, float(beta), dtype=torch.float64, normalized=normalized)
        graph_set_scale(g, scale.detach())
        U0 = None
        if Q is not None:
            U0, _ = solve_seeds(g, Q, lam, seed_node, seed_label, C)
        U, info = cg_solve(g, seed_node, seed_label, C, tol=tol, U0=U0)
        ctx.g = g
        ctx.seeds = (seed_node, seed_label, C)
        ctx.basis = (Q, lam)
        ctx.tol = tol
        ctx.cg_iters = info["iters"]
        ctx.save_for_backward(U)
        return U

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        g = ctx.g
        seed_node, seed_label, C = ctx.seeds
        Q, lam = ctx.basis
        X0 = spectral_apply(g, Q, lam, gU) if Q is not None and Q.dtype == torch.float64 else None
        A, info = cg_solve_rhs(g, seed_node, seed_label, C, gU, tol=ctx.tol, X0=X0)
        dw, dJ, db, ds = grad_edges(g, U, A)
        return dJ, db, ds, None, None, None, None, None, None, None, None, None


def random_walker(J, beta, scale, dims, conn, seed_node, seed_label, C, Q=None, lam=None, tol=1e-12,
                  normalized=True):
    """Differentiable exact random walker (see RandomWalkerFn)."""
    return RandomWalkerFn.apply(J, beta, scale, dims, conn, seed_node, seed_label, C, Q, lam, tol, normalized)


# ---------------------------------------------------------------------------------------------
# precision form
# ---------------------------------------------------------------------------------------------
class PairBasis:
    """The BF16 pair form of an eigenbasis: `data` is a (RW_PAIR_COLS + m, N) bfloat16 tensor (column-major
    N x (RW_PAIR_COLS + m)) holding the rounding remainders of columns 1 .. RW_PAIR_COLS, then the plain BF16
    copy.  Accepted wherever a basis Q of shape (m, N) is."""

    def __init__(self, data: torch.Tensor):
        if data.dtype != torch.bfloat16 or data.dim() != 2 or data.shape[0] <= RW_PAIR_COLS:
            raise ValueError("a pair form is a (RW_PAIR_COLS + m, N) bfloat16 tensor")
        self.data = data.contiguous()

    @property
    def shape(self):
        return (self.data.shape[0] - RW_PAIR_COLS, self.data.shape[1])

    @property
    def device(self):
        return self.data.device

    def plain(self) -> torch.Tensor:
        """The plain BF16 block (m, N) (a view)."""
        return self.data[RW_PAIR_COLS:]

    def value(self) -> torch.Tensor:
        """The basis the pair form represents, hi + lo, as float64 (m, N) (analysis and tests)."""
        v = self.plain().double()
        k = min(RW_PAIR_COLS, v.shape[0] - 1)
        v[1:1 + k] += self.data[:k].double()
        return v


def _qarg(Q):
    """(pointer, dtype code) of a basis argument: a tensor or a PairBasis."""
    if isinstance(Q, PairBasis):
        return _ptr(Q.data), RW_BF16_PAIR
    return _ptr(Q), _TORCH_DT[Q.dtype]


def to_pair(Q: torch.Tensor) -> PairBasis:
    """The BF16 pair form of a float64 / float32 basis Q (m, N), made by the library."""
    Q = Q.contiguous()
    m, N = Q.shape
    out = torch.empty((RW_PAIR_COLS + m, N), dtype=torch.bfloat16, device=Q.device)
    _check(lib().rw_convert_block(_ptr(Q), _TORCH_DT[Q.dtype], _ptr(out), RW_BF16_PAIR, N, m, _stream(Q.device)))
    return PairBasis(out)


def convert_block(X: torch.Tensor, dtype) -> torch.Tensor:
    """Copy of a (cols, rows) block (column-major rows x cols) converted by the library (RNE)."""
    X = X.contiguous()
    out = torch.empty(X.shape, dtype=dtype, device=X.device)
    cols = X.shape[0] if X.dim() > 1 else 1
    rows = X.numel() // cols
    _check(lib().rw_convert_block(_ptr(X), _TORCH_DT[X.dtype], _ptr(out), _TORCH_DT[dtype], rows, cols,
                                  _stream(X.device)))
    return out


def project_basis(Q: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """P = Q^T X for Q (m, N) (column-major N x m; float32 or bfloat16) and X (C, N) float32: (C, m) float64
    tensor holding the column-major m x C result."""
    m, N = Q.shape
    C = X.shape[0]
    X = X.to(torch.float32).contiguous()
    P = torch.empty((C, m), dtype=torch.float64, device=Q.device)
    nb = ct.c_size_t()
    _check(lib().rw_project_workspace_bytes(N, m, C, ct.byref(nb)))
    work = _workspace(nb.value, Q.device)
    _check(lib().rw_project_basis(_ptr(Q.contiguous()), _TORCH_DT[Q.dtype], N, m, _ptr(X), C, _ptr(P), _ptr(work),
                                  nb.value, _stream(Q.device)))
    return P


# ---------------------------------------------------------------------------------------------
# batching form
# ---------------------------------------------------------------------------------------------
class BatchSolver:
    """Online solves for many images at once (fixed m per image), one interaction round per run().

    images: sequence of dicts {"graph": Graph, "Q": (m, N) tensor, "lam": (m,) float64 tensor,
    "S_cap": int, "C_cap": int}; all graphs share one dtype and all bases one dtype.  U[i] is the
    (C_cap, N_i) output of image i (first C rows valid after a round with C labels).  With
    use_graph=True the first run() captures the enqueue into a torch.cuda.CUDAGraph (a HIP graph)
    and later rounds replay it."""

    def __init__(self, images, use_graph: bool = True):
        self.images = list(images)
        n = len(self.images)
        if n == 0:
            raise ValueError("empty batch")
        self.device = self.images[0]["graph"].device
        self.U = []
        arr = (rw_batch_image * n)()
        self._keep = []
        for i, im in enumerate(self.images):
            g, Q, lam = im["graph"], im["Q"].contiguous(), im["lam"].contiguous()
            U = torch.zeros((int(im["C_cap"]), g.N), dtype=g.dtype, device=g.device)
            self.U.append(U)
            self._keep += [g, Q, lam]
            arr[i].g = g.handle
            arr[i].Q = Q.data_ptr()
            arr[i].q_dtype = _TORCH_DT[Q.dtype]
            arr[i].lambda_ = lam.data_ptr()
            arr[i].m = int(im.get("m", Q.shape[0]))
            arr[i].S_cap = int(im["S_cap"])
            arr[i].C_cap = int(im["C_cap"])
            arr[i].U = U.data_ptr()
        self._arr = arr
        nb = ct.c_size_t()
        _check(lib().rw_batch_workspace_bytes(arr, n, ct.byref(nb)))
        self.work = _workspace(nb.value, self.device)
        h = ct.c_void_p()
        _check(lib().rw_batch_create(arr, n, _ptr(self.work), nb.value, _stream(self.device), ct.byref(h)))
        self.handle = h
        self.use_graph = use_graph
        self.graph = None
        self._stream = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rw_batch_destroy(h)
            self.handle = None

    def info(self):
        th, npt, tuned = ct.c_int(), ct.c_int(), ct.c_int()
        us = ct.c_double()
        _check(lib().rw_batch_info(self.handle, ct.byref(th), ct.byref(npt), ct.byref(tuned), ct.byref(us)))
        return {"threads": th.value, "nodes_per_thread": npt.value, "tuned_now": bool(tuned.value),
                "tune_us": us.value}

    def set_seeds(self, rounds):
        """rounds: per image (C, seed_node, seed_label)."""
        if len(rounds) != len(self.images):
            raise ValueError("one (C, nodes, labels) per image")
        Cs = np.array([int(r[0]) for r in rounds], dtype=np.int32)
        nodes = [np.asarray(r[1], dtype=np.int64) for r in rounds]
        labs = [np.asarray(r[2], dtype=np.int32) for r in rounds]
        off = np.zeros(len(rounds) + 1, dtype=np.int64)
        off[1:] = np.cumsum([a.size for a in nodes])
        alln = np.ascontiguousarray(np.concatenate(nodes)) if nodes else np.zeros(0, np.int64)
        alll = np.ascontiguousarray(np.concatenate(labs)) if labs else np.zeros(0, np.int32)
        # on the stream that runs the rounds: the previous round is ordered before the upload
        _check(lib().rw_batch_set_seeds(self.handle, ct.c_void_p(Cs.ctypes.data), ct.c_void_p(off.ctypes.data),
                                        ct.c_void_p(alln.ctypes.data), ct.c_void_p(alll.ctypes.data),
                                        _stream(self.device)))
        self.C = Cs

    def enqueue(self, stream=None):
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        _check(lib().rw_batch_enqueue(self.handle, ct.c_void_p(st)))

    def run(self):
        """Enqueue the round set by set_seeds (graph replay when use_graph)."""
        if not self.use_graph:
            self.enqueue()
            return
        if self.graph is None:
            self._stream = torch.cuda.Stream(self.device)
            self._stream.wait_stream(torch.cuda.current_stream(self.device))
            with torch.cuda.stream(self._stream):
                self.enqueue(self._stream)        # eager round (also warms up the launches)
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=self._stream):
                self.enqueue(self._stream)
            torch.cuda.current_stream(self.device).wait_stream(self._stream)
        else:
            self.graph.replay()

    def status(self):
        mp = ct.c_double()
        _check(lib().rw_batch_status(self.handle, ct.byref(mp), _stream(self.device)))
        return mp.value

    def outputs(self):
        return [U[: int(c)] for U, c in zip(self.U, self.C)]
