"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every entry point the
header declares, and validates arguments before touching a device."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rw.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:const char\*|int)\s+(rw_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_core_entry_points():
    names = declared()
    for n in ("rw_build_graph", "rw_precompute_eig", "rw_solve_seeds", "rw_update_eig", "rw_apply_laplacian",
              "rw_cg_solve", "rw_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1607_04174_amd as rw
    if not os.path.exists(rw.LIB_PATH):
        pytest.skip("librw.so not built")
    L = ct.CDLL(rw.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared symbol
    assert set(declared()) <= set(rw.declared_symbols())


def test_host_validation_without_device():
    import paper_1607_04174_amd as rw
    if not os.path.exists(rw.LIB_PATH):
        pytest.skip("librw.so not built")
    L = rw.lib()
    d = rw.rw_graph_desc()
    d.ndim = 2
    d.dims[0], d.dims[1], d.dims[2] = 10, 10, 1
    d.conn = 6
    d.dtype = rw.RW_F32
    nb = ct.c_size_t()
    assert L.rw_graph_bytes(ct.byref(d), ct.byref(nb)) == rw.RW_EINVAL
    assert b"connectivity" in L.rw_last_error()
    d.conn = 8
    assert L.rw_graph_bytes(ct.byref(d), ct.byref(nb)) == rw.RW_OK
    assert nb.value > 100 * 4 * 4
    d.dims[2] = 2
    assert L.rw_graph_bytes(ct.byref(d), ct.byref(nb)) == rw.RW_EINVAL
    assert L.rw_version() >= 1


def test_checkpoint_header_is_validated_on_the_host(tmp_path):
    """rw_eig_read_header reads and checks a checkpoint's header without touching a device: a missing file,
    a foreign file and inconsistent sizes are refused; a well-formed header comes back field by field."""
    import paper_1607_04174_amd as rw
    with pytest.raises(rw.RWError):
        rw.eig_read_header(str(tmp_path / "missing.rweig"))
    bad = tmp_path / "garbage.rweig"
    bad.write_bytes(b"not a checkpoint" * 16)
    with pytest.raises(rw.RWError):
        rw.eig_read_header(str(bad))
    h = rw.rw_eig_header()
    assert ct.sizeof(h) == 128
    h.magic = b"RWEIGv1"
    h.version, h.ndim, h.conn, h.graph_dtype, h.weight_form, h.normalized = 1, 2, 4, 1, 0, 1
    h.dims[0], h.dims[1], h.dims[2] = 7, 5, 1
    h.beta, h.m, h.q_dtype, h.tol, h.weight_hash = 90.0, 3, 1, 1e-5, 12345
    h.q_bytes, h.lambda_bytes = 35 * 3 * 4, 3 * 8
    good = tmp_path / "good.rweig"
    good.write_bytes(bytes(h) + bytes(35 * 3 * 4 + 3 * 8))
    d = rw.eig_read_header(str(good))
    assert (d["dims"], d["m"], d["q_dtype"], d["beta"], d["weight_hash"]) == ((7, 5, 1), 3, 1, 90.0, 12345)
    h.q_bytes += 4                                    # sizes that do not match the grid
    good.write_bytes(bytes(h))
    with pytest.raises(rw.RWError):
        rw.eig_read_header(str(good))
