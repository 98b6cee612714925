"""The C ABI library: every symbol declared in include/hq.h is exported, and
argument errors are rejected on the host before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hq_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1708_08427_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhq.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1708_08427_amd import _lib
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(declared_functions()) == bound


def test_status_strings(lib):
    assert lib.hq_status_string(0) == b"HQ_OK"
    assert lib.hq_status_string(5) == b"HQ_E_UNSUPPORTED"


def _build(lib, offsets, pos_ptr=1):
    off = np.asarray(offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib.hq_build(ctypes.c_void_p(pos_ptr), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      len(off) - 1, None, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("offsets", [[1, 5], [0, 1], [0, 4, 5], [0, 4, 3], [0]])
def test_invalid_offsets_rejected_on_host(lib, offsets):
    st, h = _build(lib, offsets)
    assert st == 1 and not h.value
    assert lib.hq_last_error()


def test_null_arguments_rejected(lib):
    off = np.array([0, 4], dtype=np.int64)
    h = ctypes.c_void_p()
    assert lib.hq_build(None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, None, None,
                        ctypes.byref(h)) == 1
    assert lib.hq_build(ctypes.c_void_p(1), None, 1, None, None, ctypes.byref(h)) == 1
    assert lib.hq_apply(None, None, None, 0, 1, 0, None) == 1
    assert lib.hq_query(None, None) == 1
    assert lib.hq_rigid_motion(None, None, None, None, None, None, None) == 1
    lib.hq_destroy(None)


def test_bad_options_rejected(lib):
    from paper_1708_08427_amd._lib import Options
    off = np.array([0, 4], dtype=np.int64)
    h = ctypes.c_void_p()
    bad = [Options(1, 0, 0, 0), Options(4096, 0, 0, 0), Options(0, 7, 0, 0), Options(0, 0, 0, 99),
           Options(run_nodes=4), Options(waves_per_cu=65), Options(keep_node_data=2),
           Options(later_tile_units=1), Options(later_tile_units=2048), Options(first_waves_per_cu=-1),
           Options(first_waves_per_cu=65)]
    for opt in bad:
        st = lib.hq_build(ctypes.c_void_p(1), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1,
                          ctypes.byref(opt), None, ctypes.byref(h))
        assert st == 1


def test_workspace_bytes_host_only():
    """hq_workspace_bytes needs no device: it only sizes the pieces."""
    import paper_1708_08427_amd as hq
    off = np.array([0, 500, 1700, 1702], dtype=np.int64)
    base = hq.workspace_bytes(off)
    assert base > 0 and base % 256 == 0
    # exchange entries grow with max_nrhs and the tile bound, Krylov vectors
    # appear with krylov_nrhs, a smaller tile bound shrinks the tables
    assert hq.workspace_bytes(off, max_nrhs=64) > base
    assert hq.workspace_bytes(off, krylov_nrhs=4) > base
    assert hq.workspace_bytes(off, max_tiles=16) < base
    assert hq.workspace_bytes(off, store=2) < hq.workspace_bytes(off, store=3)
    with pytest.raises(hq.HQError):
        hq.workspace_bytes([0, 1])
    with pytest.raises(hq.HQError):
        hq.workspace_bytes(off, max_nrhs=-1)
