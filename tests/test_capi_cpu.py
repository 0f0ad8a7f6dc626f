"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/kadabra.h, and rejects malformed input before touching
the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1903_09422_amd import _lib
from paper_1903_09422_amd import graphs as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "kadabra.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kadabra_\w+)\s*\(", src)))


def test_header_lists_expected_entry_points():
    names = header_functions()
    assert {"kadabra_create_graph", "kadabra_run", "kadabra_get_scores"} <= set(names)
    assert names == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert L.kadabra_version() >= 10000


def _create(n, row_ptr, col, num_arcs=None):
    L = _lib.lib()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    h = C.c_void_p(1234)
    rc = L.kadabra_create_graph(n, cl.size if num_arcs is None else num_arcs, rp.ctypes.data,
                                cl.ctypes.data if cl.size else None, C.byref(h))
    return rc, h, L.kadabra_last_error().decode()


def test_create_rejects_malformed_csr():
    g = G.path_graph(4)  # 0-1-2-3
    rp, col = g.row_ptr.copy(), g.col.copy()
    cases = []
    cases.append((1, np.array([0, 0]), np.array([], dtype=np.int32), None, "n must be"))
    bad = rp.copy(); bad[0] = 1
    cases.append((4, bad, col, None, "row_ptr[0]"))
    cases.append((4, rp, col, col.size - 1, "num_arcs"))
    bad = col.copy(); bad[0] = 7
    cases.append((4, rp, bad, None, "out of range"))
    bad = col.copy(); bad[0] = 0  # vertex 0's neighbour is itself
    cases.append((4, rp, bad, None, "self-loop"))
    bad = rp.copy(); bad[2] = bad[1] - 1
    cases.append((4, bad, col, None, "decreases"))
    asym = G.from_edges(3, [0], [1], lcc=False)
    col3 = np.array([1, 0, 2], dtype=np.int32)  # 1 -> 0 and 1 -> 2 but 2 has no arcs
    cases.append((3, np.array([0, 1, 3, 3]), col3, None, "no reverse"))
    unsorted = G.star_graph(3)
    c2 = unsorted.col.copy(); c2[[0, 1]] = c2[[1, 0]]
    cases.append((4, unsorted.row_ptr, c2, None, "ascending"))
    dup = np.array([0, 2, 3], dtype=np.int32)
    cases.append((2, dup, np.array([1, 1, 0], dtype=np.int32), None, "ascending"))
    for n, r, c, na, msg in cases:
        rc, h, err = _create(n, r, c, na)
        assert rc == _lib.EINVAL, (msg, rc, err)
        assert msg in err, (msg, err)
        assert h.value is None
    _ = asym


def _guarded_i32(values):
    """values in an int32 array that ends exactly at a PROT_NONE page, so a
    read one element past its end faults instead of passing unnoticed."""
    import mmap

    page = mmap.PAGESIZE
    buf = mmap.mmap(-1, 2 * page, prot=mmap.PROT_READ | mmap.PROT_WRITE)
    base = C.addressof(C.c_char.from_buffer(buf))
    libc = C.CDLL(None, use_errno=True)
    libc.mprotect.argtypes = [C.c_void_p, C.c_size_t, C.c_int]
    assert libc.mprotect(base + page, page, 0) == 0  # PROT_NONE
    vals = np.asarray(values, dtype=np.int32)
    arr = np.frombuffer(buf, dtype=np.int32, count=vals.size, offset=page - 4 * vals.size)
    arr[:] = vals
    return buf, arr


def test_create_rejects_row_bound_past_arcs_before_reading_col():
    """row_ptr = [0, 3, 3, 2] with num_arcs = 2: row 0 claims arcs 0..2, but
    col has only two entries.  The bounds must be rejected before col is read
    (col ends at a guard page here, so reading col[2] would fault)."""
    buf, col = _guarded_i32([1, 2])
    L = _lib.lib()
    rp = np.array([0, 3, 3, 2], dtype=np.int32)
    h = C.c_void_p(1234)
    rc = L.kadabra_create_graph(3, 2, rp.ctypes.data, col.ctypes.data, C.byref(h))
    err = L.kadabra_last_error().decode()
    assert rc == _lib.EINVAL and h.value is None, (rc, err)
    assert "exceeds num_arcs" in err, err
    # a row bound past the arcs in the middle, the last one consistent
    rp = np.array([0, 1, 5, 2], dtype=np.int32)
    rc = L.kadabra_create_graph(3, 2, rp.ctypes.data, col.ctypes.data, C.byref(h))
    assert rc == _lib.EINVAL and h.value is None
    del col
    buf.close()


def test_create_rejects_oversize():
    n = 1 << 23
    rc, h, err = _create(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert rc == _lib.ERANGE and h.value is None and "2^23" in err


def test_null_arguments():
    L = _lib.lib()
    assert L.kadabra_set_param(None, b"check_interval", 5) == _lib.EINVAL
    assert L.kadabra_run(None, 0.1, 0.1, 1) == _lib.EINVAL
    assert L.kadabra_get_scores(None, None, None, None) == _lib.EINVAL
    assert L.kadabra_cancel(None) == _lib.EINVAL
    L.kadabra_destroy_graph(None)  # no-op
    rc = L.kadabra_create_graph(4, 0, None, None, None)
    assert rc == _lib.EINVAL
    assert L.kadabra_eval_stop_fg(0, None, 1, 1, 1.0, None, None) == _lib.EINVAL
    out = C.c_void_p(99)
    assert L.kadabra_server_create(None, 0, 0, 0, C.byref(out)) == _lib.EINVAL
    assert out.value is None
    assert L.kadabra_server_submit(None, 0, 0.1, 0.1, 1, 8, None) == _lib.EINVAL
    assert L.kadabra_server_wait(None, 1, 0.0, None) == _lib.EINVAL
    assert L.kadabra_server_result(None, 1, None, None, None, None) == _lib.EINVAL
    assert L.kadabra_server_release(None, 1) == _lib.EINVAL
    assert L.kadabra_server_info_get(None, None, 0) == _lib.EINVAL
    L.kadabra_server_destroy(None)  # no-op


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
