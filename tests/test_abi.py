"""The C-ABI library (no GPU needed): it loads, exports every function that
include/curveball.h declares, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1804_08487_amd as cb

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "curveball.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:cb_status|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for core in ("graph_upload", "global_trade", "graph_download", "graph_free"):
        assert core in names
    assert sorted(names) == sorted(cb.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = cb.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def _upload(n, rp, col):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    st = cb.lib().graph_upload(n, rp.ctypes.data, col.ctypes.data if len(col) else None,
                               None, cb.CB_VALIDATE, ctypes.byref(h))
    return st, cb.lib().cb_last_error().decode()


@pytest.mark.parametrize("n,rp,col,status", [
    (-1, [0], [], cb.CB_EINVAL),
    (2, [1, 1, 2], [1, 0], cb.CB_EINVAL),              # row_ptr[0] != 0
    (2, [0, 1, 0], [1], cb.CB_EINVAL),                 # not monotone
    (3, [0, 1, 2, 3], [1, 0, 0], cb.CB_ENOTSIMPLE),    # odd entry count
    (2, [0, 2, 4], [0, 1, 0, 1], cb.CB_ENOTSIMPLE),    # row longer than n - 1
])
def test_host_side_argument_errors(n, rp, col, status):
    st, msg = _upload(n, rp, col)
    assert st == status and msg


def test_null_handles():
    L = cb.lib()
    assert L.global_trade(None, 1, 0) == cb.CB_EINVAL
    assert L.graph_sync(None) == cb.CB_EINVAL
    assert L.graph_download(None, None, None) == cb.CB_EINVAL
    assert L.graph_set_option(None, cb.OPT_SMALL_MAX, 4) == cb.CB_EINVAL
    L.graph_free(None)


def test_allocator_requires_both_callbacks():
    a = cb._Allocator()
    assert cb.lib().cb_set_allocator(ctypes.byref(a)) == cb.CB_EINVAL
    assert cb.lib().cb_set_allocator(None) == cb.CB_OK


_CTYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double,
           "uint32_t": ctypes.c_uint32, "uint64_t": ctypes.c_uint64}


def _header_struct(name):
    """(field, C type) of `typedef struct { ... } name;` in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(n.strip(), typ) for n in names.split(",")]
    return fields


@pytest.mark.parametrize("cname,pystruct", [("cb_round_stats", cb.RoundStats),
                                            ("cb_tune_result", cb.TuneResult),
                                            ("cb_server_status", cb.ServerStatus)])
def test_binding_structs_mirror_the_header(cname, pystruct):
    """The ctypes mirrors list the header's fields in the same order with the
    same C types, so their layouts (offsets, padding, size) agree."""
    header = _header_struct(cname)
    mirror = [(n, t) for n, t in pystruct._fields_]
    assert [n for n, _ in header] == [n for n, _ in mirror]
    for (n, ctype), (_, pytype) in zip(header, mirror):
        assert _CTYPES[ctype] is pytype, n


def test_binding_constants_match_the_header():
    text = open(HEADER).read()
    defines = dict((k, int(v)) for k, v in re.findall(r"#define\s+(CB_\w+)\s+(\d+)u?\b", text))
    for name, value in defines.items():
        short = name[3:]
        if hasattr(cb, short):
            assert getattr(cb, short) == value, name
    opts = [k for k in defines if k.startswith("CB_OPT_")]
    assert opts and all(hasattr(cb, k[3:]) for k in opts)
