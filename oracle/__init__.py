"""CPU oracle for the global Curveball super-step (ctypes binding).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package.  The GPU library in
``paper_1804_08487_amd`` never imports, links or calls it, and the two share
no code.  The arithmetic lives in ``curveball_oracle.c`` (plain sequential C,
one function per definition of the paper); this module only marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "curveball_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
UNMATCHED = 2**31 - 1
TAG_M = 0x4D415443
TAG_F = 0x46595348

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "trades", "work", "common", "disjoint", "moved", "uv_edges", "max_s",
        "unmatched", "dep_mismatch")] + [("setup_seconds", ctypes.c_double),
                                         ("trade_seconds", ctypes.c_double),
                                         ("rebuild_seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: (float if typ is ctypes.c_double else int)(getattr(self, name))
                for name, typ in self._fields_}


def build(src: str = _SRC, out: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           *extra_flags, "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _declare(lib):
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox64.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4
    lib.orc_philox64.restype = ctypes.c_uint64
    lib.orc_bounded.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_bounded.restype = ctypes.c_uint64
    lib.orc_matching.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, _i32p, _i32p]
    lib.orc_matching.restype = ctypes.c_int
    lib.orc_split.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_split.restype = None
    lib.orc_trade_apply.argtypes = [_i32p, ctypes.c_int64, _i32p, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, _i32p,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                    _i32p, _i32p, _i32p, _i32p, _i64p]
    lib.orc_trade_apply.restype = ctypes.c_int
    lib.orc_depcount.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p, _i32p, _i32p]
    lib.orc_depcount.restype = ctypes.c_int
    lib.orc_global_trade_o1.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.POINTER(Stats)]
    lib.orc_global_trade_o1.restype = ctypes.c_int
    lib.orc_global_trade_o2.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.POINTER(Stats), ctypes.c_int64]
    lib.orc_global_trade_o2.restype = ctypes.c_int
    lib.orc_check_graph.argtypes = [ctypes.c_int64, _i64p, _i32p]
    lib.orc_check_graph.restype = ctypes.c_int
    lib.orc_cbu_pair.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, _i32p, _i32p]
    lib.orc_cbu_pair.restype = None
    lib.orc_cbu_o1.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.POINTER(Stats)]
    lib.orc_cbu_o1.restype = ctypes.c_int
    return lib


class Oracle:
    """Binding to one compiled copy of the oracle (the default build or a
    variant compiled elsewhere, e.g. by the mutation tests)."""

    def __init__(self, path: str = LIB_PATH):
        if path == LIB_PATH and not os.path.exists(path):
            build()
        self.lib = _declare(ctypes.CDLL(path))

    # -- random numbers -------------------------------------------------
    def philox4x32_10(self, ctr, key):
        c = (ctypes.c_uint32 * 4)(*ctr)
        k = (ctypes.c_uint32 * 2)(*key)
        o = (ctypes.c_uint32 * 4)()
        self.lib.orc_philox4x32_10(c, k, o)
        return tuple(int(x) for x in o)

    def philox64(self, seed, c0, c1, c2, c3):
        return int(self.lib.orc_philox64(seed, c0, c1, c2, c3))

    def bounded(self, x, k):
        return int(self.lib.orc_bounded(x, k))

    # -- matching -------------------------------------------------------
    def matching(self, n, seed, rnd):
        order = np.empty(max(n, 1), dtype=np.int32)
        trade_of = np.empty(max(n, 1), dtype=np.int32)
        rc = self.lib.orc_matching(n, seed, rnd, _ptr32(order), _ptr32(trade_of))
        if rc:
            raise RuntimeError(f"orc_matching failed: {rc}")
        return order[:n], trade_of[:n]

    # -- one trade ------------------------------------------------------
    def split(self, D, a, seed, rnd, trade):
        D = np.ascontiguousarray(D, dtype=np.int32).copy()
        self.lib.orc_split(_ptr32(D), len(D), a, seed, rnd, trade)
        return D

    def trade_apply(self, Au, Av, u, v, arrangement=None, seed=0, rnd=0, trade=0):
        Au = np.ascontiguousarray(Au, dtype=np.int32)
        Av = np.ascontiguousarray(Av, dtype=np.int32)
        du, dv = len(Au), len(Av)
        Bu = np.empty(max(du, 1), np.int32)
        Bv = np.empty(max(dv, 1), np.int32)
        mtv = np.empty(max(du + dv, 1), np.int32)
        mtu = np.empty(max(du + dv, 1), np.int32)
        info = (ctypes.c_int64 * 6)()
        arr = None
        if arrangement is not None:
            arr = np.ascontiguousarray(arrangement, dtype=np.int32)
        rc = self.lib.orc_trade_apply(_ptr32(Au), du, _ptr32(Av), dv, u, v,
                                      _ptr32(arr) if arr is not None else None,
                                      seed, rnd, trade, _ptr32(Bu), _ptr32(Bv),
                                      _ptr32(mtv), _ptr32(mtu), info)
        if rc:
            raise ValueError(f"orc_trade_apply failed: {rc}")
        inf = [int(x) for x in info]
        return Bu[:du].copy(), Bv[:dv].copy(), mtv[:inf[4]].copy(), mtu[:inf[5]].copy(), {
            "common": inf[0], "a": inf[1], "b": inf[2], "uv": inf[3]}

    # -- whole rounds -----------------------------------------------------
    def depcount(self, row_ptr, col, trade_of, order):
        n = len(row_ptr) - 1
        dep = np.empty(max(n // 2, 1), np.int32)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        rc = self.lib.orc_depcount(n, _ptr64(rp), _ptr32(cl), _ptr32(trade_of),
                                   _ptr32(order), _ptr32(dep))
        if rc:
            raise RuntimeError(f"orc_depcount failed: {rc}")
        return dep[:n // 2]

    def global_trade(self, row_ptr, col, seed, rnd, form="o1", max_trades=-1):
        """Apply one global trade; returns (new col, stats dict)."""
        n = len(row_ptr) - 1
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        out = np.array(col, dtype=np.int32, copy=True)
        st = Stats()
        if form == "o1":
            rc = self.lib.orc_global_trade_o1(n, _ptr64(rp), _ptr32(out), seed, rnd,
                                              ctypes.byref(st))
        elif form == "o2":
            rc = self.lib.orc_global_trade_o2(n, _ptr64(rp), _ptr32(out), seed, rnd,
                                              ctypes.byref(st), max_trades)
        else:
            raise ValueError(form)
        if rc:
            raise RuntimeError(f"oracle global trade ({form}) failed: {rc}")
        return out, st.as_dict()

    def cbu_pair(self, n, seed, step):
        u, v = ctypes.c_int32(), ctypes.c_int32()
        self.lib.orc_cbu_pair(n, seed, step, ctypes.byref(u), ctypes.byref(v))
        return int(u.value), int(v.value)

    def cbu(self, row_ptr, col, seed, step0, steps):
        """Apply uniform single trades step0 .. step0 + steps - 1; returns
        (new col, stats dict)."""
        n = len(row_ptr) - 1
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        out = np.array(col, dtype=np.int32, copy=True)
        st = Stats()
        rc = self.lib.orc_cbu_o1(n, _ptr64(rp), _ptr32(out), seed, step0, steps, ctypes.byref(st))
        if rc:
            raise RuntimeError(f"oracle single trades failed: {rc}")
        return out, st.as_dict()

    def check_graph(self, row_ptr, col):
        n = len(row_ptr) - 1
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        if len(cl) == 0:
            cl = np.zeros(1, np.int32)
        return int(self.lib.orc_check_graph(n, _ptr64(rp), _ptr32(cl)))


def _ptr32(a):
    if a is None:
        return None
    if len(a) == 0:
        a = np.zeros(1, np.int32)
    return a.ctypes.data_as(_i32p)


def _ptr64(a):
    return a.ctypes.data_as(_i64p)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
