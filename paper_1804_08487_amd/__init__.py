"""Global Curveball super-step on MI355X (gfx950): Python binding.

Argument marshalling only: every step of a global trade runs in the HIP
kernels of ``libcurveball.so`` behind the C ABI declared in
``include/curveball.h``.  PyTorch supplies the stream (and, optionally, the
device memory through its caching allocator); it does no computation here.
If the shared library is missing the import of :func:`lib` fails loudly -
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcurveball.so")

CB_OK, CB_EINVAL, CB_ENOTSIMPLE, CB_ENOMEM, CB_EDEVICE, CB_EWATCHDOG, CB_EPOISONED = range(7)
STATUS_NAMES = {0: "CB_OK", 1: "CB_EINVAL", 2: "CB_ENOTSIMPLE", 3: "CB_ENOMEM",
                4: "CB_EDEVICE", 5: "CB_EWATCHDOG", 6: "CB_EPOISONED"}
CB_VALIDATE = 1
STEP_MATCHING, STEP_DEPSCAN, STEP_TRADE, STEP_REBUILD = 1, 2, 3, 4
STATE_PERM, STATE_TRADE_OF, STATE_DEP, STATE_COL, STATE_OUT_CUR, STATE_INBOX_CUR, STATE_TRACE, STATE_OWN_CUR = range(1, 9)
(OPT_SMALL_MAX, OPT_BIG_WORKERS, OPT_GRID_BLOCKS, OPT_WATCHDOG_MS, OPT_TIMING, OPT_LOCAL_STACK,
 OPT_BIG_LDS_MAX, OPT_GIANT_DEG, OPT_DEBUG_CHECKS, OPT_TRACE, OPT_HELP_MIN, OPT_HELP_GROUPS,
 OPT_HELP_CHUNK, OPT_FUSE_NEXT, OPT_IDLE_BACKOFF, OPT_CU_POOL) = range(1, 17)
UNMATCHED = 2**31 - 1

# Every symbol declared in include/curveball.h.
EXPORTS = ("cb_set_allocator", "graph_upload", "graph_info", "global_trade", "graph_sync",
           "graph_download", "graph_free", "cb_last_error", "global_trade_steps",
           "graph_download_state", "graph_set_option", "graph_stats", "graph_kernel_times",
           "batch_upload", "batch_run", "batch_info", "batch_download", "graph_autotune",
           "global_trade_static", "server_create", "server_submit", "server_step",
           "server_request_state", "server_result", "server_release", "server_free", "cbu_trades")


class CurveballError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)),
                ("user", ctypes.c_void_p)]


class RoundStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "trades", "small_trades", "big_trades", "sources", "queue_pushes", "work",
        "forwarded", "emitted", "small_workers", "big_workers")] + [
        (name, ctypes.c_double) for name in (
            "small_busy_us", "big_busy_us", "big_gather_us", "big_split_us", "big_write_us",
            "big_release_us", "big_max_us")] + [
        (name, ctypes.c_int64) for name in ("moved", "counted_trades")]

    def as_dict(self):
        return {name: (getattr(self, name) if isinstance(getattr(self, name), float)
                       else int(getattr(self, name))) for name, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("small_max", ctypes.c_int32), ("help_min", ctypes.c_int32),
                ("help_chunk", ctypes.c_int32), ("big_workers", ctypes.c_int32),
                ("local_stack", ctypes.c_int32), ("idle_backoff", ctypes.c_int32),
                ("cu_pool", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("ms_per_round", ctypes.c_double), ("default_ms_per_round", ctypes.c_double),
                ("evaluated", ctypes.c_int32), ("cached", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStatus(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "queued", "active_chains", "finished_requests", "steps", "repacks", "active_bytes",
        "budget_bytes")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1804_08487_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        L.cb_set_allocator.argtypes = [ctypes.POINTER(_Allocator)]
        L.graph_upload.argtypes = [i64, vp, vp, vp, u32, ctypes.POINTER(vp)]
        L.graph_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.global_trade.argtypes = [vp, u64, u32]
        L.graph_sync.argtypes = [vp]
        L.graph_download.argtypes = [vp, vp, vp]
        L.graph_free.argtypes = [vp]
        L.graph_free.restype = None
        L.cb_last_error.argtypes = []
        L.cb_last_error.restype = ctypes.c_char_p
        L.global_trade_steps.argtypes = [vp, u64, u32, i32]
        L.graph_download_state.argtypes = [vp, i32, vp, i64]
        L.graph_set_option.argtypes = [vp, i32, i64]
        L.graph_stats.argtypes = [vp, ctypes.POINTER(RoundStats)]
        L.graph_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i64)]
        L.batch_upload.argtypes = [i32, vp, vp, vp, vp, vp, vp, u32, ctypes.POINTER(vp)]
        L.batch_run.argtypes = [vp, u32]
        L.batch_info.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(u32)]
        L.batch_download.argtypes = [vp, i32, vp]
        L.graph_autotune.argtypes = [vp, u32, i32, ctypes.POINTER(TuneResult)]
        L.global_trade_static.argtypes = [i64, vp, vp, u64, u32, vp]
        L.server_create.argtypes = [ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.server_submit.argtypes = [vp, i64, vp, vp, i32, u32, u64, ctypes.POINTER(i64)]
        L.server_step.argtypes = [vp, ctypes.POINTER(ServerStatus)]
        L.server_request_state.argtypes = [vp, i64, ctypes.POINTER(i32)]
        L.server_result.argtypes = [vp, i64, i32, vp]
        L.server_release.argtypes = [vp, i64]
        L.cbu_trades.argtypes = [vp, u64, u64, u64]
        L.server_free.argtypes = [vp]
        L.server_free.restype = None
        for name in EXPORTS:
            if name not in ("graph_free", "cb_last_error", "server_free"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != CB_OK:
        raise CurveballError(status, lib().cb_last_error().decode(errors="replace"))


_torch_alloc_refs = None


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through PyTorch's caching
    allocator (current device, current stream)."""
    global _torch_alloc_refs
    if not enable:
        _check(lib().cb_set_allocator(None))
        _torch_alloc_refs = None
        return
    import torch

    @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    a = _Allocator(_alloc, _free, None)
    _torch_alloc_refs = (a, _alloc, _free)
    _check(lib().cb_set_allocator(ctypes.byref(a)))


def current_stream_handle():
    """hipStream_t of PyTorch's current stream on the current device."""
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def global_trade_static(row_ptr, col_device_ptr: int, seed: int, rnd: int, stream=None):
    """One global trade of a graph held by the caller (host row_ptr, device col
    at `col_device_ptr`, overwritten with the result), with no allocation."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    if stream is None:
        stream = current_stream_handle()
    _check(lib().global_trade_static(len(rp) - 1, rp.ctypes.data, col_device_ptr, seed, rnd, stream))


class Graph:
    """One device-resident chain: a simple undirected graph in CSR form."""

    def __init__(self, row_ptr, col, stream=None, validate: bool = True):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        self.row_ptr = rp.copy()
        n = len(rp) - 1
        h = ctypes.c_void_p()
        if stream is None:
            stream = current_stream_handle()
        self._stream = stream
        _check(lib().graph_upload(n, rp.ctypes.data, cl.ctypes.data if len(cl) else None, stream,
                                  CB_VALIDATE if validate else 0, ctypes.byref(h)))
        self._h = h
        self.n = n
        self.nnz = int(rp[-1])

    # ---- the super-step -------------------------------------------------
    def global_trade(self, seed: int, rnd: int):
        _check(lib().global_trade(self._h, seed, rnd))

    def run_steps(self, seed: int, rnd: int, last_step: int):
        _check(lib().global_trade_steps(self._h, seed, rnd, last_step))

    def sync(self):
        _check(lib().graph_sync(self._h))

    def download(self):
        col = np.empty(max(self.nnz, 1), np.int32)
        _check(lib().graph_download(self._h, None, col.ctypes.data))
        return col[:self.nnz]

    def state(self, which: int):
        count = {STATE_PERM: self.n, STATE_TRADE_OF: self.n, STATE_DEP: self.n // 2,
                 STATE_COL: self.nnz, STATE_OUT_CUR: self.n, STATE_INBOX_CUR: self.n, STATE_OWN_CUR: self.n,
                 STATE_TRACE: 24 * (self.n // 2)}[which]
        out = np.empty(max(count, 1), np.int64 if which == STATE_TRACE else np.int32)
        _check(lib().graph_download_state(self._h, which, out.ctypes.data, count))
        return out[:count]

    def set_option(self, option: int, value: int):
        _check(lib().graph_set_option(self._h, option, value))

    def stats(self):
        st = RoundStats()
        _check(lib().graph_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def kernel_times(self):
        ms = (ctypes.c_double * 4)()
        rounds = ctypes.c_int64()
        _check(lib().graph_kernel_times(self._h, ms, 4, ctypes.byref(rounds)))
        return [float(x) for x in ms], int(rounds.value)

    def single_trades(self, seed: int, step0: int, steps: int):
        """Uniform single trades step0 .. step0 + steps - 1 (see ``cbu_trades``)."""
        _check(lib().cbu_trades(self._h, seed, step0, steps))

    def autotune(self, trial_rounds: int = 2, use_cache: bool = True):
        res = TuneResult()
        _check(lib().graph_autotune(self._h, trial_rounds, 1 if use_cache else 0, ctypes.byref(res)))
        return res.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().graph_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(Graph):
    """Independent chains advancing together on one GPU: chain c is the graph
    ``graphs[c] = (row_ptr, col)`` with chain seed ``seeds[c]``; every round
    of the batch is one global trade of every chain (see ``batch_upload``)."""

    def __init__(self, graphs, seeds, first_rounds=None, stream=None, validate: bool = True):
        self._keep = []
        C = len(graphs)
        ns = np.array([len(rp) - 1 for rp, _ in graphs], np.int64)
        rps = (ctypes.c_void_p * C)()
        cols = (ctypes.c_void_p * C)()
        self.row_ptrs = []
        for c, (rp, col) in enumerate(graphs):
            rp = np.ascontiguousarray(rp, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            if len(col) == 0:
                col = np.zeros(1, np.int32)
            self._keep += [rp, col]
            self.row_ptrs.append(rp.copy())
            rps[c] = rp.ctypes.data
            cols[c] = col.ctypes.data
        sd = np.array([int(x) & (2**64 - 1) for x in seeds], np.uint64)
        fr = None if first_rounds is None else np.array(first_rounds, np.uint32)
        if stream is None:
            stream = current_stream_handle()
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib().batch_upload(C, ns.ctypes.data, ctypes.cast(rps, ctypes.c_void_p),
                                  ctypes.cast(cols, ctypes.c_void_p), sd.ctypes.data,
                                  fr.ctypes.data if fr is not None else None, stream,
                                  CB_VALIDATE if validate else 0, ctypes.byref(h)))
        self._keep = []
        self._h = h
        self.chains = C
        self.n = int(ns.sum())
        self.nnz = int(sum(int(rp[-1]) for rp in self.row_ptrs))

    def run(self, rounds: int):
        _check(lib().batch_run(self._h, rounds))

    def info(self, chain: int):
        n, nnz, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint32()
        _check(lib().batch_info(self._h, chain, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(r)))
        return int(n.value), int(nnz.value), int(r.value)

    def download_chain(self, chain: int):
        _, nnz, _ = self.info(chain)
        col = np.empty(max(nnz, 1), np.int32)
        _check(lib().batch_download(self._h, chain, col.ctypes.data))
        return col[:nnz]


class Server:
    """Continuous-batching request server (see ``server_create``): requests
    "samples of G after r rounds" join the running batch as memory allows."""

    def __init__(self, hbm_budget_bytes: int, stream=None):
        if stream is None:
            stream = current_stream_handle()
        h = ctypes.c_void_p()
        _check(lib().server_create(int(hbm_budget_bytes), stream, ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def submit(self, row_ptr, col, samples: int, rounds: int, seed: int) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        rid = ctypes.c_int64()
        _check(lib().server_submit(self._h, len(rp) - 1, rp.ctypes.data, cl.ctypes.data if len(cl) else None,
                                   samples, rounds, int(seed) & (2**64 - 1), ctypes.byref(rid)))
        self._sizes[int(rid.value)] = (int(rp[-1]), samples)
        return int(rid.value)

    def step(self):
        st = ServerStatus()
        _check(lib().server_step(self._h, ctypes.byref(st)))
        return st.as_dict()

    def finished(self, rid: int) -> bool:
        f = ctypes.c_int32()
        _check(lib().server_request_state(self._h, rid, ctypes.byref(f)))
        return bool(f.value)

    def result(self, rid: int, sample: int):
        nnz, _ = self._sizes[rid]
        out = np.empty(max(nnz, 1), np.int32)
        _check(lib().server_result(self._h, rid, sample, out.ctypes.data))
        return out[:nnz]

    def release(self, rid: int):
        _check(lib().server_release(self._h, rid))
        self._sizes.pop(rid, None)

    def close(self):
        if getattr(self, "_h", None):
            lib().server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
