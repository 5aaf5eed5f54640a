"""Thin ctypes binding of libxdrop (``include/xdrop.h``).

Argument marshalling only: every step of the extension runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  The library must be
built (``python -m paper_2002_05200_amd.build``); importing the binding never
falls back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libxdrop binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxdrop.so")

(XD_OK, XD_EINVAL, XD_ENOMEM, XD_EDEVICE, XD_EBUSY, XD_EOVERFLOW, XD_ECANCELED, XD_ENOTREADY,
 XD_ETIMEDOUT) = range(9)
SCHED_AUTO, SCHED_PLAIN, SCHED_PERSISTENT = 0, 1, 2
TIER_CELLS = (1, 2, 4, 8, 16, 32)

PAIR_DTYPE = np.dtype([("a_off", "<u8"), ("b_off", "<u8"), ("a_len", "<u4"), ("b_len", "<u4"),
                       ("a_seed", "<u4"), ("b_seed", "<u4"), ("k", "<u4"), ("x", "<i4")])
RESULT_DTYPE = np.dtype([("score", "<i4"), ("left_score", "<i4"), ("right_score", "<i4"),
                         ("seed_score", "<i4"), ("a_begin", "<u4"), ("a_end", "<u4"),
                         ("b_begin", "<u4"), ("b_end", "<u4"), ("left_cells", "<u8"),
                         ("right_cells", "<u8"), ("status", "<i4"), ("reserved", "<i4")])
assert PAIR_DTYPE.itemsize == 40 and RESULT_DTYPE.itemsize == 56

SEED_DTYPE = np.dtype([("a_seed", "<u4"), ("b_seed", "<u4"), ("found", "<i4"), ("status", "<i4"),
                       ("bin_matches", "<u8"), ("matches", "<u8")])
assert SEED_DTYPE.itemsize == 32
SEED_FIELDS = ["a_seed", "b_seed", "bin_matches", "matches", "found", "status"]

RESULT_FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
                 "b_begin", "b_end", "left_cells", "right_cells", "status"]


class Scores(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("min_tier", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("sort_jobs", ctypes.c_int32),
                ("long_job", ctypes.c_int32), ("long_tier_bias", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("impl", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("multi_wave", ctypes.c_int32),
                ("max_save_slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("jobs", ctypes.c_uint64 * 7), ("cells", ctypes.c_uint64 * 7),
                ("escalated", ctypes.c_uint64 * 7), ("restarted", ctypes.c_uint64 * 7),
                ("wasted_cells", ctypes.c_uint64 * 7), ("stage_ms", ctypes.c_float * 9),
                ("profiled", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("max_batch_pairs", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("mem_budget", ctypes.c_uint64), ("extend_opts", Opts),
                ("group_by_class", ctypes.c_int32), ("watchdog_ms", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("a_words", ctypes.c_uint64),
                ("b", ctypes.c_void_p), ("b_words", ctypes.c_uint64),
                ("pairs", ctypes.c_void_p), ("n_pairs", ctypes.c_uint32),
                ("scores", Scores)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("max_inflight", ctypes.c_uint64),
                ("canceled", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("arena_words", ctypes.c_uint64), ("waiting_polls", ctypes.c_uint64),
                ("timed_out", ctypes.c_uint64)]


class XdropError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libxdrop status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libxdrop.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2002_05200_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        p, u64, sz, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
        L.xd_pack.argtypes = [ctypes.c_char_p, sz, p]
        L.xd_pack.restype = i32
        L.xd_pack_codes.argtypes = [p, sz, p, u64]
        L.xd_pack_codes.restype = i32
        L.xd_ctx_create.argtypes = [i32, sz, ctypes.POINTER(p)]
        L.xd_ctx_create.restype = i32
        L.xd_ctx_destroy.argtypes = [p]
        L.xd_ctx_destroy.restype = None
        L.xd_ctx_memory.argtypes = [p, ctypes.POINTER(u64)]
        L.xd_ctx_memory.restype = i32
        L.xdrop_extend.argtypes = [p, p, u64, p, u64, p, sz, Scores, p, p, p]
        L.xdrop_extend.restype = i32
        L.xdrop_extend_matrix.argtypes = [p, p, u64, p, u64, p, sz, p, ctypes.c_int32, p, p, p]
        L.xdrop_extend_matrix.restype = i32
        L.xd_find_seeds.argtypes = [p, p, u64, p, u64, p, sz, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_int32, p, p]
        L.xd_find_seeds.restype = i32
        L.xdrop_extend_noalloc.argtypes = [i32, p, u64, p, u64, p, sz, Scores, p, p, p]
        L.xdrop_extend_noalloc.restype = i32
        L.xdrop_extend_host.argtypes = [p, p, u64, p, u64, p, sz, Scores, p, p]
        L.xdrop_extend_host.restype = i32
        L.xd_last_stats.argtypes = [p, ctypes.POINTER(Stats)]
        L.xd_last_stats.restype = i32
        L.xd_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(p)]
        L.xd_server_create.restype = i32
        L.xd_server_submit.argtypes = [p, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        L.xd_server_submit.restype = i32
        L.xd_server_poll.argtypes = [p, u64, p, ctypes.c_int32, ctypes.POINTER(u64)]
        L.xd_server_poll.restype = i32
        L.xd_server_cancel.argtypes = [p, u64]
        L.xd_server_cancel.restype = i32
        L.xd_server_get_stats.argtypes = [p, ctypes.POINTER(ServerStats)]
        L.xd_server_get_stats.restype = i32
        L.xd_server_destroy.argtypes = [p]
        L.xd_server_destroy.restype = None
        L.xd_last_error.argtypes = []
        L.xd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().xd_last_error().decode(errors="replace")


def _check(status: int):
    if status != XD_OK:
        raise XdropError(status, last_error())


def pack_codes(codes: np.ndarray, pad_words: int = 0) -> np.ndarray:
    """2-bit packs base codes 0..3 with the library's host packer."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    nw = (len(codes) + 15) // 16 + pad_words
    words = np.zeros(max(nw, 1), dtype=np.uint32)
    _check(lib().xd_pack_codes(codes.ctypes.data_as(ctypes.c_void_p), len(codes),
                               words.ctypes.data_as(ctypes.c_void_p), 0))
    return words


def pack_ascii(text: bytes) -> np.ndarray:
    words = np.zeros(max((len(text) + 15) // 16, 1), dtype=np.uint32)
    _check(lib().xd_pack(text, len(text), words.ctypes.data_as(ctypes.c_void_p)))
    return words


def make_pairs(bt) -> np.ndarray:
    """xd_pair records of a generator batch."""
    pr = np.zeros(bt.n, PAIR_DTYPE)
    pr["a_off"] = bt.a_off
    pr["b_off"] = bt.b_off
    pr["a_len"] = bt.a_len
    pr["b_len"] = bt.b_len
    pr["a_seed"] = bt.a_seed
    pr["b_seed"] = bt.b_seed
    pr["k"] = bt.k
    pr["x"] = bt.x
    return pr


def _dev_bytes(arr: np.ndarray, device) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8).reshape(-1))
    return t.to(device, non_blocking=False)


class DeviceBatch:
    """A batch resident in device memory: packed arenas, pair records, results."""

    def __init__(self, bt, device="cuda:0"):
        self.n = bt.n
        self.scores = tuple(bt.scores)
        self.a_words = pack_codes(bt.a)
        self.b_words = pack_codes(bt.b)
        self.pairs = make_pairs(bt)
        self.d_a = _dev_bytes(self.a_words, device)
        self.d_b = _dev_bytes(self.b_words, device)
        self.d_pairs = _dev_bytes(self.pairs, device)
        self.d_out = torch.empty(max(self.n, 1) * RESULT_DTYPE.itemsize, dtype=torch.uint8,
                                 device=device)

    def results(self) -> np.ndarray:
        raw = self.d_out[: self.n * RESULT_DTYPE.itemsize].cpu().numpy()
        return raw.view(RESULT_DTYPE).copy()


def make_opts(sched: int = SCHED_AUTO, min_tier: int = 0, waves_per_cu: int = 0,
              sort_jobs: int = 1, long_job: int = 0, long_tier_bias: int = 0,
              profile: int = 0, impl: int = 0, graph: int = 0, multi_wave: int = 0,
              max_save_slots: int = 0) -> Opts:
    o = Opts()
    o.sched, o.min_tier, o.waves_per_cu = sched, min_tier, waves_per_cu
    o.sort_jobs, o.long_job, o.long_tier_bias = sort_jobs, long_job, long_tier_bias
    o.profile, o.impl, o.graph, o.multi_wave = profile, impl, graph, multi_wave
    o.max_save_slots = max_save_slots
    return o


class Context:
    """An xd_ctx on one device."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        torch.cuda.init()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().xd_ctx_create(device, mem_budget, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().xd_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extend_device(self, db: DeviceBatch, stream: Optional[torch.cuda.Stream] = None,
                      opts: Optional[Opts] = None, scores: Optional[Sequence[int]] = None):
        """Enqueues xdrop_extend on ``stream`` (default: torch's current stream)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        sc = Scores(*(scores if scores is not None else db.scores))
        _check(lib().xdrop_extend(self.h, db.d_a.data_ptr(), len(db.a_words), db.d_b.data_ptr(),
                                  len(db.b_words), db.d_pairs.data_ptr(), db.n, sc,
                                  db.d_out.data_ptr(), ctypes.c_void_p(s.cuda_stream),
                                  ctypes.byref(opts) if opts is not None else None))

    def extend_device_matrix(self, db: DeviceBatch, matrix, gap: int,
                             stream: Optional[torch.cuda.Stream] = None,
                             opts: Optional[Opts] = None):
        """Enqueues xdrop_extend_matrix: matrix[p][q] scores base p of A
        against base q of B (4 x 4, codes A=0 C=1 G=2 T=3)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        tbl = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32).reshape(16))
        _check(lib().xdrop_extend_matrix(
            self.h, db.d_a.data_ptr(), len(db.a_words), db.d_b.data_ptr(), len(db.b_words),
            db.d_pairs.data_ptr(), db.n, tbl.ctypes.data_as(ctypes.c_void_p), int(gap),
            db.d_out.data_ptr(), ctypes.c_void_p(s.cuda_stream),
            ctypes.byref(opts) if opts is not None else None))

    def extend_matrix(self, bt, matrix, gap: int, opts: Optional[Opts] = None) -> np.ndarray:
        """Synchronous convenience of extend_device_matrix."""
        db = DeviceBatch(bt, f"cuda:{self.device}")
        self.extend_device_matrix(db, matrix, gap, opts=opts)
        torch.cuda.synchronize(self.device)
        return db.results()

    def find_seeds_device(self, db: DeviceBatch, k: int = 17, width: int = 500,
                          set_pairs: bool = False, d_seeds: Optional[torch.Tensor] = None,
                          stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Enqueues xd_find_seeds over the batch's reads; returns the device
        buffer of xd_seed records.  With set_pairs the batch's pair records
        get the found seeds (and k)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        if d_seeds is None:
            d_seeds = torch.empty(max(db.n, 1) * SEED_DTYPE.itemsize, dtype=torch.uint8,
                                  device=db.d_pairs.device)
        _check(lib().xd_find_seeds(self.h, db.d_a.data_ptr(), len(db.a_words), db.d_b.data_ptr(),
                                   len(db.b_words), db.d_pairs.data_ptr(), db.n, int(k),
                                   int(width), int(bool(set_pairs)), d_seeds.data_ptr(),
                                   ctypes.c_void_p(s.cuda_stream)))
        return d_seeds

    def find_seeds(self, bt, k: int = 17, width: int = 500) -> np.ndarray:
        """Synchronous convenience: the xd_seed records of every pair of bt."""
        db = DeviceBatch(bt, f"cuda:{self.device}")
        d = self.find_seeds_device(db, k=k, width=width)
        torch.cuda.synchronize(self.device)
        return d[: db.n * SEED_DTYPE.itemsize].cpu().numpy().view(SEED_DTYPE).copy()

    def extend(self, bt, opts: Optional[Opts] = None, device: Optional[str] = None) -> np.ndarray:
        """Synchronous convenience: upload, extend, download."""
        db = DeviceBatch(bt, device or f"cuda:{self.device}")
        self.extend_device(db, opts=opts)
        torch.cuda.synchronize(self.device)
        return db.results()

    def extend_host(self, bt, opts: Optional[Opts] = None) -> np.ndarray:
        """xdrop_extend_host: host arrays in, host results out."""
        return self.extend_host_packed(pack_codes(bt.a), pack_codes(bt.b), make_pairs(bt),
                                       bt.scores, opts)

    def extend_host_packed(self, a_words: np.ndarray, b_words: np.ndarray, pairs: np.ndarray,
                           scores: Sequence[int], opts: Optional[Opts] = None) -> np.ndarray:
        """xdrop_extend_host on packed arenas and xd_pair records held on the host."""
        a = np.ascontiguousarray(a_words, dtype=np.uint32)
        b = np.ascontiguousarray(b_words, dtype=np.uint32)
        pr = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
        out = np.zeros(len(pr), RESULT_DTYPE)
        _check(lib().xdrop_extend_host(
            self.h, a.ctypes.data_as(ctypes.c_void_p), len(a), b.ctypes.data_as(ctypes.c_void_p),
            len(b), pr.ctypes.data_as(ctypes.c_void_p), len(pr), Scores(*scores),
            out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts) if opts is not None else None))
        return out

    def memory(self) -> int:
        """xd_ctx_memory: device bytes the context holds."""
        b = ctypes.c_uint64()
        _check(lib().xd_ctx_memory(self.h, ctypes.byref(b)))
        return b.value

    def stats(self) -> dict:
        """xd_last_stats: per-tier jobs / cells / escalations / restarts, stage times."""
        st = Stats()
        _check(lib().xd_last_stats(self.h, ctypes.byref(st)))
        out = {"jobs": np.array(list(st.jobs), np.int64),
               "cells": np.array(list(st.cells), np.int64),
               "escalated": np.array(list(st.escalated), np.int64),
               "restarted": np.array(list(st.restarted), np.int64),
               "wasted_cells": np.array(list(st.wasted_cells), np.int64)}
        if st.profiled:
            out["stage_ms"] = np.array(list(st.stage_ms), np.float64)
        return out


NOALLOC_MAX_PAIRS = 8192


def extend_noalloc(db: DeviceBatch, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                   opts: Optional[Opts] = None, scores: Optional[Sequence[int]] = None):
    """Enqueues xdrop_extend_noalloc (no context, no device allocation) on
    ``stream`` (default: torch's current stream of ``device``)."""
    s = stream if stream is not None else torch.cuda.current_stream(device)
    sc = Scores(*(scores if scores is not None else db.scores))
    _check(lib().xdrop_extend_noalloc(device, db.d_a.data_ptr(), len(db.a_words),
                                      db.d_b.data_ptr(), len(db.b_words), db.d_pairs.data_ptr(),
                                      db.n, sc, db.d_out.data_ptr(),
                                      ctypes.c_void_p(s.cuda_stream),
                                      ctypes.byref(opts) if opts is not None else None))


class PackedRequest:
    """A request ready to submit: packed reads and pair records on the host."""

    def __init__(self, bt):
        self.n = bt.n
        self.a_words = pack_codes(bt.a)
        self.b_words = pack_codes(bt.b)
        self.pairs = make_pairs(bt)
        self.req = Request(self.a_words.ctypes.data, len(self.a_words), self.b_words.ctypes.data,
                           len(self.b_words), self.pairs.ctypes.data, bt.n, Scores(*bt.scores))


class Server:
    """xd_server: continuous batching of extension requests on one device."""

    def __init__(self, device: int = 0, slots: int = 4, max_batch_pairs: int = 2048,
                 graph: int = 0, mem_budget: int = 0, opts: Optional[Opts] = None,
                 group_by_class: int = 1, watchdog_ms: int = 0):
        torch.cuda.init()
        o = ServerOpts()
        o.device, o.slots, o.max_batch_pairs, o.graph = device, slots, max_batch_pairs, graph
        o.mem_budget = mem_budget
        o.group_by_class = group_by_class
        o.watchdog_ms = watchdog_ms
        o.extend_opts = opts if opts is not None else make_opts()
        h = ctypes.c_void_p()
        _check(lib().xd_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def submit(self, req: PackedRequest) -> int:
        t = ctypes.c_uint64()
        _check(lib().xd_server_submit(self.h, ctypes.byref(req.req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, n_pairs: int, wait_ms: int = -1):
        """(results, done_ns) once the ticket is done, else None."""
        out = np.zeros(n_pairs, RESULT_DTYPE)
        done = ctypes.c_uint64()
        st = lib().xd_server_poll(self.h, ticket, out.ctypes.data_as(ctypes.c_void_p), wait_ms,
                                  ctypes.byref(done))
        if st == XD_ENOTREADY:
            return None
        _check(st)
        return out, done.value

    def cancel(self, ticket: int) -> int:
        """xd_server_cancel: XD_OK if the request left the queue, XD_EBUSY if
        it is already on the device or done."""
        st = lib().xd_server_cancel(self.h, ticket)
        if st not in (XD_OK, XD_EBUSY):
            _check(st)
        return st

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().xd_server_get_stats(self.h, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            lib().xd_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
