"""ctypes wrapper of the C oracle (``xdrop_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xdrop_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SEED_SRC = os.path.join(HERE, "seed_oracle.c")
SEED_LIB = os.path.join(HERE, "libseedoracle.so")
NEG = -(1 << 63)

PAIR_FIELDS = ["score", "left_score", "right_score", "seed_score",
               "a_begin", "a_end", "b_begin", "b_end",
               "left_cells", "right_cells",
               "left_bi", "left_bj", "right_bi", "right_bj", "status"]
PAIR_DTYPE = np.dtype([(f, np.int64) for f in PAIR_FIELDS])


class _Ext(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("best", "bi", "bj", "cells", "ndiag", "wmax")]


class _Trace(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("n", ctypes.c_int64)] + [
        (f, ctypes.POINTER(ctypes.c_int64)) for f in ("lo", "hi", "la", "lb", "best", "vmax")]


def _compile(src: str, lib_path: str, force: bool) -> str:
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(src):
        tmp = lib_path + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-Wall",
                               "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, lib_path)
    return lib_path


def build(force: bool = False) -> str:
    """Compile the oracles with gcc (plain C, -O3, no intrinsics, no threads)."""
    _compile(SEED_SRC, SEED_LIB, force)
    return _compile(SRC, LIB, force)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.ox_extend.argtypes = [p, i64, p, i64, i64, i64, i64, i64,
                                ctypes.POINTER(_Ext), ctypes.POINTER(_Trace)]
        L.ox_extend.restype = ctypes.c_int
        L.ox_pair.argtypes = [p, i64, p, i64, i64, i64, i64, i64, i64, i64, i64, p]
        L.ox_pair.restype = ctypes.c_int
        L.ox_batch.argtypes = [p, p, p, p, p, p, p, p, p, i64, i64, i64, i64, i64, p]
        L.ox_batch.restype = ctypes.c_double
        L.ox_extend_matrix.argtypes = [p, i64, p, i64, p, i64, i64,
                                       ctypes.POINTER(_Ext), ctypes.POINTER(_Trace)]
        L.ox_extend_matrix.restype = ctypes.c_int
        L.ox_pair_matrix.argtypes = [p, i64, p, i64, i64, i64, i64, p, i64, i64, p]
        L.ox_pair_matrix.restype = ctypes.c_int
        L.ox_batch_matrix.argtypes = [p, p, p, p, p, p, p, p, p, i64, i64, p, i64, p]
        L.ox_batch_matrix.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.c_void_p)


def extend(a, b, match=1, mismatch=-1, gap=-1, x=10, trace: bool = False):
    """One extension of a against b (codes 0..3).  Returns a dict."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = _Ext()
    tr = None
    bufs = None
    if trace:
        cap = len(a) + len(b) + 1
        bufs = {f: np.zeros(cap, np.int64) for f in ("lo", "hi", "la", "lb", "best", "vmax")}
        tr = _Trace(cap, 0, *[bufs[f].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                              for f in ("lo", "hi", "la", "lb", "best", "vmax")])
    rc = lib().ox_extend(_ptr(a), len(a), _ptr(b), len(b), match, mismatch, gap, x,
                         ctypes.byref(out), ctypes.byref(tr) if tr is not None else None)
    if rc:
        raise ValueError("ox_extend rejected its arguments")
    res = {f: int(getattr(out, f)) for f in ("best", "bi", "bj", "cells", "ndiag", "wmax")}
    if trace:
        res["trace"] = {f: v[: tr.n].copy() for f, v in bufs.items()}
    return res


def _table(matrix) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(matrix, dtype=np.int64).reshape(16))
    return t


def extend_matrix(a, b, matrix, gap=-1, x=10, trace: bool = False):
    """One extension under a 4 x 4 substitution table (matrix[p][q] scores
    base p of a against base q of b).  Returns a dict."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    tbl = _table(matrix)
    out = _Ext()
    tr = None
    bufs = None
    if trace:
        cap = len(a) + len(b) + 1
        bufs = {f: np.zeros(cap, np.int64) for f in ("lo", "hi", "la", "lb", "best", "vmax")}
        tr = _Trace(cap, 0, *[bufs[f].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                              for f in ("lo", "hi", "la", "lb", "best", "vmax")])
    rc = lib().ox_extend_matrix(_ptr(a), len(a), _ptr(b), len(b), _ptr(tbl), gap, x,
                                ctypes.byref(out), ctypes.byref(tr) if tr is not None else None)
    if rc:
        raise ValueError("ox_extend_matrix rejected its arguments")
    res = {f: int(getattr(out, f)) for f in ("best", "bi", "bj", "cells", "ndiag", "wmax")}
    if trace:
        res["trace"] = {f: v[: tr.n].copy() for f, v in bufs.items()}
    return res


def pair_matrix(a, b, a_seed, b_seed, matrix, k=17, gap=-1, x=10) -> dict:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(1, PAIR_DTYPE)
    lib().ox_pair_matrix(_ptr(a), len(a), _ptr(b), len(b), a_seed, b_seed, k, _ptr(_table(matrix)),
                         gap, x, _ptr(out))
    return {f: int(out[f][0]) for f in PAIR_FIELDS}


def batch_matrix(bt, matrix, gap, return_time: bool = False):
    """Oracle results for a generator batch under a substitution table."""
    n = bt.n
    out = np.zeros(n, PAIR_DTYPE)
    arr = lambda v, dt: np.ascontiguousarray(v, dtype=dt)
    a = arr(bt.a, np.uint8) if len(bt.a) else np.zeros(1, np.uint8)
    b = arr(bt.b, np.uint8) if len(bt.b) else np.zeros(1, np.uint8)
    keep = [arr(bt.a_off, np.int64), arr(bt.a_len, np.int64), arr(bt.b_off, np.int64),
            arr(bt.b_len, np.int64), arr(bt.a_seed, np.int64), arr(bt.b_seed, np.int64),
            arr(bt.x, np.int32)]
    tbl = _table(matrix)
    secs = lib().ox_batch_matrix(_ptr(a), _ptr(b), *[_ptr(v) for v in keep], n, bt.k, _ptr(tbl),
                                 gap, _ptr(out))
    return (out, secs) if return_time else out


def pair(a, b, a_seed, b_seed, k=17, match=1, mismatch=-1, gap=-1, x=10) -> dict:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(1, PAIR_DTYPE)
    lib().ox_pair(_ptr(a), len(a), _ptr(b), len(b), a_seed, b_seed, k,
                  match, mismatch, gap, x, _ptr(out))
    return {f: int(out[f][0]) for f in PAIR_FIELDS}


def batch(bt, return_time: bool = False):
    """Oracle results for a generator batch, as a structured array."""
    n = bt.n
    out = np.zeros(n, PAIR_DTYPE)
    arr = lambda v, dt: np.ascontiguousarray(v, dtype=dt)
    a = arr(bt.a, np.uint8) if len(bt.a) else np.zeros(1, np.uint8)
    b = arr(bt.b, np.uint8) if len(bt.b) else np.zeros(1, np.uint8)
    keep = [arr(bt.a_off, np.int64), arr(bt.a_len, np.int64), arr(bt.b_off, np.int64),
            arr(bt.b_len, np.int64), arr(bt.a_seed, np.int64), arr(bt.b_seed, np.int64),
            arr(bt.x, np.int32)]
    m, mm, g = bt.scores
    secs = lib().ox_batch(_ptr(a), _ptr(b), *[_ptr(v) for v in keep], n, bt.k, m, mm, g,
                          _ptr(out))
    return (out, secs) if return_time else out


# ---------------------------------------------------------------------------
# seed choice (seed_oracle.c)
# ---------------------------------------------------------------------------
SEED_FIELDS = ["a_seed", "b_seed", "bin_matches", "matches", "found", "status"]
SEED_DTYPE = np.dtype([(f, np.int64) for f in SEED_FIELDS])
_seed_lib = None


def seed_lib():
    global _seed_lib
    if _seed_lib is None:
        build()
        L = ctypes.CDLL(SEED_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.os_find_seed.argtypes = [p, i64, p, i64, i64, i64, p]
        L.os_find_seed.restype = ctypes.c_int
        L.os_find_seeds.argtypes = [p, p, p, p, p, p, i64, i64, i64, p]
        L.os_find_seeds.restype = None
        _seed_lib = L
    return _seed_lib


def find_seed(a, b, k=17, width=500) -> dict:
    """Seed of one read pair by diagonal binning of its exact k-mer matches."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(1, SEED_DTYPE)
    seed_lib().os_find_seed(_ptr(a), len(a), _ptr(b), len(b), k, width, _ptr(out))
    return {f: int(out[f][0]) for f in SEED_FIELDS}


def find_seeds(bt, k=17, width=500) -> np.ndarray:
    """Seeds of every pair of a generator batch (its own seeds are ignored)."""
    out = np.zeros(bt.n, SEED_DTYPE)
    arr = lambda v, dt: np.ascontiguousarray(v, dtype=dt)
    a = arr(bt.a, np.uint8) if len(bt.a) else np.zeros(1, np.uint8)
    b = arr(bt.b, np.uint8) if len(bt.b) else np.zeros(1, np.uint8)
    keep = [arr(bt.a_off, np.int64), arr(bt.a_len, np.int64), arr(bt.b_off, np.int64),
            arr(bt.b_len, np.int64)]
    seed_lib().os_find_seeds(_ptr(a), _ptr(b), *[_ptr(v) for v in keep], bt.n, k, width,
                             _ptr(out))
    return out
