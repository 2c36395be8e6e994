"""CPU oracle - TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to ``viecut_oracle.cpp``: the plain, slow CPU
implementation of the synchronous inexact minimum-cut method that the GPU
library is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the GPU library
never calls it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "viecut_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

EV_LP, EV_CONTRACT, EV_BOUND, EV_PR, EV_UF, EV_FIX = 1, 2, 3, 4, 5, 6
F_CORRECT = 1
F_CONVERGE = 2
F_RESTRICT = 4
ST_COLLAPSED, ST_DISCONNECTED, ST_NO_PROGRESS, ST_MAX_ROUNDS = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile the oracle in-tree with g++ (OpenMP on the per-vertex LP loop)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Event(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("round", ctypes.c_int32), ("iter", ctypes.c_int32),
                ("level", ctypes.c_int32), ("n", ctypes.c_int32), ("n_prev", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("lam_hat", ctypes.c_int64), ("witness_vertex", ctypes.c_int32),
                ("witness_level", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_int32)),
                ("b", ctypes.POINTER(ctypes.c_int32)), ("c", ctypes.POINTER(ctypes.c_int32)),
                ("d", ctypes.POINTER(ctypes.c_int64)), ("e", ctypes.POINTER(ctypes.c_int32))]


_TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(_Event))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.oracle_splitmix64_output.restype = ctypes.c_uint64
        lib.oracle_splitmix64_output.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_fmix32.restype = ctypes.c_uint32
        lib.oracle_fmix32.argtypes = [ctypes.c_uint32]
        lib.oracle_prio.restype = ctypes.c_uint32
        lib.oracle_prio.argtypes = [ctypes.c_uint64, ctypes.c_int32]
        lib.oracle_stoer_wagner.restype = ctypes.c_int
        lib.oracle_stoer_wagner.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.oracle_mincut.restype = ctypes.c_int
        lib.oracle_mincut.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_uint32, vp, vp, vp, _TRACE_FN, vp]
        lib.oracle_fix_misplaced.restype = ctypes.c_int
        lib.oracle_fix_misplaced.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle error %d" % code)
        self.code = code


@dataclass
class Result:
    cut: int
    side: np.ndarray          # uint64 words, bit u set iff u is on the side without vertex 0
    rounds: int
    kernel_n: int
    witness_level: int
    status: int
    events: list = field(default_factory=list)

    def side_bool(self, n: int) -> np.ndarray:
        bits = np.unpackbits(self.side.view(np.uint8), bitorder="little")
        return bits[:n].astype(bool)


def _arr(p, count, dtype):
    if count == 0:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(p, shape=(int(count),)).copy().astype(dtype, copy=False)


def _csr_args(row_ptr, col, w):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, np.int32)
        ww = np.zeros(1, np.int32)
    return rp, c, ww


def splitmix64_output(seed: int, i: int) -> int:
    return int(_load().oracle_splitmix64_output(seed & (2**64 - 1), i))


def fmix32(h: int) -> int:
    return int(_load().oracle_fmix32(h & 0xFFFFFFFF))


def prio(s: int, x: int) -> int:
    return int(_load().oracle_prio(s & (2**64 - 1), x))


def stoer_wagner(row_ptr, col, w):
    """Exact minimum cut (value, bool side per vertex; no normalisation)."""
    rp, c, ww = _csr_args(row_ptr, col, w)
    n = rp.size - 1
    cut = ctypes.c_int64(0)
    side = np.zeros(max(n, 1), np.uint8)
    rc = _load().oracle_stoer_wagner(n, rp.ctypes.data, c.ctypes.data, ww.ctypes.data, ctypes.addressof(cut),
                                     side.ctypes.data)
    if rc:
        raise OracleError(rc)
    return int(cut.value), side[:n].astype(bool)


def fix_misplaced(row_ptr, col, w, labels):
    """The correcting step alone on given labels (values in [0, n)); returns the
    corrected labels (a removed vertex v gets label n + v)."""
    rp, c, ww = _csr_args(row_ptr, col, w)
    n = rp.size - 1
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(max(n, 1), np.int32)
    rc = _load().oracle_fix_misplaced(n, rp.ctypes.data, c.ctypes.data, ww.ctypes.data, lab.ctypes.data,
                                      out.ctypes.data)
    if rc:
        raise OracleError(rc)
    return out[:n]


def mincut(row_ptr, col, w, lp_iters: int = 2, n0: int = 10000, max_rounds: int = 64, seed: int = 0,
           trace: bool = False, correct: bool = False, converge: bool = False, restrict: bool = False) -> Result:
    """Run the whole method on a host CSR. With ``trace`` every intermediate
    state is recorded as a dict in ``Result.events``. ``correct``,
    ``converge`` and ``restrict`` turn on the correcting step, the
    convergence stop and the first-iteration restriction."""
    rp, c, ww = _csr_args(row_ptr, col, w)
    n = rp.size - 1
    words = max((n + 63) // 64, 1)
    side = np.zeros(words, np.uint64)
    info = np.zeros(4, np.int32)
    cut = ctypes.c_int64(0)
    events = []

    def on_event(_user, evp):
        ev = evp.contents
        k = ev.kind
        d = {"kind": k, "round": ev.round, "iter": ev.iter, "level": ev.level, "n": ev.n}
        if k in (EV_LP, EV_FIX):
            d["labels"] = _arr(ev.a, ev.n, np.int32)
        elif k == EV_CONTRACT:
            d["row_ptr"] = _arr(ev.a, ev.n + 1, np.int32)
            d["col"] = _arr(ev.b, ev.nnz, np.int32)
            d["w"] = _arr(ev.c, ev.nnz, np.int32)
            d["deg"] = _arr(ev.d, ev.n, np.int64)
            d["cl"] = _arr(ev.e, ev.n_prev, np.int32)
        elif k == EV_BOUND:
            d["lam_hat"] = int(ev.lam_hat)
            d["witness_vertex"] = int(ev.witness_vertex)
            d["witness_level"] = int(ev.witness_level)
        elif k == EV_PR:
            d["mark"] = _arr(ev.a, ev.nnz, np.int32)
            d["lam_hat"] = int(ev.lam_hat)
        elif k == EV_UF:
            d["rep"] = _arr(ev.a, ev.n, np.int32)
        events.append(d)

    cb = _TRACE_FN(on_event) if trace else _TRACE_FN()
    rc = _load().oracle_mincut(n, rp.ctypes.data, c.ctypes.data, ww.ctypes.data, int(lp_iters), int(n0),
                               int(max_rounds), int(seed) & (2**64 - 1),
                               (F_CORRECT if correct else 0) | (F_CONVERGE if converge else 0) |
                               (F_RESTRICT if restrict else 0),
                               ctypes.addressof(cut), side.ctypes.data,
                               info.ctypes.data, cb, None)
    if rc:
        raise OracleError(rc)
    return Result(int(cut.value), side, int(info[0]), int(info[1]), int(info[2]), int(info[3]), events)


def mincut_graph(g, **kw) -> Result:
    return mincut(g.row_ptr, g.col, g.w, **kw)
