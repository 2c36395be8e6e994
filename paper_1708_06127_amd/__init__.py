"""MI355X (gfx950) inexact minimum cut - Python binding of libviecut.so.

The binding only marshals arguments into the C ABI declared in
``include/viecut.h``; every step of the method runs in the HIP library.
PyTorch provides device memory and streams. If the library is missing or
cannot be loaded, every call raises: there is no CPU fallback.

Usage::

    import torch, paper_1708_06127_amd as vc
    cut, side, info = vc.mincut(row_ptr, col, w, n0=10000)   # int32 CUDA tensors

``side`` holds ceil(n/64) words (torch.int64 view of uint64): bit u&63 of
word u>>6 is 1 iff vertex u is on the side without vertex 0.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libviecut.so")

OK, EINVAL, EWEIGHT, EOVERFLOW, ENOMEM, EDEVICE, ENOTSYM, EBUDGET, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES = 64 << 20  # VIECUT_NOALLOC_SCRATCH_BYTES
ST_COLLAPSED, ST_DISCONNECTED, ST_NO_PROGRESS, ST_MAX_ROUNDS = 1, 2, 4, 8
F_VALIDATE, F_CORRECT, F_CONVERGE, F_RESTRICT = 1, 2, 4, 8
EXPORTED = ["viecut_default_params", "viecut_workspace_bytes", "viecut_mincut", "viecut_mincut_noalloc",
            "viecut_mincut_trace",
            "viecut_validate", "viecut_batch_workspace_bytes", "viecut_mincut_batch", "viecut_session_create",
            "viecut_session_submit", "viecut_session_step", "viecut_session_poll", "viecut_session_destroy",
            "viecut_profile_enable", "viecut_profile_read", "viecut_tuning_set", "viecut_tuning_clear",
            "viecut_tuning_get", "viecut_strerror"]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("lp_iters", ctypes.c_int32), ("n0", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("rounds", ctypes.c_int32), ("kernel_n", ctypes.c_int32),
                ("witness_level", ctypes.c_int32), ("status_bits", ctypes.c_uint32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_ms", ctypes.c_float * 8)]

    def as_dict(self):
        return {"cut": int(self.cut), "rounds": int(self.rounds), "kernel_n": int(self.kernel_n),
                "witness_level": int(self.witness_level), "status": int(self.status_bits),
                "levels": int(self.levels), "t_ms": [float(x) for x in self.t_ms]}


class Event(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("round", ctypes.c_int32), ("iter", ctypes.c_int32),
                ("level", ctypes.c_int32), ("n", ctypes.c_int32), ("n_prev", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("lam_hat", ctypes.c_int64), ("witness_vertex", ctypes.c_int32),
                ("witness_level", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_int32)),
                ("b", ctypes.POINTER(ctypes.c_int32)), ("c", ctypes.POINTER(ctypes.c_int32)),
                ("d", ctypes.POINTER(ctypes.c_int64)), ("e", ctypes.POINTER(ctypes.c_int32))]


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(Event))


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class ViecutError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("viecut error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Load libviecut.so (built by ``paper_1708_06127_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libviecut.so is not built (run __graft_entry__.build() or "
                           "python paper_1708_06127_amd/build.py)")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so that one runtime serves torch's memory and the library's launches
    _torch()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    lib.viecut_default_params.argtypes = [P(Params)]
    lib.viecut_default_params.restype = None
    lib.viecut_workspace_bytes.argtypes = [i32, i32, P(Params)]
    lib.viecut_workspace_bytes.restype = sz
    lib.viecut_mincut.argtypes = [P(Csr), P(Params), vp, sz, vp, P(Result), vp]
    lib.viecut_mincut.restype = ctypes.c_int
    lib.viecut_mincut_noalloc.argtypes = [P(Csr), P(Params), vp, P(Result), vp]
    lib.viecut_mincut_noalloc.restype = ctypes.c_int
    lib.viecut_mincut_trace.argtypes = [P(Csr), P(Params), vp, sz, vp, P(Result), vp, TRACE_FN, vp]
    lib.viecut_mincut_trace.restype = ctypes.c_int
    lib.viecut_validate.argtypes = [P(Csr), u32, vp]
    lib.viecut_validate.restype = ctypes.c_int
    lib.viecut_strerror.argtypes = [ctypes.c_int]
    lib.viecut_strerror.restype = ctypes.c_char_p
    if hasattr(lib, "viecut_mincut_batch"):
        lib.viecut_batch_workspace_bytes.argtypes = [P(Csr), i32, P(Params)]
        lib.viecut_batch_workspace_bytes.restype = sz
        lib.viecut_mincut_batch.argtypes = [P(Csr), i32, P(Params), vp, sz, vp, P(Result), P(vp)]
        lib.viecut_mincut_batch.restype = ctypes.c_int
    if hasattr(lib, "viecut_session_create"):
        lib.viecut_session_create.argtypes = [sz, P(Params), vp, P(vp)]
        lib.viecut_session_create.restype = ctypes.c_int
        lib.viecut_session_submit.argtypes = [vp, P(Csr), vp, ctypes.c_int64]
        lib.viecut_session_submit.restype = ctypes.c_int
        lib.viecut_session_step.argtypes = [vp, P(i32)]
        lib.viecut_session_step.restype = ctypes.c_int
        lib.viecut_session_poll.argtypes = [vp, P(ctypes.c_int64), P(Result), i32]
        lib.viecut_session_poll.restype = ctypes.c_int
        lib.viecut_session_destroy.argtypes = [vp]
        lib.viecut_session_destroy.restype = None
    lib.viecut_profile_enable.argtypes = [ctypes.c_int]
    lib.viecut_profile_enable.restype = ctypes.c_int
    lib.viecut_profile_read.argtypes = [P(KernelStat), i32]
    lib.viecut_profile_read.restype = ctypes.c_int
    lib.viecut_tuning_set.argtypes = [ctypes.c_int64, ctypes.c_char_p, ctypes.c_int64]
    lib.viecut_tuning_set.restype = ctypes.c_int
    lib.viecut_tuning_clear.argtypes = []
    lib.viecut_tuning_clear.restype = ctypes.c_int
    lib.viecut_tuning_get.argtypes = [ctypes.c_char_p, sz]
    lib.viecut_tuning_get.restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().viecut_strerror(code).decode()


def _check(code: int):
    if code != OK:
        raise ViecutError(code, strerror(code))


def params(lp_iters=2, n0=10000, max_rounds=64, seed=0, validate=False, correct=False, converge=False,
           restrict=False) -> Params:
    p = Params()
    load().viecut_default_params(ctypes.byref(p))
    p.lp_iters, p.n0, p.max_rounds = int(lp_iters), int(n0), int(max_rounds)
    p.seed = int(seed) & (2**64 - 1)
    p.flags = ((F_VALIDATE if validate else 0) | (F_CORRECT if correct else 0) | (F_CONVERGE if converge else 0) |
               (F_RESTRICT if restrict else 0))
    return p


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def csr(row_ptr, col, w) -> Csr:
    """C descriptor for int32 CUDA tensors (kept alive by the caller)."""
    torch = _torch()
    for t in (row_ptr, col, w):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise TypeError("row_ptr, col and w must be contiguous int32 CUDA tensors")
    c = Csr()
    c.n = row_ptr.numel() - 1
    c.nnz = col.numel()
    c.row_ptr, c.col, c.w = row_ptr.data_ptr(), col.data_ptr(), w.data_ptr()
    return c


def workspace_bytes(n: int, nnz: int, p: Params | None = None) -> int:
    p = p or params()
    return int(load().viecut_workspace_bytes(int(n), int(nnz), ctypes.byref(p)))


def workspace(n: int, nnz: int, p: Params | None = None, device="cuda"):
    """Device workspace tensor for repeated solves of graphs up to (n, nnz)."""
    torch = _torch()
    return torch.empty(workspace_bytes(n, nnz, p), dtype=torch.uint8, device=device)


@dataclass
class TraceLog:
    events: list = field(default_factory=list)


def _event_dict(ev):
    import numpy as np

    def arr(p, count, dt):
        if count <= 0:
            return np.zeros(0, dt)
        return np.ctypeslib.as_array(p, shape=(int(count),)).copy().astype(dt, copy=False)
    k = ev.kind
    d = {"kind": k, "round": ev.round, "iter": ev.iter, "level": ev.level, "n": ev.n}
    if k in (1, 6):
        d["labels"] = arr(ev.a, ev.n, np.int32)
    elif k == 2:
        d["row_ptr"] = arr(ev.a, ev.n + 1, np.int32)
        d["col"] = arr(ev.b, ev.nnz, np.int32)
        d["w"] = arr(ev.c, ev.nnz, np.int32)
        d["deg"] = arr(ev.d, ev.n, np.int64)
        d["cl"] = arr(ev.e, ev.n_prev, np.int32)
    elif k == 3:
        d["lam_hat"] = int(ev.lam_hat)
        d["witness_vertex"] = int(ev.witness_vertex)
        d["witness_level"] = int(ev.witness_level)
    elif k == 4:
        d["mark"] = arr(ev.a, ev.nnz, np.int32)
        d["lam_hat"] = int(ev.lam_hat)
    elif k == 5:
        d["rep"] = arr(ev.a, ev.n, np.int32)
    return d


def mincut(row_ptr, col, w, *, lp_iters=2, n0=10000, max_rounds=64, seed=0, validate=False, correct=False,
           converge=False, restrict=False, ws=None, side=None, stream=None, trace=False):
    """Solve one graph given as int32 CUDA tensors. Returns (cut, side, info).
    ``correct``, ``converge`` and ``restrict`` turn on the correcting step,
    the label-propagation convergence stop and the first-iteration
    restriction (VIECUT_F_CORRECT / _CONVERGE / _RESTRICT)."""
    torch = _torch()
    lib = load()
    g = csr(row_ptr, col, w)
    p = params(lp_iters, n0, max_rounds, seed, validate, correct, converge, restrict)
    words = (g.n + 63) // 64
    if side is None:
        side = torch.empty(max(words, 1), dtype=torch.int64, device=row_ptr.device)
    res = Result()
    ws_ptr, ws_bytes = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
    sp = _stream_ptr(stream)
    if trace:
        log = TraceLog()
        cb = TRACE_FN(lambda _u, evp: log.events.append(_event_dict(evp.contents)))
        rc = lib.viecut_mincut_trace(ctypes.byref(g), ctypes.byref(p), ws_ptr, ws_bytes, sp, ctypes.byref(res),
                                     side.data_ptr(), cb, None)
    else:
        rc = lib.viecut_mincut(ctypes.byref(g), ctypes.byref(p), ws_ptr, ws_bytes, sp, ctypes.byref(res),
                               side.data_ptr())
    _check(rc)
    info = res.as_dict()
    if trace:
        info["events"] = log.events
    return int(res.cut), side, info


def mincut_noalloc(row_ptr, col, w, *, side, lp_iters=2, n0=10000, max_rounds=64, seed=0, validate=False,
                   stream=None):
    """viecut_mincut_noalloc: the same solve on the library's static device
    scratch (no allocation inside the call; ``side`` must be given).
    Returns (cut, side, info)."""
    lib = load()
    g = csr(row_ptr, col, w)
    p = params(lp_iters, n0, max_rounds, seed, validate)
    res = Result()
    _check(lib.viecut_mincut_noalloc(ctypes.byref(g), ctypes.byref(p), _stream_ptr(stream), ctypes.byref(res),
                                     side.data_ptr()))
    return int(res.cut), side, res.as_dict()


def validate(row_ptr, col, w, *, check_symmetry=True, stream=None) -> int:
    """Device-side input validation; returns the status code (0 = valid)."""
    g = csr(row_ptr, col, w)
    return int(load().viecut_validate(ctypes.byref(g), F_VALIDATE if check_symmetry else 0, _stream_ptr(stream)))


def _graph_csrs(graphs):
    cs = (Csr * max(len(graphs), 1))()
    for i, (rp, col, w) in enumerate(graphs):
        cs[i] = csr(rp, col, w)
    return cs


def batch_workspace_bytes(graphs, p: Params | None = None) -> int:
    p = p or params()
    return int(load().viecut_batch_workspace_bytes(_graph_csrs(graphs), len(graphs), ctypes.byref(p)))


def mincut_batch(graphs, *, lp_iters=2, n0=10000, max_rounds=64, seed=0, validate=False, ws=None, sides=None,
                 stream=None):
    """Solve many graphs (a list of (row_ptr, col, w) int32 CUDA tensors) in
    one batched execution. Returns a list of (cut, side, info) tuples; a graph
    whose input is invalid gets (None, side, info) with info["error"] set to
    its status code, and the others are unaffected."""
    torch = _torch()
    lib = load()
    count = len(graphs)
    p = params(lp_iters, n0, max_rounds, seed, validate)
    cs = _graph_csrs(graphs)
    if sides is None:
        sides = [torch.empty(max((rp.numel() - 1 + 63) // 64, 1), dtype=torch.int64, device=rp.device)
                 for rp, _, _ in graphs]
    sp_arr = (ctypes.c_void_p * max(count, 1))(*[s.data_ptr() for s in sides])
    outs = (Result * max(count, 1))()
    ws_ptr, ws_bytes = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
    rc = lib.viecut_mincut_batch(cs, count, ctypes.byref(p), ws_ptr, ws_bytes, _stream_ptr(stream), outs, sp_arr)
    _check(rc)
    res = []
    for i in range(count):
        info = outs[i].as_dict()
        if info["status"] & 0x80000000:
            info["error"] = -(info["status"] & 0x7FFFFFFF)
            res.append((None, sides[i], info))
        else:
            res.append((int(outs[i].cut), sides[i], info))
    return res


class Session:
    """Served execution: requests stay resident on the device, are admitted
    while they fit the memory budget, and advance one batched round per
    step() together with the requests already in flight."""

    def __init__(self, hbm_budget: int, *, lp_iters=2, n0=10000, max_rounds=64, seed=0, validate=False,
                 stream=None):
        lib = load()
        self._p = params(lp_iters, n0, max_rounds, seed, validate)
        self._h = ctypes.c_void_p()
        self._keep = {}
        _check(lib.viecut_session_create(int(hbm_budget), ctypes.byref(self._p), _stream_ptr(stream),
                                         ctypes.byref(self._h)))

    def submit(self, request_id: int, row_ptr, col, w, side=None):
        torch = _torch()
        g = csr(row_ptr, col, w)
        if side is None:
            side = torch.empty(max((g.n + 63) // 64, 1), dtype=torch.int64, device=row_ptr.device)
        _check(load().viecut_session_submit(self._h, ctypes.byref(g), side.data_ptr(), int(request_id)))
        self._keep[int(request_id)] = (row_ptr, col, w, side)
        return side

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(load().viecut_session_step(self._h, ctypes.byref(n)))
        return int(n.value)

    def poll(self, max_results=4096):
        ids = (ctypes.c_int64 * max_results)()
        outs = (Result * max_results)()
        k = load().viecut_session_poll(self._h, ids, outs, max_results)
        if k < 0:
            _check(k)
        done = []
        for i in range(k):
            rid = int(ids[i])
            rp, col, w, side = self._keep.pop(rid)
            info = outs[i].as_dict()
            if info["status"] & 0x80000000:
                info["error"] = -(info["status"] & 0x7FFFFFFF)
                done.append((rid, None, side, info))
            else:
                done.append((rid, int(outs[i].cut), side, info))
        return done

    def close(self):
        if self._h:
            load().viecut_session_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    """Start (clearing the totals) or stop event timing of the arc-tile
    label-propagation kernels (see viecut_profile_enable)."""
    _check(load().viecut_profile_enable(1 if on else 0))


def profile_read():
    """Totals per timed kernel: {name: {"launches", "total_ms", "bytes"}}."""
    out = (KernelStat * 8)()
    k = load().viecut_profile_read(out, 8)
    if k < 0:
        _check(k)
    return {out[i].name.decode(): {"launches": int(out[i].launches), "total_ms": float(out[i].total_ms),
                                   "bytes": float(out[i].bytes)} for i in range(k)}


TUNING_KEYS = ("radix_large_from", "compact_direct_max", "pr_merge_tiles", "long_split", "emit_wave", "lp_group",
               "emit_group", "first_group", "huge_part")


def tuning_set(max_arcs: int, key: str, value: int):
    """Set one launch-shape choice for the size bucket bounded by max_arcs
    (< 0: unbounded); see viecut_tuning_set."""
    _check(load().viecut_tuning_set(int(max_arcs), key.encode(), int(value)))


def tuning_clear():
    _check(load().viecut_tuning_clear())


def tuning_get() -> str:
    lib = load()
    n = lib.viecut_tuning_get(None, 0)
    buf = ctypes.create_string_buffer(max(n, 1))
    lib.viecut_tuning_get(buf, len(buf))
    return buf.value.decode()


def tuning_load_text(text: str):
    """Replace the table by the one in `text` (the file format, as
    tuning_get returns it)."""
    tuning_clear()
    for line in text.splitlines():
        parts = line.split()
        if len(parts) < 2 or parts[0] != "bucket":
            continue
        bound = int(parts[1])
        for kv in parts[2:]:
            k, _, v = kv.partition("=")
            tuning_set(bound, k, int(v))
