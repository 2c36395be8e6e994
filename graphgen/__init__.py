"""Seeded synthetic graph generators (test and benchmark inputs only).

Nothing in here computes any part of the minimum-cut method: the module
builds the input graphs that the CPU oracle and the GPU library are both run
on. The native part (``graphgen.cpp``) is compiled with g++ on first use, or
by ``__graft_entry__.build()``.

Every graph is returned as a :class:`Graph` holding a symmetric int32 CSR
(``row_ptr[n+1]``, ``col[nnz]``, ``w[nnz]``), rows strictly increasing, no
self loops, weights >= 1.

Workload recipes (shapes of the paper's instance families, see the paper's
instance appendix):

* :func:`planted` - two random blocks joined by a few cross edges;
* :func:`rhg` - random hyperbolic graph, threshold model, power-law exponent
  gamma (the paper uses gamma = 5, average degree 2^5..2^8);
* :func:`rmat_core` - R-MAT, duplicates merged into weights, k-core on
  distinct-neighbour degree, largest connected component (stands in for the
  paper's real-world k-core instances, whose datasets are not used here).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the native generator library in-tree."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Out(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pad", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("col", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_int32)), ("info", ctypes.c_double * 8)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.gg_planted.restype = vp
        lib.gg_planted.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64]
        lib.gg_rhg.restype = vp
        lib.gg_clustered_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_uint64]
        lib.gg_clustered_er.restype = vp
        lib.gg_rhg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_uint64, ctypes.c_int32]
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        lib.gg_from_edges.restype = vp
        lib.gg_from_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        lib.gg_kcore_lcc.restype = vp
        lib.gg_kcore_lcc.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, ctypes.c_int32]
        lib.gg_rhg_expected_degree.restype = ctypes.c_double
        lib.gg_rhg_expected_degree.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric int32 CSR graph held in host memory."""
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        """Weighted degree per vertex (int64)."""
        cs = np.concatenate([[0], np.cumsum(self.w, dtype=np.int64)])
        return cs[self.row_ptr[1:]] - cs[self.row_ptr[:-1]]


def _take(ptr, name, info_keys=()) -> Graph:
    lib = _load()
    o = ctypes.cast(ptr, ctypes.POINTER(_Out)).contents
    n, nnz = o.n, o.nnz
    rp = np.ctypeslib.as_array(o.row_ptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(o.col, shape=(max(nnz, 1),))[:nnz].copy()
    w = np.ctypeslib.as_array(o.w, shape=(max(nnz, 1),))[:nnz].copy()
    info = {k: float(o.info[i]) for i, k in enumerate(info_keys)}
    lib.gg_free(ptr)
    return Graph(rp, col, w, name, info)


def planted(n: int, d: float, kx: int, wlo: int = 1, whi: int = 1, seed: int = 0) -> Graph:
    """Planted-cut graph: a seeded random permutation splits the vertices into
    blocks of floor(n/2) and ceil(n/2); each block is a random Hamiltonian
    cycle plus uniformly random distinct pairs up to round(n_b*d/2) edges;
    ``kx`` distinct random cross pairs join the blocks; weights uniform in
    [wlo, whi]."""
    p = _load().gg_planted(int(n), float(d), int(kx), int(wlo), int(whi), int(seed) & (2**64 - 1))
    return _take(p, "planted(n=%d,d=%g,kx=%d,w=[%d,%d],seed=%d)" % (n, d, kx, wlo, whi, seed), ("kx",))


def clustered_er(n: int, d: float, k: int, seed: int = 0) -> Graph:
    """Clustered Erdos-Renyi graph: each pair is an edge with probability
    d / 100, weights uniform in [1, 100], multiplied by n inside a cluster;
    k balanced clusters from a seeded permutation."""
    p = _load().gg_clustered_er(int(n), float(d), int(k), int(seed) & (2**64 - 1))
    return _take(p, "clustered_er(n=%d,d=%g,k=%d,seed=%d)" % (n, d, k, seed), ("k",))


def rhg(n: int, avg_deg: float, gamma: float = 5.0, seed: int = 0, wlo: int = 1, whi: int = 1,
        lcc: bool = True) -> Graph:
    """Threshold random hyperbolic graph with n points, target average degree
    ``avg_deg`` and power-law exponent ``gamma``; the disk radius is chosen
    from the model's expected degree and corrected until the realised average
    degree is within 1 %. Vertex ids follow angular order; with ``lcc`` the
    largest connected component is kept and renumbered in that order."""
    p = _load().gg_rhg(int(n), float(avg_deg), float(gamma), int(wlo), int(whi), int(seed) & (2**64 - 1),
                       1 if lcc else 0)
    return _take(p, "rhg(n=%d,deg=%g,gamma=%g,seed=%d)" % (n, avg_deg, gamma, seed), ("R", "avg_deg", "n_gen"))


def rmat_core(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19, seed: int = 0,
              kcore: int = 10, lcc: bool = True) -> Graph:
    """R-MAT with 2^scale vertices and ef*2^scale samples, self loops dropped,
    symmetrised with duplicate pairs merged into the weight; then the k-core
    on distinct-neighbour degree and its largest connected component."""
    p = _load().gg_rmat(int(scale), int(ef), float(a), float(b), float(c), int(seed) & (2**64 - 1), int(kcore),
                        1 if lcc else 0)
    return _take(p, "rmat(scale=%d,ef=%d,core=%d,seed=%d)" % (scale, ef, kcore, seed),
                 ("n_raw", "nnz_raw", "n_core"))


def from_edges(n: int, edges, weights=None) -> Graph:
    """Symmetric CSR from an undirected edge list; duplicate pairs are summed."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    if np.any(e[:, 0] == e[:, 1]):
        raise ValueError("self loops are not allowed")
    u = np.ascontiguousarray(e[:, 0])
    v = np.ascontiguousarray(e[:, 1])
    wv = np.ascontiguousarray(np.ones(len(e), np.int32) if weights is None else np.asarray(weights, np.int32))
    p = _load().gg_from_edges(int(n), len(e), u.ctypes.data, v.ctypes.data, wv.ctypes.data)
    return _take(p, "edges(n=%d,m=%d)" % (n, len(e)))


def kcore_lcc(g: Graph, k: int, lcc: bool = True) -> Graph:
    p = _load().gg_kcore_lcc(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, g.w.ctypes.data, int(k),
                             1 if lcc else 0)
    return _take(p, g.name + "|core%d" % k)


def rhg_expected_degree(n: int, R: float, gamma: float = 5.0) -> float:
    return float(_load().gg_rhg_expected_degree(int(n), float(R), float(gamma)))


# ----------------------------------------------------------------- recipes
def c1_planted(seed: int = 0) -> Graph:
    """Planted cut, n = 2,000: two blocks of 1,000, average degree 32, unit
    weights, 5 cross edges."""
    return planted(2000, 32.0, 5, 1, 1, seed)


def c2_rhg(seed: int = 1) -> Graph:
    """Random hyperbolic graph, n = 2^20, average degree 32, gamma = 5, unit
    weights (the shape of the paper's smallest RHG point)."""
    return rhg(1 << 20, 32.0, 5.0, seed)


def c3_rmat(seed: int = 2, scale: int = 22) -> Graph:
    """R-MAT scale 22, edge factor 16, a/b/c = 0.57/0.19/0.19, 10-core, LCC."""
    return rmat_core(scale, 16, 0.57, 0.19, 0.19, seed, 10, True)


def c4_params(count: int = 4096, seed: int = 3):
    """Per-graph parameters of the planted batch: n ~ U{64..8192},
    d ~ U[8, 64], w ~ U{1..100}, k_x ~ U{1..20}; graph i uses seed + i."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(64, 8193, size=count)
    ds = rng.uniform(8.0, 64.0, size=count)
    kx = rng.integers(1, 21, size=count)
    return [(int(ns[i]), float(ds[i]), int(kx[i]), 1, 100, seed + i) for i in range(count)]


def c4_batch(count: int = 4096, seed: int = 3, members=None, threads: int = 0):
    """The planted batch (or the listed members of it), generated on a
    thread pool (the generator releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    ps = c4_params(count, seed)
    idx = list(range(count)) if members is None else list(members)
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda i: planted(*ps[i]), idx))


def c5_request_params(count: int, seed: int = 4):
    """Served-stream request mix: n log-uniform in [100, 2^20]; half RHG
    (gamma 5, average degree U[16, 64]), half planted (d U[8, 64],
    k_x U{1..20}); weights U{1..100}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(100), math.log(1 << 20)))))
        if rng.random() < 0.5:
            out.append(("rhg", n, float(rng.uniform(16.0, 64.0)), seed * 1000003 + i))
        else:
            out.append(("planted", n, float(rng.uniform(8.0, 64.0)), int(rng.integers(1, 21)), seed * 1000003 + i))
    return out


def c5_make(p) -> Graph:
    if p[0] == "rhg":
        _, n, deg, s = p
        return rhg(max(n, 8), deg, 5.0, s, 1, 100, True)
    _, n, d, kx, s = p
    return planted(n, d, kx, 1, 100, s)


def reweight_device(row_ptr, col, seed: int):
    """Fresh symmetric weights U{1..100} for a device CSR (torch int32 tensors,
    rows sorted by column): every undirected edge {u, v} gets one draw of a
    seeded torch generator on the tensors' device, shared by its two arcs.
    Used to make each request of a served stream a distinct weighted graph on
    a topology drawn from a pool."""
    import torch
    dev = col.device
    n = row_ptr.numel() - 1
    nnz = col.numel()
    if nnz == 0:
        return torch.zeros(0, dtype=torch.int32, device=dev)
    rows = torch.repeat_interleave(torch.arange(n, device=dev, dtype=torch.int64),
                                   (row_ptr[1:] - row_ptr[:-1]).to(torch.int64))
    c = col.to(torch.int64)
    keys = rows * n + c               # ascending: rows ascend, columns ascend within a row
    rev = torch.searchsorted(keys, c * n + rows)   # position of the reverse arc (v, u)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) & (2**63 - 1))
    draw = torch.randint(1, 101, (nnz,), generator=gen, device=dev, dtype=torch.int32)
    return torch.where(rows < c, draw, draw[rev]).contiguous()
