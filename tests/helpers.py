"""Independent checking helpers for the tests: brute-force minimum cut,
cut capacity of a side, random small graphs. None of this shares code with
the oracle or the GPU library."""
from __future__ import annotations

import itertools

import numpy as np

import graphgen as gg


def edges_of(row_ptr, col, w):
    """Undirected edge list (u < v) with weights from a symmetric CSR."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    col = np.asarray(col, dtype=np.int64)
    keep = rows < col
    return rows[keep], col[keep], np.asarray(w, dtype=np.int64)[keep]


def cut_value(g, side_bool) -> int:
    """Capacity c(A) of the cut (A, V \\ A) given a bool per vertex (Section 3, Preliminaries)."""
    u, v, w = edges_of(g.row_ptr, g.col, g.w)
    s = np.asarray(side_bool, dtype=bool)
    return int(w[s[u] != s[v]].sum())


def brute_mincut(g):
    """lambda(G) = min over non-empty proper subsets A of c(A), by enumerating
    every bipartition (vertex n-1 fixed on the complement side). n <= 20."""
    n = g.n
    assert 2 <= n <= 20
    u, v, w = edges_of(g.row_ptr, g.col, g.w)
    masks = np.arange(1, 1 << (n - 1), dtype=np.int64)
    best = None
    arg = None
    chunk = 1 << 16
    for s in range(0, masks.size, chunk):
        m = masks[s:s + chunk]
        tot = np.zeros(m.size, np.int64)
        for a, b, c in zip(u, v, w):
            tot += c * (((m >> a) & 1) != ((m >> b) & 1))
        i = int(np.argmin(tot))
        if best is None or tot[i] < best:
            best, arg = int(tot[i]), int(m[i])
    side = np.array([(arg >> i) & 1 for i in range(n)], dtype=bool)
    return best, side


def all_min_sides(g):
    """Every minimum bipartition as a frozenset side without vertex n-1 (n <= 14)."""
    n = g.n
    u, v, w = edges_of(g.row_ptr, g.col, g.w)
    masks = np.arange(1, 1 << (n - 1), dtype=np.int64)
    tot = np.zeros(masks.size, np.int64)
    for a, b, c in zip(u, v, w):
        tot += c * (((masks >> a) & 1) != ((masks >> b) & 1))
    lam = int(tot.min())
    return lam, [int(m) for m in masks[tot == lam]]


def random_graph(n, p, wmax, seed, connected=True):
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
    if connected:
        perm = rng.permutation(n)
        pairs += [(int(min(perm[i], perm[i + 1])), int(max(perm[i], perm[i + 1]))) for i in range(n - 1)]
    pairs = sorted(set(pairs))
    if not pairs:
        pairs = [(0, 1)]
    ws = rng.integers(1, wmax + 1, size=len(pairs))
    return gg.from_edges(n, pairs, ws)


def side_from_words(words, n):
    bits = np.unpackbits(np.asarray(words, dtype=np.uint64).view(np.uint8), bitorder="little")
    return bits[:n].astype(bool)


def load_golden(name):
    """Parse a tests/golden fixture: returns (graph, facts) where facts holds
    the hand-derived '# key = value' lines."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    facts, rows = {}, []
    for line in open(path):
        line = line.strip()
        if not line:
            continue
        if line.startswith("#"):
            body = line[1:].strip()
            if " = " in body and body.split(" = ")[0] in ("lambda", "delta", "side"):
                k, v = body.split(" = ", 1)
                facts[k] = [int(x) for x in v.split()] if k == "side" else int(v)
            continue
        rows.append([int(x) for x in line.split()])
    n, m = rows[0]
    e = rows[1:]
    assert len(e) == m
    g = gg.from_edges(n, [(a, b) for a, b, _ in e], [c for _, _, c in e])
    return g, facts
