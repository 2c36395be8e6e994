"""Shared helpers of the GPU parity tests: device copies of host graphs, and
canonical forms of the oracle's and the library's trace records."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(g):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.col, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.w, np.int32)).cuda())


def side_words(t, n):
    words = (n + 63) // 64
    return t.cpu().numpy().view(np.uint64)[:words].copy()


def canon(events, graphs_from_contract=True):
    """Comparable form of a trace: PR marks become the set of marked
    undirected edges (the oracle marks both arcs, the library the v < x one)."""
    out = []
    cur = None
    for ev in events:
        k = ev["kind"]
        if k == 1:
            out.append(("lp", ev["round"], ev["iter"], ev["labels"].tobytes()))
        elif k == 6:
            out.append(("fix", ev["round"], ev["labels"].tobytes()))
        elif k == 2:
            out.append(("graph", ev["level"], ev["row_ptr"].tobytes(), ev["col"].tobytes(), ev["w"].tobytes(),
                        ev["deg"].tobytes(), ev["cl"].tobytes()))
            cur = ev
        elif k == 3:
            out.append(("bound", ev["level"], ev["lam_hat"], ev["witness_vertex"], ev["witness_level"]))
        elif k == 4:
            out.append(("pr_lam", ev["level"], ev["lam_hat"]))
            out.append(("pr", ev["level"], ev["mark"]))  # resolved below against the graph
        elif k == 5:
            out.append(("uf", ev["level"], ev["rep"].tobytes()))
    return out


def marked_edges(row_ptr, col, mark):
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    m = np.asarray(mark) != 0
    a = np.minimum(rows[m], col[m])
    b = np.maximum(rows[m], col[m])
    return sorted(set(zip(a.tolist(), b.tolist())))


def canon_with_graphs(events, g0):
    """canon(), with PR marks resolved to edge sets using the graph they refer to."""
    out = []
    rp, col = g0.row_ptr, g0.col
    for ev in events:
        k = ev["kind"]
        if k == 2:
            rp, col = ev["row_ptr"], ev["col"]
        if k == 4:
            out.append(("pr", ev["level"], ev["lam_hat"], tuple(marked_edges(rp, col, ev["mark"]))))
        else:
            out.extend(canon([ev]))
    return out
