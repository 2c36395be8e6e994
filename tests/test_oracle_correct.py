"""Pins of the oracle's correcting step (Section 4.1, "correcting algorithm";
fixMisplacedVertices in Algorithm 1), under the reading the build takes: after
label propagation a cluster C with 2 <= |C| <= floor(log2 n) loses at most one
vertex, the member v whose removal leaves C - {v} with the smallest weighted
degree in the contracted graph (smallest v on ties), and only if that degree is
strictly below the minimum weighted degree of the contracted graph without
corrections; the removed vertex becomes a singleton with label n + v.

The pins: the misplaced-vertex situation of the paper's figure, built by hand
with every cut derived in the comments; the size limit; and, on small random
graphs and clusterings, brute force from the definition of a cut's capacity
(the weighted degree of a cluster in the contracted graph is the capacity of
the cut around it in G, Section 3)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import brute_mincut, cut_value, random_graph, side_from_words


def figure_graph():
    """The situation of the misplaced-vertex figure: A = {0, 1} (edge weight
    10); the centre vertex 2 has weight 2 to each of 0 and 1 (4 to A) and
    weight 3 to B = {3, 4, 5} and to D = {6, 7, 8} (triangles of weight 5,
    joined by (4, 7) and (5, 8) of weight 5). Label propagation's choice for
    2 is A (4 > 3), which gives the clusters {0,1,2}, B, D.
    Weighted degrees of the contracted graph: {0,1,2}: 3 + 3 = 6;
    B: 3 + 5 + 5 = 13; D: 13; minimum 6.
    Removing 0 from {0,1,2}: {1,2} has 10 + 2 + 3 + 3 = 18; removing 1: 18;
    removing 2: {0,1} has 2 + 2 = 4 < 6, so vertex 2 is misplaced.
    B without 3: {4,5}: 5 + 5 + 5 + 5 = 20; without 4: {3,5}: 5 + 5 + 3 + 5
    = 18; without 5: 18; D the same: nothing below 6.
    The minimum cut of G is 4 ({0,1} against the rest; every vertex has
    degree >= 10), which the uncorrected contraction loses (its minimum
    degree is 6) and the corrected one keeps (the singleton 2 separates
    {0,1}, of degree 4)."""
    e = [(0, 1, 10), (0, 2, 2), (1, 2, 2), (2, 3, 3), (2, 6, 3),
         (3, 4, 5), (3, 5, 5), (4, 5, 5), (6, 7, 5), (6, 8, 5), (7, 8, 5), (4, 7, 5), (5, 8, 5)]
    return gg.from_edges(9, [(a, b) for a, b, _ in e], [c for _, _, c in e])


def test_figure_case_makes_the_centre_a_singleton():
    g = figure_graph()
    labels = np.array([0, 0, 0, 3, 3, 3, 6, 6, 6])
    out = oracle.fix_misplaced(g.row_ptr, g.col, g.w, labels)
    assert out.tolist() == [0, 0, 9 + 2, 3, 3, 3, 6, 6, 6]
    lam, _ = brute_mincut(g)
    assert lam == 4


def test_figure_case_cluster_over_the_size_limit_is_kept():
    """The same situation with A = {0, 1, 9} (9 joined to 0 and 1 by weight
    10): the cluster {0, 1, 2, 9} has 4 members, above floor(log2 10) = 3,
    so it is not checked (A's degree without 2 would be 4 < 6)."""
    g0 = figure_graph()
    rows = np.repeat(np.arange(g0.n), np.diff(g0.row_ptr))
    keep = rows < g0.col
    e = list(zip(rows[keep].tolist(), g0.col[keep].tolist()))
    wts = g0.w[keep].tolist()
    e += [(0, 9), (1, 9)]
    wts += [10, 10]
    g = gg.from_edges(10, e, wts)
    labels = np.array([0, 0, 0, 3, 3, 3, 6, 6, 6, 0])
    assert oracle.fix_misplaced(g.row_ptr, g.col, g.w, labels).tolist() == labels.tolist()
    # with 16 vertices (six more in a heavy path hanging off vertex 8) the
    # limit is 4 and the centre is removed
    e2 = e + [(8, 10), (10, 11), (11, 12), (12, 13), (13, 14), (14, 15)]
    g2 = gg.from_edges(16, e2, wts + [50] * 6)
    lab2 = np.concatenate([labels, np.arange(10, 16)])
    out = oracle.fix_misplaced(g2.row_ptr, g2.col, g2.w, lab2)
    want = lab2.copy()
    want[2] = 16 + 2
    assert out.tolist() == want.tolist()


def test_singletons_and_a_single_cluster_are_never_changed():
    g = figure_graph()
    ident = np.arange(g.n)
    assert oracle.fix_misplaced(g.row_ptr, g.col, g.w, ident).tolist() == ident.tolist()
    one = np.zeros(g.n, np.int64)  # one cluster of 9 > 3 members, degree 0
    assert oracle.fix_misplaced(g.row_ptr, g.col, g.w, one).tolist() == one.tolist()


def brute_fix(g, labels):
    """The correcting step from the definition: cluster degrees as capacities
    of cuts of G (helpers.cut_value), every candidate removal evaluated as
    its own cut."""
    n = g.n
    limit = int(np.floor(np.log2(n)))
    clusters = {}
    for v in range(n):
        clusters.setdefault(int(labels[v]), []).append(v)

    def cap(vs):
        side = np.zeros(n, bool)
        side[vs] = True
        return cut_value(g, side)
    delta_c = min(cap(m) for m in clusters.values())
    out = np.array(labels, dtype=np.int64)
    for lab, mem in clusters.items():
        if not 2 <= len(mem) <= limit:
            continue
        vals = [(cap([x for x in mem if x != v]), v) for v in mem]
        best, v = min(vals)
        if best < delta_c:
            out[v] = n + v
    return out


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_on_random_clusterings(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(4, 40))
    g = random_graph(n, float(rng.uniform(0.08, 0.5)), int(rng.choice([1, 3, 20])), 9000 + seed,
                     connected=bool(seed % 4))
    k = int(rng.integers(1, max(2, n // 2)))
    labels = rng.integers(0, n, size=k)[rng.integers(0, k, size=n)]  # k (or fewer) random label values
    assert oracle.fix_misplaced(g.row_ptr, g.col, g.w, labels).tolist() == brute_fix(g, labels).tolist()


@pytest.mark.parametrize("seed", range(30))
def test_method_with_the_correcting_step_keeps_the_sandwich(seed):
    """With the correcting step the method still returns a genuine cut of
    capacity between lambda and the minimum degree."""
    rng = np.random.default_rng(9500 + seed)
    n = int(rng.integers(6, 15))
    g = random_graph(n, float(rng.uniform(0.2, 0.7)), int(rng.choice([1, 3, 10])), 9500 + seed)
    lam, _ = brute_mincut(g)
    r = oracle.mincut_graph(g, lp_iters=2, n0=1, seed=seed, correct=True, trace=True)
    side = side_from_words(r.side, g.n)
    assert not side[0] and 0 < side.sum() < g.n
    assert cut_value(g, side) == r.cut
    assert lam <= r.cut <= int(g.degrees().min())
    # every correction event is the step applied to the round's last LP
    # labels on the graph of that round
    cur = (g.row_ptr, g.col, g.w)
    last = None
    for ev in r.events:
        if ev["kind"] == oracle.EV_CONTRACT:
            cur = (ev["row_ptr"], ev["col"], ev["w"])
        elif ev["kind"] == oracle.EV_LP:
            last = ev["labels"]
        elif ev["kind"] == oracle.EV_FIX:
            assert ev["labels"].tolist() == oracle.fix_misplaced(*cur, last).tolist()


def test_correcting_step_recovers_the_figure_minimum_cut():
    """Whole method on the figure graph with the clustering forced by one LP
    iteration is not controllable, so the contraction is checked directly:
    contracting the corrected clustering keeps lambda = 4 (Lemma 1 applies:
    {0,1} | 2 | B | D respects the minimum cut {0,1}), the uncorrected one
    has minimum degree 6."""
    g = figure_graph()
    labels = np.array([0, 0, 0, 3, 3, 3, 6, 6, 6])
    fixed = oracle.fix_misplaced(g.row_ptr, g.col, g.w, labels)

    def contracted_min_degree(lab):
        vals = []
        for x in np.unique(lab):
            vals.append(cut_value(g, lab == x))
        return min(vals)
    assert contracted_min_degree(labels) == 6
    assert contracted_min_degree(fixed) == 4
