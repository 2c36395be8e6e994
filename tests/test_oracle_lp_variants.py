"""Pins of the oracle's label-propagation variants (Section 4.1 and
appendix D, "Algorithm Configuration"), under the readings the build takes:

* convergence stop: iteration t is the last one when at most floor(n/10000)
  vertices got a label different from the one they had before it;
* first-iteration restriction (a synchronous reading of "a vertex may not
  leave its block once another vertex moved into it"): after iteration 1 of
  a round, every vertex that another vertex chose keeps its own label.

The pins are hand-derived label trajectories on graphs whose choices do not
depend on the priorities (or depend on them only through which vertex is
smallest, which the tests read back from the trace and then check for
consistency), and on random graphs the variants' definitions applied to the
plain method's own trajectories."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import random_graph


def hub_graph(leaves):
    """Triangle {0, 1, 2} of weight 100, every leaf joined to 0, 1 and 2 by
    weight 1. Iteration 1 (identity labels): a leaf sees S = 1 for each hub,
    so it takes the hub m of smallest priority; a hub sees its two partners
    at 100 each, so the two hubs other than m take m and m takes m2, the
    smaller-priority one of the other two. Iteration 2: a leaf has S(m) = 2,
    S(m2) = 1 and keeps m; the hubs other than m see S(m) = 100 + leaves and
    keep m; m sees S(m) = 200 + leaves and S(m2) = 0 and moves to m: one
    change. Iteration 3: every label is m, no change."""
    e, w = [(0, 1), (0, 2), (1, 2)], [100, 100, 100]
    for x in range(3, 3 + leaves):
        e += [(0, x), (1, x), (2, x)]
        w += [1, 1, 1]
    return gg.from_edges(3 + leaves, e, w)


def lp_events(r, rnd=0):
    return [ev for ev in r.events if ev["kind"] == oracle.EV_LP and ev["round"] == rnd]


def check_hub_trajectory(g, evs):
    n = g.n
    l1 = evs[0]["labels"]
    m = int(l1[3])
    assert m in (0, 1, 2) and np.all(l1[3:] == m)
    m2 = int(l1[m])
    assert m2 in (0, 1, 2) and m2 != m
    others = [h for h in (0, 1, 2) if h != m]
    assert all(int(l1[h]) == m for h in others)
    if len(evs) > 1:
        assert np.all(evs[1]["labels"] == m)  # only m changed
        assert int((evs[1]["labels"] != l1).sum()) == 1
    if len(evs) > 2:
        assert np.all(evs[2]["labels"] == m)
    return m, m2


@pytest.mark.parametrize("leaves,expect", [(9996, 3), (10000, 2)])
def test_convergence_stop_at_the_threshold(leaves, expect):
    """n = 9,999: the threshold floor(n/10000) is 0, so the stop comes after
    iteration 3 (no change); n = 10,003: threshold 1, and iteration 2 changes
    exactly one vertex, so it is the last."""
    g = hub_graph(leaves)
    r = oracle.mincut_graph(g, lp_iters=25, n0=1, seed=3, converge=True, trace=True)
    evs = lp_events(r)
    assert len(evs) == expect
    check_hub_trajectory(g, evs)
    assert r.kernel_n == 1 and r.status & oracle.ST_COLLAPSED


def test_without_the_stop_all_iterations_run():
    g = hub_graph(20)
    r = oracle.mincut_graph(g, lp_iters=7, n0=1, seed=3, trace=True)
    evs = lp_events(r)
    assert len(evs) == 7
    check_hub_trajectory(g, evs)
    for ev in evs[2:]:
        assert np.array_equal(ev["labels"], evs[2]["labels"])


def test_oscillating_matching_never_converges():
    """Heavy pairs (2i, 2i+1) of weight 10, consecutive pairs joined by
    weight 1: every vertex prefers its partner, so synchronous LP swaps the
    pair labels in every iteration and every vertex changes: all l
    iterations run with the stop."""
    k = 6
    e = [(2 * i, 2 * i + 1) for i in range(k)] + [(2 * i + 1, 2 * i + 2) for i in range(k - 1)]
    w = [10] * k + [1] * (k - 1)
    g = gg.from_edges(2 * k, e, w)
    r = oracle.mincut_graph(g, lp_iters=9, n0=1, seed=1, converge=True, trace=True)
    evs = lp_events(r)
    assert len(evs) == 9
    swap = np.arange(2 * k) ^ 1
    for t, ev in enumerate(evs, start=1):
        assert np.array_equal(ev["labels"], swap if t % 2 else np.arange(2 * k))


def test_restriction_on_the_hub_graph():
    """Choices of iteration 1: leaves and the hubs other than m choose m, m
    chooses m2. Chosen vertices m and m2 keep their labels; the rest keep
    their choice: m's cluster has every vertex but m2, and m2 is alone."""
    g = hub_graph(30)
    plain = lp_events(oracle.mincut_graph(g, lp_iters=1, n0=1, seed=5, trace=True))[0]["labels"]
    m, m2 = int(plain[3]), int(plain[int(plain[3])])
    r = oracle.mincut_graph(g, lp_iters=1, n0=1, seed=5, restrict=True, trace=True)
    l1 = lp_events(r)[0]["labels"]
    want = np.full(g.n, m)
    want[m2] = m2
    assert np.array_equal(l1, want)


def test_restriction_stops_the_pair_swap():
    """In the heavy-pair graph every vertex is chosen by its partner, so
    with the restriction nobody moves in iteration 1."""
    k = 5
    e = [(2 * i, 2 * i + 1) for i in range(k)] + [(2 * i + 1, 2 * i + 2) for i in range(k - 1)]
    g = gg.from_edges(2 * k, e, [10] * k + [1] * (k - 1))
    r = oracle.mincut_graph(g, lp_iters=1, n0=1, seed=2, restrict=True, trace=True)
    assert np.array_equal(lp_events(r)[0]["labels"], np.arange(2 * k))


@pytest.mark.parametrize("seed", range(30))
def test_variants_follow_their_definitions(seed):
    """On random connected graphs: the restricted iteration 1 is the plain
    iteration 1 with every chosen vertex put back; with the stop, the LP
    trajectory of round 0 is the plain trajectory cut after the first
    iteration that changes no label (n < 10000)."""
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(5, 60))
    g = random_graph(n, float(rng.uniform(0.05, 0.4)), int(rng.choice([1, 2, 9])), 700 + seed)
    plain = lp_events(oracle.mincut_graph(g, lp_iters=12, n0=1, seed=seed, max_rounds=1, trace=True))
    p1 = plain[0]["labels"]
    chosen = np.zeros(n, bool)
    moved = p1 != np.arange(n)
    chosen[p1[moved]] = True
    want = np.where(chosen, np.arange(n), p1)
    r = oracle.mincut_graph(g, lp_iters=1, n0=1, seed=seed, max_rounds=1, restrict=True, trace=True)
    assert np.array_equal(lp_events(r)[0]["labels"], want)
    prev = np.arange(n)
    stop = len(plain)
    for t, ev in enumerate(plain, start=1):
        if np.array_equal(ev["labels"], prev):
            stop = t
            break
        prev = ev["labels"]
    conv = lp_events(oracle.mincut_graph(g, lp_iters=12, n0=1, seed=seed, max_rounds=1, converge=True,
                                         trace=True))
    assert len(conv) == stop
    for a, b in zip(conv, plain):
        assert np.array_equal(a["labels"], b["labels"])
