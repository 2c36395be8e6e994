"""Pins of the oracle's loop statistics: rounds started, the size of the graph
the loop stopped at (kernel_n), the level of the bound's witness
(witness_level, -1 when the exact solve gave the cut), the status bits
(COLLAPSED, DISCONNECTED, NO_PROGRESS, MAX_ROUNDS) and the returned side.

Every expected value below is derived by hand in the case's comment from the
method's steps (Section 4.1: label propagation, cluster contraction, the
Padberg-Rinaldi conditions, the minimum-degree bound of Section 4; the loop
of Algorithm 1 in appendix A) under the readings the build takes (synchronous
label propagation with keep-own-label ties, strict conditions 2 and 3, one
PR pass per round, a round that leaves n unchanged stops the loop). Where a
derivation holds for every tie-break priority it is checked over several
seeds. Nothing here was produced by the oracle or the GPU library.

Facts used repeatedly (fmix32 is a bijection, so distinct labels never tie
on priority):
  * Unit K_n, n >= 3, two LP iterations: let a be the vertex of smallest
    priority and b the second smallest. Iteration 1 (labels = ids, every
    S(x) = 1, the own label scores 0): every v != a takes a, and a takes b.
    Iteration 2: for v not in {a, b}, S(a) = n - 2 > S(b) = 1 and v already
    holds a; b holds a and S(a) = n - 2 is the maximum; a sees every
    neighbour labelled a (S(a) = n - 1) and moves to a. One cluster.
    For n = 3 the same holds through the keep-own-label rule (b and the
    third vertex see S(a) = S(b) and already hold a).
  * Two unit K_a (a >= 5) joined by one edge of weight 1: the argument
    above runs inside each block (the bridge adds at most 1 to a foreign
    label, against >= a - 3 >= 2 for the block's label), so two LP
    iterations leave exactly the two blocks as clusters.
  * Unit K_5: condition 4 marks every edge (1 + 3 common neighbours = 4 =
    lambda-hat).
"""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import cut_value, load_golden, side_from_words

COLL, DISC, NOPR, MAXR = oracle.ST_COLLAPSED, oracle.ST_DISCONNECTED, oracle.ST_NO_PROGRESS, oracle.ST_MAX_ROUNDS
SEEDS = [0, 1, 7, 12345]


def run(g, lp, n0, max_rounds=64, seed=0):
    return oracle.mincut_graph(g, lp_iters=lp, n0=n0, max_rounds=max_rounds, seed=seed)


def stats(r):
    return (r.cut, r.rounds, r.kernel_n, r.witness_level, r.status)


def side_set(r, n):
    return set(np.flatnonzero(side_from_words(r.side, n)).tolist())


def cycle(n, weights):
    return gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)], weights)


# ----------------------------------------------------------- NO_PROGRESS ----
@pytest.mark.parametrize("n", [5, 6, 11, 40])
def test_unit_cycle_without_lp_makes_no_progress(n):
    """Unit C_n (n >= 5), no LP, n0 = 1. lambda-hat_0 = 2 with witness vertex
    0. Every edge: condition 1 (1 >= 2) fails, condition 2 (2 < 2) fails,
    adjacent cycle vertices have no common neighbour for n >= 4 (conditions
    3 and 4: 1 >= 2 fails). No mark, so n is unchanged: the round ends with
    NO_PROGRESS after 1 round and the exact solve on C_n gives 2, which does
    not beat lambda-hat: the witness {0} (level 0) is returned, normalised
    to V minus {0}."""
    g = cycle(n, [1] * n)
    r = run(g, 0, 1)
    assert stats(r) == (2, 1, n, 0, NOPR)
    assert side_set(r, n) == set(range(1, n))


def test_weighted_cycle_without_lp_makes_no_progress():
    """C_6 with weight 3 (the golden file): lambda-hat_0 = 6, condition 1
    (3 >= 6), 2 (6 < 6), 4 (3 >= 6) all fail and there are no common
    neighbours: NO_PROGRESS after 1 round, the cut 6 is the level-0 bound."""
    g, _ = load_golden("cycle6_w3.txt")
    r = run(g, 0, 1)
    assert stats(r) == (6, 1, 6, 0, NOPR)
    assert side_set(r, 6) == {1, 2, 3, 4, 5}


@pytest.mark.parametrize("n", [12, 20])
def test_alternating_cycle_progress_then_no_progress(n):
    """C_n (n even, n/2 >= 5... here 12 and 20) with weights 2, 1, 2, 1, ...
    on edges (0,1), (1,2), ...; no LP, n0 = 1. Every vertex has degree 3:
    lambda-hat_0 = 3, witness 0. Round 1: a weight-2 edge {v, v+1} has
    c(v) = 3 < 2*2 (condition 2), a weight-1 edge meets none (1 >= 3, 3 < 2,
    no common neighbours). The marked edges form a perfect matching
    {0,1}, {2,3}, ...; contracting it leaves a unit C_{n/2} (ids by smallest
    member: coarse 0 = {0,1}) of degree 2 < 3: lambda-hat = 2, witness
    coarse vertex 0 at level 1. Progress (n -> n/2), so round 2 starts:
    the unit cycle C_{n/2} meets no condition (as above): NO_PROGRESS after
    2 rounds, kernel n/2; the exact solve's 2 does not beat lambda-hat.
    Side {0,1} normalised: V minus {0,1}.
    A NO_PROGRESS test placed before the PR contraction would stop round 1
    at kernel n; an off-by-one round count would give 1 or 3."""
    g = cycle(n, [2 if i % 2 == 0 else 1 for i in range(n)])
    r = run(g, 0, 1)
    assert stats(r) == (2, 2, n // 2, 1, NOPR)
    assert side_set(r, n) == set(range(2, n))


# ------------------------------------------------------------ MAX_ROUNDS ----
@pytest.mark.parametrize("lp", [0, 2])
def test_zero_round_cap(lp):
    """max_rounds = 0 with n > n0: the cap is hit before the first round:
    MAX_ROUNDS, 0 rounds, the exact solve runs on the input. Unit C_7:
    lambda = delta = 2, so the level-0 witness {0} is kept."""
    g = cycle(7, [1] * 7)
    r = run(g, lp, 1, max_rounds=0)
    assert stats(r) == (2, 0, 7, 0, MAXR)


def test_zero_round_cap_exact_solve_beats_the_bound():
    """Barbell (two unit K5 joined by one edge, lambda = 1, delta = 4) with
    max_rounds = 0: no round runs, the exact solve on the input gives 1 < 4,
    so witness_level = -1 and the side is the block {5..9} (after the
    normalisation that keeps vertex 0 on side 0)."""
    g, _ = load_golden("barbell.txt")
    r = run(g, 2, 1, max_rounds=0)
    assert stats(r) == (1, 0, 10, -1, MAXR)
    assert side_set(r, 10) == set(range(5, 10))


def test_round_cap_after_one_round():
    """The alternating C_12 of test_alternating_cycle_progress_then_no_progress
    with max_rounds = 1: round 1 contracts to a unit C_6 (lambda-hat 2 at
    level 1); 6 > n0 and 1 round >= the cap: MAX_ROUNDS with rounds = 1 and
    kernel_n = 6; the exact solve's 2 does not beat lambda-hat."""
    g = cycle(12, [2 if i % 2 == 0 else 1 for i in range(12)])
    r = run(g, 0, 1, max_rounds=1)
    assert stats(r) == (2, 1, 6, 1, MAXR)
    assert side_set(r, 12) == set(range(2, 12))


# -------------------------------------------------------------- COLLAPSED ----
@pytest.mark.parametrize("n", [3, 4, 9, 30])
@pytest.mark.parametrize("seed", SEEDS)
def test_unit_clique_collapses_in_one_round(n, seed):
    """Unit K_n, two LP iterations, n0 = 1: one cluster (module docstring),
    so the cluster contraction leaves one vertex: COLLAPSED after 1 round,
    kernel 1. The cut is lambda-hat_0 = n - 1 with witness vertex 0 at
    level 0 (lambda = delta: nothing lowers it); side V minus {0}."""
    g = gg.from_edges(n, list(itertools.combinations(range(n), 2)))
    r = run(g, 2, 1, seed=seed)
    assert stats(r) == (n - 1, 1, 1, 0, COLL)
    assert side_set(r, n) == set(range(1, n))


@pytest.mark.parametrize("lp", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", SEEDS)
def test_k5_collapses_for_every_lp(lp, seed):
    """Unit K_5, n0 = 1, lambda = delta = 4.
    lp = 0: condition 4 marks every edge: one vertex after round 1.
    lp = 1: every v != a takes label a and a takes b: clusters V minus {a}
      and {a}, joined by weight 4 = lambda-hat: condition 1 marks it.
    lp = 2, 3: one cluster (module docstring; a third iteration keeps it).
    In every case COLLAPSED after 1 round, witness 0 at level 0."""
    g, _ = load_golden("k5_unit.txt")
    r = run(g, lp, 1, seed=seed)
    assert stats(r) == (4, 1, 1, 0, COLL)
    assert side_set(r, 5) == {1, 2, 3, 4}


@pytest.mark.parametrize("lp", [2, 3])
@pytest.mark.parametrize("seed", SEEDS)
def test_barbell_collapses_through_the_bridge(lp, seed):
    """Barbell, lp >= 2, n0 = 1: LP gives the two blocks (module docstring);
    the block with the smaller label values ({0..4}) becomes coarse vertex 0.
    Level 1: two vertices joined by weight 1, degree 1 < 4: lambda-hat = 1,
    witness coarse 0 at level 1. Condition 1 (1 >= 1) marks the bridge: the
    PR contraction collapses the graph in the same round. COLLAPSED, 1
    round, cut 1, side {5..9}."""
    g, _ = load_golden("barbell.txt")
    r = run(g, lp, 1, seed=seed)
    assert stats(r) == (1, 1, 1, 1, COLL)
    assert side_set(r, 10) == set(range(5, 10))


def test_barbell_without_lp_takes_two_rounds():
    """Barbell, no LP, n0 = 1, lambda-hat_0 = 4. Round 1: every block edge
    has 3 common neighbours, so condition 4 gives 1 + 3 = 4 >= 4; the bridge
    meets none (1 >= 4, 5 < 2, no common neighbour). Contraction: two
    vertices (coarse 0 = {0..4}) with degree 1: lambda-hat = 1 at level 1.
    Round 2: condition 1 marks the bridge, the graph collapses. COLLAPSED
    after 2 rounds, witness level 1, cut 1, side {5..9}."""
    g, _ = load_golden("barbell.txt")
    r = run(g, 0, 1)
    assert stats(r) == (1, 2, 1, 1, COLL)
    assert side_set(r, 10) == set(range(5, 10))


def test_strict_pr_fixture_without_lp():
    """strict_pr (two K4 of weight 5 joined through vertex 8 by weight-2
    edges to 0 and 4), no LP, n0 = 1. lambda-hat_0 = 4 (vertex 8). Round 1:
    block edges meet condition 1 (5 >= 4); the weight-2 edges meet none
    (2 >= 4; 4 < 4 and 17 < 4 fail; 0 and 8 have no common neighbour).
    Contraction: A = {0..3} -> 0, B = {4..7} -> 1, 8 -> 2, degrees 2, 2, 4:
    lambda-hat = 2 with witness coarse 0 at level 1. Round 2: both edges
    meet condition 1 (2 >= 2): collapse. COLLAPSED, 2 rounds, cut 2, side
    A normalised: {4, ..., 8}."""
    g, _ = load_golden("strict_pr.txt")
    r = run(g, 0, 1)
    assert stats(r) == (2, 2, 1, 1, COLL)
    assert side_set(r, 9) == {4, 5, 6, 7, 8}


@pytest.mark.parametrize("seed", SEEDS)
def test_strict_pr_fixture_with_lp(seed):
    """strict_pr with two LP iterations: each K4 block becomes one cluster
    (the clique argument; vertex 0's extra weight-2 neighbour cannot beat
    the block's 10). Vertex 8 sees labels L1(0) in {1,2,3} and L1(4) in
    {5,6,7} with weight 2 each, its own label (0 or 4) scores 0, so it moves
    to one of them: it joins a block or stays a singleton, depending on the
    priorities. Either way level 1 has a vertex of degree 2 < 4
    (lambda-hat = 2 at level 1) and every remaining edge has weight 2 or 4
    >= 2, so condition 1 collapses the graph in round 1. The returned side
    is one block, with or without vertex 8."""
    g, _ = load_golden("strict_pr.txt")
    r = run(g, 2, 1, seed=seed)
    assert stats(r) == (2, 1, 1, 1, COLL)
    assert side_set(r, 9) in ({4, 5, 6, 7}, {4, 5, 6, 7, 8})


def test_weighted_path_without_lp_takes_two_rounds():
    """Path 0-1-2-3 with weights 7, 2, 9; degrees 7, 9, 11, 9; no LP, n0 = 1.
    Round 1 (lambda-hat 7): edges of weight 7 and 9 meet condition 1; the
    weight-2 edge meets none. Contraction: {0,1} -> 0, {2,3} -> 1 joined by
    weight 2: lambda-hat = 2 at level 1. Round 2: condition 1 (2 >= 2)
    collapses it. COLLAPSED after 2 rounds, witness level 1, cut 2, side
    {2, 3}."""
    g, _ = load_golden("weighted_path4.txt")
    r = run(g, 0, 1)
    assert stats(r) == (2, 2, 1, 1, COLL)
    assert side_set(r, 4) == {2, 3}


@pytest.mark.parametrize("seed", SEEDS)
def test_weighted_path_with_lp_counts_identity_contractions(seed):
    """Same path with two LP iterations. Iteration 1: 0 -> 1, 1 -> 0 (7 > 2),
    2 -> 3 (9 > 2), 3 -> 2. Iteration 2: 0 sees label 0 (7) and moves to 0;
    1 sees labels 1 (7) and 3 (2), moves to 1; 2 sees 0 (2) and 2 (9), moves
    to 2; 3 moves to 3. The labels are the identity again, for every seed
    (no ties occur). The cluster contraction is the identity but still a
    contraction (level 1), the bound stays 7. PR as without LP contracts to
    two vertices at level 2: lambda-hat = 2, witness level 2. Round 2: on
    two vertices LP oscillates again (level 3, identity) and condition 1
    collapses the graph (level 4). COLLAPSED, 2 rounds, witness level 2."""
    g, _ = load_golden("weighted_path4.txt")
    r = run(g, 2, 1, seed=seed)
    assert stats(r) == (2, 2, 1, 2, COLL)
    assert side_set(r, 4) == {2, 3}


# ----------------------------------------------------------- DISCONNECTED ----
@pytest.mark.parametrize("lp", [0, 2])
@pytest.mark.parametrize("seed", SEEDS)
def test_two_triangles_disconnect_after_one_round(lp, seed):
    """Two disjoint triangles of weight 4, n0 = 1, lambda-hat_0 = 8.
    lp = 0: each triangle edge has a common neighbour u with 8 < 2(4 + 4)
    at both ends (condition 3): every edge is marked. lp = 2: each triangle
    becomes one cluster (the clique argument for n = 3). Either way level 1
    has two isolated vertices: lambda-hat = 0, DISCONNECTED after 1 round,
    witness coarse 0 = {0,1,2} at level 1, side {3,4,5}."""
    g, _ = load_golden("two_triangles_disconnected.txt")
    r = run(g, lp, 1, seed=seed)
    assert stats(r) == (0, 1, 2, 1, DISC)
    assert side_set(r, 6) == {3, 4, 5}


def test_isolated_vertex_disconnects_at_level_zero():
    """A vertex of degree 0 in the input: lambda-hat_0 = 0, the loop never
    starts: 0 rounds, kernel = the input, DISCONNECTED, witness the isolated
    vertex at level 0."""
    g = gg.from_edges(5, [(0, 1), (1, 2), (2, 3)])
    r = run(g, 2, 1)
    assert stats(r) == (0, 0, 5, 0, DISC)
    assert side_set(r, 5) == {4}


# ----------------------------------------------------- n <= n0 at the start ----
@pytest.mark.parametrize("name,cut,level,side", [
    ("barbell.txt", 1, -1, set(range(5, 10))),          # lambda 1 < delta 4: the exact solve wins
    ("strict_pr.txt", 2, -1, None),                      # lambda 2 < delta 4
    ("weighted_path4.txt", 2, -1, {2, 3}),               # lambda 2 < delta 7
    ("k5_unit.txt", 4, 0, {1, 2, 3, 4}),                 # lambda = delta: the level-0 witness stays
    ("cycle6_w3.txt", 6, 0, {1, 2, 3, 4, 5}),            # lambda = delta
])
def test_no_round_when_the_input_is_small(name, cut, level, side):
    """n <= n0: no round starts (rounds 0, status 0, kernel = input); the
    exact solve gives lambda, which replaces the bound only if strictly
    smaller than delta (witness_level -1), else the level-0 witness (the
    smallest vertex of minimum degree) stays."""
    g, _ = load_golden(name)
    for lp in (0, 2):
        r = run(g, lp, 100)
        assert stats(r) == (cut, 0, g.n, level, 0)
        if side is not None:
            assert side_set(r, g.n) == side
        assert cut_value(g, side_from_words(r.side, g.n)) == cut


# ----------------------------------------------------------- any graph ----
@pytest.mark.parametrize("seed", range(40))
def test_loop_statistics_are_consistent(seed):
    """Properties of the loop statistics that hold on every input:
    at most one stop bit; MAX_ROUNDS iff the cap was reached with more than
    n0 vertices left; a plain exit (no bit) means kernel_n <= n0; COLLAPSED
    means one vertex; DISCONNECTED means cut 0; witness_level -1 means the
    exact solve beat the level-0 bound delta."""
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(4, 60))
    from helpers import random_graph
    g = random_graph(n, float(rng.uniform(0.05, 0.5)), int(rng.choice([1, 3, 50])), 7000 + seed,
                     connected=bool(seed % 5))
    delta = int(g.degrees().min())
    for lp, n0, cap in [(0, 1, 64), (2, 1, 64), (2, 3, 1), (1, 2, 2), (3, 1, 0)]:
        r = run(g, lp, n0, max_rounds=cap, seed=seed)
        bits = [b for b in (COLL, DISC, NOPR, MAXR) if r.status & b]
        assert len(bits) <= 1 and r.status & ~(COLL | DISC | NOPR | MAXR) == 0
        assert 0 <= r.rounds <= cap
        if r.status & MAXR:
            assert r.rounds == cap and r.kernel_n > n0
        if r.status == 0:
            assert r.kernel_n <= n0
        if r.status & COLL:
            assert r.kernel_n == 1
        if r.status & NOPR:
            assert r.kernel_n > n0 and r.rounds >= 1
        if r.status & DISC:
            assert r.cut == 0
        if r.witness_level == -1:
            assert r.cut < delta and not r.status & (COLL | DISC)
        else:
            assert r.witness_level >= 0
        if r.rounds == 0:
            assert r.kernel_n == n and r.witness_level in (0, -1)
