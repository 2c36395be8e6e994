"""GPU parity of the batched and served paths: every graph solved inside a
batch (one disjoint union on the device) or a session (requests joining while
others are in flight) must give exactly the oracle's result for that graph
alone - cut value, side bitmap, rounds, kernel size, witness level and status
bits - whatever else shares the device with it."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1708_06127_amd as vc
from gpu_common import log, side_words, to_dev
from helpers import load_golden, random_graph

pytestmark = pytest.mark.gpu

GOLDEN = ["strict_pr.txt", "cycle6_w3.txt", "k5_unit.txt", "barbell.txt", "weighted_path4.txt",
          "two_triangles_disconnected.txt"]


def hub_graph(seed, hub_deg):
    rng = np.random.default_rng(seed)
    n = hub_deg + 1
    e = [(0, i) for i in range(1, n)]
    for c in range(1, n - 8, 8):
        e += [(c + a, c + b) for a, b in itertools.combinations(range(8), 2)]
    e += [(i, i + 1) for i in range(1, n - 1)]
    e += [(int(a), int(b)) for a, b in rng.integers(1, n, (n, 2)) if a != b]
    return gg.from_edges(n, e, rng.integers(1, 5, len(e)))


def mixed_graphs():
    gs = [load_golden(name)[0] for name in GOLDEN]
    for seed in range(12):
        rng = np.random.default_rng(7000 + seed)
        n = int(rng.integers(3, 90))
        gs.append(random_graph(n, float(rng.uniform(0.03, 0.6)), int(rng.choice([1, 2, 7, 100])), 7000 + seed,
                               connected=bool(seed % 5)))
    gs += [gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)], [w] * n) for n, w in [(3, 1), (1000, 3)]]
    gs += [gg.from_edges(n, list(itertools.combinations(range(n), 2))) for n in (2, 33)]
    gs += [gg.c1_planted(s) for s in range(3)]
    gs += gg.c4_batch(4096, members=[5, 400, 2000])
    gs.append(gg.rhg(1 << 13, 32.0, 5.0, 3))
    gs.append(gg.rhg(6000, 24.0, 5.0, 9, wlo=1, whi=100))
    gs.append(hub_graph(700, 700))
    gs.append(hub_graph(9000, 9000))  # rows beyond 4096 arcs: the chunked path
    gs.append(gg.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4)]))  # isolated vertex
    return gs


def expect(g, kw):
    r = oracle.mincut_graph(g, **kw)
    return (r.cut, r.side.tobytes(), r.rounds, r.kernel_n, r.witness_level, r.status)


def got(g, cut, side, info):
    return (cut, side_words(side, g.n).tobytes(), info["rounds"], info["kernel_n"], info["witness_level"],
            info["status"])


@pytest.fixture(scope="module")
def mixed():
    gs = mixed_graphs()
    return gs, [to_dev(g) for g in gs]


@pytest.mark.parametrize("lp,n0,seed", [(2, 64, 0), (2, 1, 5), (0, 16, 0), (1, 100, 3), (3, 2, 11),
                                        (2, 10000, 0)])
def test_batch_equals_oracle(mixed, lp, n0, seed):
    gs, dev = mixed
    kw = dict(lp_iters=lp, n0=n0, seed=seed)
    log("batch", len(gs), "graphs", kw)
    res = vc.mincut_batch(dev, **kw)
    for i, (g, (cut, side, info)) in enumerate(zip(gs, res)):
        assert "error" not in info, (i, info)
        assert got(g, cut, side, info) == expect(g, kw), (i, g.n, kw)


def test_batch_max_rounds(mixed):
    gs, dev = mixed
    kw = dict(lp_iters=2, n0=1, seed=2, max_rounds=1)
    res = vc.mincut_batch(dev, **kw)
    for i, (g, (cut, side, info)) in enumerate(zip(gs, res)):
        assert got(g, cut, side, info) == expect(g, kw), (i, g.n)


def test_batch_order_and_company_do_not_matter(mixed):
    """A graph's result does not depend on its neighbours in the union."""
    gs, dev = mixed
    kw = dict(lp_iters=2, n0=8, seed=1)
    full = vc.mincut_batch(dev, **kw)
    order = list(reversed(range(len(gs))))
    rev = vc.mincut_batch([dev[i] for i in order], **kw)
    for j, i in enumerate(order):
        assert got(gs[i], *rev[j]) == got(gs[i], *full[i]), i
    for i in (0, 9, len(gs) - 3):
        alone = vc.mincut_batch([dev[i]], **kw)[0]
        assert got(gs[i], *alone) == got(gs[i], *full[i]), i


def test_batch_input_errors_are_per_graph():
    import torch
    ok = [gg.c1_planted(0), gg.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)])]
    good = [to_dev(g) for g in ok]
    base = gg.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    rp, col, w = to_dev(base)
    w0 = w.clone()
    w0[2] = 0
    c_out = col.clone()
    c_out[0] = 99
    c_self = col.clone()
    c_self[0] = 0
    r_bad = rp.clone()
    r_bad[2] = 100
    big = to_dev(gg.from_edges(3, [(0, 1), (1, 2)], [2**31 - 1, 5]))
    w_asym = w.clone()
    w_asym[0] = 3
    cases = [(rp, col, w0, vc.EWEIGHT), (rp, c_out, w, vc.EINVAL), (rp, c_self, w, vc.EINVAL),
             (r_bad, col, w, vc.EINVAL), (*big, vc.EOVERFLOW), (rp, col, w_asym, vc.ENOTSYM)]
    graphs = [good[0]] + [c[:3] for c in cases] + [good[1]]
    res = vc.mincut_batch(graphs, lp_iters=2, n0=1, validate=True)
    for (r, (_, _, _, code)) in zip(res[1:-1], cases):
        assert r[2].get("error") == code, (r[2], code)
    for g, r in zip(ok, (res[0], res[-1])):
        assert got(g, *r) == expect(g, dict(lp_iters=2, n0=1, seed=0))
    torch.cuda.synchronize()


def test_batch_c4_members_vs_single_path():
    """256 members of the planted batch: batched == the single-graph path, and
    a sample == the oracle."""
    members = list(range(0, 4096, 16))
    gs = gg.c4_batch(4096, members=members)
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=0)
    res = vc.mincut_batch(dev, **kw)
    for i, (g, d, r) in enumerate(zip(gs, dev, res)):
        one = vc.mincut(*d, **kw)
        assert got(g, *r) == got(g, *one), (members[i], g.n)
        if i % 32 == 0:
            assert got(g, *r) == expect(g, kw), members[i]


def test_batch_c4_full_sample():
    """The whole 4,096-graph planted batch in one call (9.4 million segments at
    the first contraction: the LDS-window compaction): sampled members ==
    the single-graph path, and a few == the oracle."""
    import torch
    gs = gg.c4_batch(4096)
    log("c4 full batch generated", sum(g.nnz for g in gs))
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=0)
    res = vc.mincut_batch(dev, **kw)
    for i in range(0, 4096, 97):
        one = vc.mincut(*dev[i], **kw)
        assert got(gs[i], *res[i]) == got(gs[i], *one), (i, gs[i].n)
        if i % 1067 == 0:
            assert got(gs[i], *res[i]) == expect(gs[i], kw), i
    del dev, res
    torch.cuda.synchronize()


# ------------------------------------------------------------ sessions
def test_session_staggered_arrivals(mixed):
    """Requests submitted while others are in flight join at the next step;
    every result equals the oracle's for that graph alone."""
    gs, dev = mixed
    kw = dict(lp_iters=2, n0=32, seed=4)
    sess = vc.Session(8 << 30, **kw)
    order = list(range(len(gs)))
    rng = np.random.default_rng(0)
    rng.shuffle(order)
    results = {}
    pending = list(order)
    steps = 0
    while pending or len(results) < len(gs):
        for _ in range(int(rng.integers(0, 4))):  # 0-3 arrivals per step
            if pending:
                i = pending.pop()
                sess.submit(i, *dev[i])
        n = sess.step()
        steps += 1
        for rid, cut, side, info in sess.poll():
            results[rid] = (cut, side, info)
        assert steps < 10000
        if not pending and n == 0:
            break
    assert len(results) == len(gs)
    for i, g in enumerate(gs):
        assert got(g, *results[i]) == expect(g, kw), i
        assert results[i][2]["t_ms"][5] >= 0
    sess.close()


def test_session_budget_admission():
    """A tight budget queues requests until memory frees up; a request that
    can never fit is refused."""
    gs = [gg.c1_planted(s) for s in range(6)]
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=0)
    one = vc.batch_workspace_bytes([dev[0]], vc.params(**kw))
    sess = vc.Session(int(one * 3), **kw)  # capacity derived from the budget: about two graphs at a time
    for i, d in enumerate(dev):
        sess.submit(i, *d)
    results = {}
    for _ in range(1000):
        n = sess.step()
        for rid, cut, side, info in sess.poll():
            results[rid] = (cut, side, info)
        if n == 0:
            break
    assert len(results) == len(gs)
    for i, g in enumerate(gs):
        assert got(g, *results[i]) == expect(g, kw), i
    waits = sorted(r[2]["t_ms"][6] for r in results.values())
    assert waits[-1] > 10 * max(waits[0], 0.01), waits  # later requests queued for memory
    huge = to_dev(gg.rhg(1 << 16, 32.0, 5.0, 1))
    with pytest.raises(vc.ViecutError) as e:
        sess.submit(99, *huge)
    assert e.value.code == vc.EBUDGET
    sess.close()


def _serve_all(sess, dev, order, arrivals_per_step=None, rng=None):
    results = {}
    pending = list(order)
    steps = 0
    while True:
        k = len(pending) if arrivals_per_step is None else int(rng.integers(0, arrivals_per_step + 1))
        for _ in range(k):
            if pending:
                i = pending.pop(0)
                sess.submit(i, *dev[i])
        n = sess.step()
        steps += 1
        for rid, cut, side, info in sess.poll():
            results[rid] = (cut, side, info)
        assert steps < 20000
        if not pending and n == 0:
            break
    return results


def test_session_waves_reuse_slots():
    """Regression: requests admitted in waves, most of which leave the loop
    by collapsing (their rows stay in the union until the next relabelling),
    so later requests reuse slots of finished ones. Every result equals the
    oracle's for that graph alone."""
    gs = [gg.planted(int(n), float(d), 8, 1, 100, 900 + s)
          for s, (n, d) in enumerate([(24000, 16), (30000, 20), (20000, 24), (36000, 16), (28000, 20),
                                      (22000, 18), (32000, 16), (26000, 22), (34000, 18), (21000, 20)])]
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=0)
    one = max(vc.batch_workspace_bytes([d], vc.params(**kw)) for d in dev)
    sess = vc.Session(int(one * 2.6), **kw)  # one lane, two or three requests at a time
    results = _serve_all(sess, dev, list(range(len(gs))))
    sess.close()
    statuses = set()
    for i, g in enumerate(gs):
        want = expect(g, kw)
        statuses.add(want[5])
        assert got(g, *results[i]) == want, (i, g.n)
    assert oracle.ST_COLLAPSED in statuses  # the case that leaves rows behind is exercised


def test_session_two_lanes():
    """Small and large requests (more than 2^20 arcs) in one session: the
    large lane runs on its own stream and thread, admits in waves, and every
    result equals the oracle's for that graph alone."""
    large = [gg.planted(int(n), 32.0, 10, 1, 100, 950 + s) for s, n in enumerate([40000, 36000, 44000, 38000])]
    assert all(g.nnz > (1 << 20) for g in large)
    small = [gg.c1_planted(s) for s in range(4)] + [gg.rhg(6000, 24.0, 5.0, 9, wlo=1, whi=100)] + \
        [load_golden(name)[0] for name in GOLDEN]
    gs = large + small
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=1)
    one = max(vc.batch_workspace_bytes([d], vc.params(**kw)) for d in dev[:len(large)])
    sess = vc.Session(int(max(one * 2.5 / 0.75, 600 << 20)), **kw)
    rng = np.random.default_rng(3)
    order = list(range(len(gs)))
    rng.shuffle(order)
    results = _serve_all(sess, dev, order, arrivals_per_step=2, rng=rng)
    sess.close()
    for i, g in enumerate(gs):
        assert got(g, *results[i]) == expect(g, kw), (i, g.n)
