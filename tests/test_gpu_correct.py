"""GPU parity of the correcting step (flag VIECUT_F_CORRECT, Section 4.1's
correcting algorithm): the library against the oracle with the step on,
bit-exact on the result and - on the traced cases - on every intermediate
state, including the corrected labels of every round."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import load_golden, random_graph
from test_gpu_parity import GOLDEN, compare, hub_graph

pytestmark = pytest.mark.gpu


def corrections(info):
    """Rounds whose correcting step changed a label (kind 6 events)."""
    fixes = 0
    last = None
    for ev in info.get("events", []):
        if ev["kind"] == 1:
            last = ev["labels"]
        elif ev["kind"] == 6 and last is not None and (ev["labels"] != last).any():
            fixes += 1
    return fixes


@pytest.mark.parametrize("name", GOLDEN)
@pytest.mark.parametrize("lp", [1, 2])
def test_golden_with_correction(name, lp):
    g, _ = load_golden(name)
    compare(g, name, trace=True, lp_iters=lp, n0=1, seed=lp, correct=True)


@pytest.mark.parametrize("seed", range(40))
def test_random_small_with_correction(seed):
    rng = np.random.default_rng(8800 + seed)
    n = int(rng.integers(4, 120))
    g = random_graph(n, float(rng.uniform(0.03, 0.5)), int(rng.choice([1, 2, 7, 100])), 8800 + seed,
                     connected=bool(seed % 5))
    compare(g, "random-fix%d" % seed, trace=True, lp_iters=int(rng.integers(1, 4)), n0=int(rng.integers(1, 6)),
            seed=seed, correct=True)


def test_some_cases_do_correct():
    """The random cases above include rounds where the step removes a
    vertex (checked on the oracle's trace, so the parity runs cover it)."""
    hit = 0
    for seed in range(40):
        rng = np.random.default_rng(8800 + seed)
        n = int(rng.integers(4, 120))
        g = random_graph(n, float(rng.uniform(0.03, 0.5)), int(rng.choice([1, 2, 7, 100])), 8800 + seed,
                         connected=bool(seed % 5))
        r = oracle.mincut_graph(g, lp_iters=int(rng.integers(1, 4)), n0=int(rng.integers(1, 6)), seed=seed,
                                correct=True, trace=True)
        hit += corrections({"events": r.events}) > 0
    assert hit >= 3


@pytest.mark.parametrize("seed", range(8))
def test_planted_with_correction(seed):
    g = gg.c1_planted(seed)
    compare(g, "c1-fix-%d" % seed, trace=(seed < 2), lp_iters=2, n0=64, seed=0, correct=True)


@pytest.mark.parametrize("hub_deg", [700, 9000])
def test_degree_classes_with_correction(hub_deg):
    g = hub_graph(hub_deg, hub_deg)
    compare(g, "hub-fix%d" % hub_deg, trace=True, lp_iters=2, n0=16, seed=3, correct=True)


def test_rhg_with_correction():
    g = gg.rhg(1 << 14, 32.0, 5.0, 4, wlo=1, whi=50)
    compare(g, "rhg14-fix", trace=True, lp_iters=2, n0=64, correct=True)


def test_full_size_rhg_with_correction():
    g = gg.c2_rhg()
    compare(g, "c2-fix", trace=False, lp_iters=2, n0=10000, seed=0, correct=True)
    compare(g, "c2-fix-n0-64", trace=False, lp_iters=2, n0=64, seed=0, correct=True)


def test_batch_refuses_the_correcting_step():
    import ctypes

    import torch

    import paper_1708_06127_amd as vc
    from gpu_common import to_dev
    g = gg.c1_planted(0)
    dev = to_dev(g)
    cs = (vc.Csr * 1)(vc.csr(*dev))
    p = vc.params(n0=64, correct=True)
    outs = (vc.Result * 1)()
    side = torch.empty((g.n + 63) // 64, dtype=torch.int64, device="cuda")
    sides = (ctypes.c_void_p * 1)(side.data_ptr())
    assert vc.load().viecut_mincut_batch(cs, 1, ctypes.byref(p), None, 0, None, outs, sides) == vc.EINVAL
