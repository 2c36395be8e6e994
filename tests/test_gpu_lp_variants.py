"""GPU parity of the label-propagation variants (VIECUT_F_CONVERGE: the
convergence stop of appendix D's configuration study; VIECUT_F_RESTRICT:
Section 4.1's first-iteration restriction, read synchronously): the library
against the oracle with each variant on, bit-exact on the result and, on the
traced cases, on every intermediate state (so the number of LP iterations
each round ran is compared too)."""
import numpy as np
import pytest

import graphgen as gg
from helpers import load_golden, random_graph
from test_gpu_parity import GOLDEN, compare, hub_graph
from test_oracle_lp_variants import hub_graph as star_hub

pytestmark = pytest.mark.gpu

VARIANTS = [dict(converge=True), dict(restrict=True), dict(converge=True, restrict=True),
            dict(converge=True, correct=True)]


@pytest.mark.parametrize("name", GOLDEN)
@pytest.mark.parametrize("var", range(len(VARIANTS)))
def test_golden_variants(name, var):
    g, _ = load_golden(name)
    compare(g, name, trace=True, lp_iters=6, n0=1, seed=var, **VARIANTS[var])


@pytest.mark.parametrize("seed", range(32))
def test_random_small_variants(seed):
    rng = np.random.default_rng(9300 + seed)
    n = int(rng.integers(4, 150))
    g = random_graph(n, float(rng.uniform(0.03, 0.5)), int(rng.choice([1, 2, 7, 100])), 9300 + seed,
                     connected=bool(seed % 5))
    compare(g, "random-var%d" % seed, trace=True, lp_iters=int(rng.integers(1, 12)), n0=int(rng.integers(1, 6)),
            seed=seed, **VARIANTS[seed % len(VARIANTS)])


@pytest.mark.parametrize("leaves", [9996, 10000])
def test_convergence_threshold(leaves):
    """Both sides of the floor(n / 10000) threshold (the oracle's pin graph)."""
    g = star_hub(leaves)
    compare(g, "hub-conv%d" % leaves, trace=True, lp_iters=25, n0=1, seed=3, converge=True)


def test_oscillation_runs_all_iterations():
    k = 300
    e = [(2 * i, 2 * i + 1) for i in range(k)] + [(2 * i + 1, 2 * i + 2) for i in range(k - 1)]
    g = gg.from_edges(2 * k, e, [10] * k + [1] * (k - 1))
    compare(g, "pairs-conv", trace=True, lp_iters=9, n0=1, seed=1, converge=True)
    compare(g, "pairs-restrict", trace=True, lp_iters=3, n0=1, seed=1, restrict=True)


@pytest.mark.parametrize("hub_deg", [700, 9000])
def test_degree_classes_variants(hub_deg):
    g = hub_graph(hub_deg, hub_deg)
    compare(g, "hub-var%d" % hub_deg, trace=True, lp_iters=5, n0=16, seed=3, converge=True, restrict=True)


def test_rhg_variants():
    g = gg.rhg(1 << 14, 32.0, 5.0, 4, wlo=1, whi=50)
    compare(g, "rhg14-conv", trace=True, lp_iters=25, n0=64, converge=True)
    compare(g, "rhg14-restrict", trace=True, lp_iters=2, n0=64, restrict=True)


def test_full_size_rhg_variants():
    g = gg.c2_rhg()
    compare(g, "c2-conv", trace=False, lp_iters=8, n0=10000, seed=0, converge=True)
    compare(g, "c2-restrict", trace=False, lp_iters=2, n0=10000, seed=0, restrict=True)


@pytest.mark.parametrize("flag", ["converge", "restrict"])
def test_batch_and_session_refuse_the_variants(flag):
    import ctypes

    import torch

    import paper_1708_06127_amd as vc
    from gpu_common import to_dev
    g = gg.c1_planted(0)
    dev = to_dev(g)
    cs = (vc.Csr * 1)(vc.csr(*dev))
    p = vc.params(n0=64, **{flag: True})
    outs = (vc.Result * 1)()
    side = torch.empty((g.n + 63) // 64, dtype=torch.int64, device="cuda")
    sides = (ctypes.c_void_p * 1)(side.data_ptr())
    assert vc.load().viecut_mincut_batch(cs, 1, ctypes.byref(p), None, 0, None, outs, sides) == vc.EINVAL
    sess = ctypes.c_void_p()
    assert vc.load().viecut_session_create(1 << 30, ctypes.byref(p), None, ctypes.byref(sess)) == vc.EINVAL
