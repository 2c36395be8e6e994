"""Every launch-shape schedule gives the same results: the batched and single
paths under the extreme settings of the tuning table (every choice away from
its default) against the oracle."""
import pytest

import graphgen as gg
import paper_1708_06127_amd as vc
from gpu_common import log, to_dev
from test_gpu_batch import expect, got, mixed_graphs
from test_gpu_parity import compare, hub_graph

pytestmark = pytest.mark.gpu

EXTREMES = [
    {"radix_large_from": 0, "compact_direct_max": 0, "pr_merge_tiles": 0, "long_split": 256, "emit_wave": 0,
     "lp_group": 1, "emit_group": 1, "first_group": 2, "huge_part": 0},
    {"radix_large_from": 1 << 40, "compact_direct_max": 1 << 40, "pr_merge_tiles": 1 << 40, "long_split": 768,
     "emit_wave": 1, "lp_group": 3, "emit_group": 2, "first_group": 1},
    {"lp_group": 4},
]


@pytest.fixture
def schedule(request):
    saved = vc.tuning_get()
    vc.tuning_clear()
    for k, v in request.param.items():
        vc.tuning_set(-1, k, v)
    log("schedule", vc.tuning_get().splitlines()[-1])
    yield request.param
    vc.tuning_load_text(saved)


@pytest.mark.parametrize("schedule", EXTREMES, indirect=True)
def test_batch_under_schedule(schedule):
    gs = mixed_graphs()
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=16, seed=2)
    res = vc.mincut_batch(dev, **kw)
    for i, (g, r) in enumerate(zip(gs, res)):
        assert got(g, *r) == expect(g, kw), i


@pytest.mark.parametrize("schedule", EXTREMES, indirect=True)
def test_single_under_schedule(schedule):
    for hub in (700, 9000):
        compare(hub_graph(hub, hub), "hub%d" % hub, trace=True, lp_iters=2, n0=16, seed=hub)
    compare(gg.rmat_core(15, 16, seed=2, kcore=10), "rmat15", trace=True, lp_iters=2, n0=64)
    compare(gg.rhg(1 << 14, 32.0, 5.0, 1), "rhg14", trace=True, lp_iters=2, n0=64)
