"""GPU checks of viecut_mincut_noalloc (the allocation-free single solve on the
static device scratch) through the C ABI: each call's result (cut, side
bitmap, loop statistics) equals viecut_mincut's on the same graph, on two
calls in a row with the second input smaller than the first, so that what the
first call left in the scratch cannot leak into the second. The oracle is
checked beside them."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1708_06127_amd as vc
from gpu_common import log, side_words, to_dev
from helpers import random_graph

pytestmark = pytest.mark.gpu


def solve_both(g, **kw):
    import torch
    lib = vc.load()
    rp, col, w = to_dev(g)
    c = vc.csr(rp, col, w)
    p = vc.params(**kw)
    words = max((g.n + 63) // 64, 1)
    sp = vc._stream_ptr(None)
    side_a = torch.full((words,), -1, dtype=torch.int64, device="cuda")
    side_b = torch.full((words,), -1, dtype=torch.int64, device="cuda")
    ra, rb = vc.Result(), vc.Result()
    assert vc.workspace_bytes(g.n, g.nnz) <= vc.NOALLOC_SCRATCH_BYTES
    rc = lib.viecut_mincut_noalloc(ctypes.byref(c), ctypes.byref(p), sp, ctypes.byref(ra), side_a.data_ptr())
    assert rc == vc.OK, vc.strerror(rc)
    rc = lib.viecut_mincut(ctypes.byref(c), ctypes.byref(p), None, 0, sp, ctypes.byref(rb), side_b.data_ptr())
    assert rc == vc.OK, vc.strerror(rc)
    torch.cuda.synchronize()
    a = ra.as_dict()
    b = rb.as_dict()
    keys = ("cut", "rounds", "kernel_n", "witness_level", "status", "levels")
    assert tuple(a[k] for k in keys) == tuple(b[k] for k in keys), (a, b)
    sa, sb = side_words(side_a, g.n), side_words(side_b, g.n)
    assert np.array_equal(sa, sb)
    ref = oracle.mincut_graph(g, **{k: v for k, v in kw.items() if k != "validate"})
    assert (a["cut"], a["rounds"], a["kernel_n"], a["witness_level"], a["status"]) == \
        (ref.cut, ref.rounds, ref.kernel_n, ref.witness_level, ref.status)
    assert np.array_equal(sa, ref.side)
    return a


@pytest.mark.parametrize("first,second", [
    ("planted2000", "random300"),
    ("c4_largest", "planted100"),
])
def test_noalloc_equals_single_path_on_consecutive_calls(first, second):
    def make(name):
        if name == "planted2000":
            return gg.c1_planted(0), dict(lp_iters=2, n0=64, seed=0)
        if name == "random300":
            return random_graph(300, 0.05, 7, 91), dict(lp_iters=2, n0=8, seed=3)
        if name == "planted100":
            return gg.planted(100, 12.0, 3, 1, 100, 17), dict(lp_iters=2, n0=16, seed=1)
        if name == "c4_largest":  # the largest shape of the planted batch: n = 8192, d = 64
            return gg.planted(8192, 64.0, 20, 1, 100, 5), dict(lp_iters=2, n0=64, seed=0)
        raise KeyError(name)
    g1, kw1 = make(first)
    g2, kw2 = make(second)
    assert g2.nnz < g1.nnz and g2.n < g1.n
    log("noalloc", first, "n=%d nnz=%d" % (g1.n, g1.nnz), "then", second, "n=%d nnz=%d" % (g2.n, g2.nnz))
    solve_both(g1, **kw1)
    solve_both(g2, **kw2)


def test_noalloc_refuses_a_graph_beyond_the_scratch():
    import torch
    g = gg.planted(40000, 64.0, 5, 1, 1, 2)
    assert vc.workspace_bytes(g.n, g.nnz) > vc.NOALLOC_SCRATCH_BYTES
    rp, col, w = to_dev(g)
    side = torch.zeros((g.n + 63) // 64, dtype=torch.int64, device="cuda")
    with pytest.raises(vc.ViecutError) as e:
        vc.mincut_noalloc(rp, col, w, side=side, n0=64)
    assert e.value.code == vc.ETOOBIG
    assert int(side.abs().sum()) == 0  # nothing written on error
    # the entry point still works afterwards
    solve_both(gg.c1_planted(1), lp_iters=2, n0=64, seed=0)
