"""The oracle on the clustered Erdos-Renyi family (the paper's appendix on
instances): small instances against brute force (exact with n0 >= n, the
sandwich lambda <= cut <= minimum degree with the contraction loop), and
the int32 weight limit that the family exceeds at the paper's sizes."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import brute_mincut, cut_value, side_from_words


@pytest.mark.parametrize("seed", range(12))
def test_small_clustered_er(seed):
    rng = np.random.default_rng(4400 + seed)
    n = int(rng.integers(8, 17))
    g = gg.clustered_er(n, float(rng.choice([30.0, 60.0, 100.0])), int(rng.integers(2, 5)), seed)
    if g.nnz == 0 or int(g.degrees().min()) == 0:
        pytest.skip("isolated vertex: covered by the disconnected pins")
    lam, _ = brute_mincut(g)
    exact = oracle.mincut_graph(g, lp_iters=2, n0=n, seed=seed)
    assert exact.cut == lam
    r = oracle.mincut_graph(g, lp_iters=2, n0=1, seed=seed)
    side = side_from_words(r.side, g.n)
    assert not side[0] and 0 < side.sum() < g.n and cut_value(g, side) == r.cut
    assert lam <= r.cut <= int(g.degrees().min())


def test_paper_sizes_exceed_int32_weights():
    """At n = 2,000 and 10 % density the intra-cluster weights (up to 100 n)
    push the total weight past INT32_MAX: the oracle refuses with the
    overflow code instead of computing with wrapped sums."""
    g = gg.clustered_er(2000, 10.0, 4, 1)
    assert int(g.w.astype(np.int64).sum()) // 2 > 2**31 - 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.mincut_graph(g, lp_iters=2, n0=64)
    assert e.value.code == -3
