"""Branch streams dominated by a few hot sites (run with -m gpu): segments
of 65536 executions and more are counted in pieces that add into a per-site
table; shorter long segments, more hot segments than tables, and histories
too long for a table, take the hash-table kernel.  Every case against the
oracle."""
import numpy as np
import pytest

import oracle
from oracle.compare import compare
from helpers import branch_trace

pytestmark = pytest.mark.gpu

ZERO, PATTERN = 2, 8


def check(tr):
    from gpu_util import run
    got = run(tr)[0]
    bad = compare(got, oracle.characterize(tr))
    assert not bad, "\n".join(bad[:20])
    return got


def outcomes(rng, s, n_sites):
    # per site: fair, biased, or a periodic pattern with noise
    kind = rng.integers(0, 3, size=n_sites)
    p = rng.random(n_sites)
    y = np.empty(s.size, dtype=np.uint8)
    for k in range(n_sites):
        idx = np.nonzero(s == k)[0]
        if kind[k] == 0:
            y[idx] = rng.random(idx.size) < 0.5
        elif kind[k] == 1:
            y[idx] = rng.random(idx.size) < 0.02 + 0.96 * p[k]
        else:
            period = int(rng.integers(2, 40))
            y[idx] = ((np.arange(idx.size) % period) == 0) ^ (rng.random(idx.size) < 0.01)
    return y


@pytest.mark.parametrize("flags,m", [(0, 16), (0, 8), (0, 1), (ZERO, 16), (PATTERN, 16),
                                     (ZERO | PATTERN, 12)])
def test_three_hot_sites(flags, m):
    rng = np.random.default_rng(500 + 10 * flags + m)
    n = 600000
    s = rng.choice(3, size=n, p=[0.6, 0.3, 0.1]).astype(np.uint32)
    t = branch_trace(s, outcomes(rng, s, 3), 3, m)
    t.branch_flags = flags
    print("flags", flags, "m", m, flush=True)
    check(t)


def test_hot_sites_beside_small_ones():
    # hot segments after runs of small ones: a work block's leading segments
    # are counted apart from its last, hot, segment
    rng = np.random.default_rng(77)
    n = 800000
    s = np.where(rng.random(n) < 0.5, rng.integers(0, 4000, size=n), 4000 + rng.integers(0, 4, size=n))
    s = s.astype(np.uint32)
    check(branch_trace(s, outcomes(rng, s, 4004), 4004, 16))


def test_more_hot_segments_than_tables():
    # 80 sites of 70000 executions each: 64 get tables, the rest go to the
    # hash-table kernel
    rng = np.random.default_rng(78)
    s = np.repeat(np.arange(80, dtype=np.uint32), 70000)
    rng.shuffle(s)
    check(branch_trace(s, outcomes(rng, s, 80), 80, 16))


def test_hot_sites_with_long_histories():
    # m > 16: no table; the hash-table kernel takes the hot segments
    rng = np.random.default_rng(79)
    s = rng.integers(0, 2, size=120000).astype(np.uint32)
    check(branch_trace(s, outcomes(rng, s, 2), 2, 20))
