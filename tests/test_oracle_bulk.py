"""The vectorised oracle (oracle/bulk.py) against the C oracle, field by
field, on small traces: it restates the same definitions for traces too large
for the C oracle, so it must agree with it exactly (same bar as the GPU)."""
import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle import bulk
from oracle.compare import compare
from helpers import BARRIER, branch_trace, mem_trace, mk, random_trace, table


def agree(tr):
    want = oracle.characterize(tr)
    got = bulk.characterize(tr, threads=4)
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])
    ncls = len(got["_class_hist"])
    assert np.array_equal(got["_class_hist"], oracle.class_hist(tr, ncls)[:ncls])
    return got


@pytest.mark.parametrize("seed", range(12))
def test_random_traces(seed):
    rng = np.random.default_rng(500 + seed)
    agree(random_trace(rng, int(rng.integers(1, 50)), int(rng.integers(0, 4000)),
                       int(rng.integers(1, 300)), int(rng.integers(1, 33))))


def test_config2_small():
    agree(tg.generate_host(tg.config2(n_wi=1 << 11)))


def test_config1():
    agree(tg.generate_host(tg.config1()))


def test_empty_and_single():
    agree(mk(np.zeros(0, dtype=np.uint16), [0]))
    agree(mk(np.zeros(0, dtype=np.uint16), [0, 0, 0]))
    agree(mem_trace(np.array([4096], dtype=np.uint64), np.array([1], dtype=np.uint8)))
    agree(branch_trace(np.zeros(3), np.array([1, 0, 1], dtype=np.uint8), 1, 4))


def test_barrier_layouts():
    # barriers at work-item starts / ends, several in a row, none at all
    tab = table([(0, 1, 0), (1, 1, BARRIER)])
    op = np.array([1, 0, 0, 1, 1, 0, 1, 0, 0, 0, 1], dtype=np.uint16)
    agree(mk(op, [1, 3, 0, 4, 3], tab=tab))
    agree(mk(np.zeros(9, dtype=np.uint16), [2, 3, 4], tab=tab))


def test_long_histories_and_many_sites():
    rng = np.random.default_rng(77)
    s = rng.integers(0, 3000, size=30000).astype(np.uint32)
    agree(branch_trace(s, (rng.random(30000) < 0.3).astype(np.uint8), 3000, 32))


@pytest.mark.parametrize("flags", [2, 4, 6, 8, 10, 12, 14])
def test_branch_variants(flags):
    # zero-initialised / global histories and the pattern entropy
    rng = np.random.default_rng(900 + flags)
    for m in (1, 7, 16):
        s = rng.integers(0, 40, size=5000).astype(np.uint32)
        t = branch_trace(s, (rng.random(5000) < 0.4).astype(np.uint8), 40, m)
        t.branch_flags = flags
        agree(t)
