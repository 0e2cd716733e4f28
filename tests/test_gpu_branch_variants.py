"""Branch-entropy variants on the GPU (zero-initialised histories, the
global history, the pattern entropy) against the oracle, element by
element, and their interplay with batches (run with -m gpu)."""
import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle.compare import compare
from helpers import branch_trace, random_trace

pytestmark = pytest.mark.gpu

ZERO, GLOBAL, PATTERN = 2, 4, 8
COMBOS = [ZERO, GLOBAL, PATTERN, ZERO | GLOBAL, ZERO | PATTERN, GLOBAL | PATTERN,
          ZERO | GLOBAL | PATTERN]


def check(tr):
    from gpu_util import run
    got = run(tr)[0]
    want = oracle.characterize(tr)
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])
    return got


@pytest.mark.parametrize("flags", COMBOS)
def test_random_traces_each_variant(flags):
    rng = np.random.default_rng(7000 + flags)
    for k in range(4):
        m = int(rng.integers(1, 21))
        t = random_trace(rng, int(rng.integers(1, 30)), int(rng.integers(0, 3000)),
                         int(rng.integers(1, 500)), m, addr_bits=12)
        t.branch_flags = flags
        print("flags", flags, "case", k, "m", m, t.br_site.size, flush=True)
        check(t)


@pytest.mark.parametrize("flags", COMBOS)
def test_branch_heavy_stream_each_variant(flags):
    # many sites, long streams: several windows work blocks, split passes,
    # sites crossing 64-lane chunks, both record widths through the sort
    rng = np.random.default_rng(8000 + flags)
    n = 300000
    s = (rng.zipf(1.3, size=n) % 5000).astype(np.uint32)
    y = (rng.random(n) < np.where(s % 3 == 0, 0.5, 0.05)).astype(np.uint8)
    m = 16
    t = branch_trace(s, y, 5000, m)
    t.branch_flags = flags
    print("flags", flags, flush=True)
    check(t)


@pytest.mark.parametrize("flags,m", [(ZERO, 32), (GLOBAL, 31), (GLOBAL | ZERO, 1),
                                     (PATTERN, 20), (GLOBAL | PATTERN, 20), (ZERO | PATTERN, 1)])
def test_history_length_limits(flags, m):
    rng = np.random.default_rng(m * 100 + flags)
    s = rng.integers(0, 40, size=40000).astype(np.uint32)
    t = branch_trace(s, (rng.random(40000) < 0.3).astype(np.uint8), 40, m)
    t.branch_flags = flags
    check(t)


def test_small_config_each_variant():
    h = tg.generate_host(tg.config2(n_wi=1 << 12))
    for flags in (ZERO | PATTERN, GLOBAL | PATTERN):
        h.branch_flags = flags
        print("config2 2^12 flags", flags, flush=True)
        check(h)


def test_unsupported_and_invalid_flags():
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    t = branch_trace([0, 1, 0], [1, 0, 1], 2, 32)
    dev = aiwc.host_to_device(t, 0)
    for flags, status in ((GLOBAL, 5), (PATTERN, 5), (16, 1)):
        with pytest.raises(aiwc.AiwcError) as e:
            aiwc.device_trace(c, dev, t.table, 2, 32, branch_flags=flags)
        assert e.value.status == status
    t = branch_trace([0, 1, 0], [1, 0, 1], 2, 21)
    dev = aiwc.host_to_device(t, 0)
    with pytest.raises(aiwc.AiwcError):
        aiwc.device_trace(c, dev, t.table, 2, 21, branch_flags=PATTERN)


def test_batch_mixing_variants():
    # one batched call over traces of every variant: each must equal its
    # plain result and the oracle
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx, same
    c = ctx()
    rng = np.random.default_rng(55)
    keep, hs, trs = [], [], []
    for flags in [0] + COMBOS:
        t = random_trace(rng, int(rng.integers(1, 25)), 2500, 200, 12)
        t.branch_flags = flags
        dev = aiwc.host_to_device(t, 0)
        keep.append(dev)
        trs.append(t)
        hs.append(aiwc.device_trace(c, dev, t.table, int(t.n_sites), 12, branch_flags=flags))
    for use_graph in (False, True):
        res = [m.read() for m in c.characterize_batch(hs, use_graph=use_graph)]
        for t, h, r in zip(trs, hs, res):
            bad = compare(r, oracle.characterize(t))
            assert not bad, f"flags {t.branch_flags}: " + "\n".join(bad[:10])
            p = c.characterize(h).read()
            assert same(p, r)
