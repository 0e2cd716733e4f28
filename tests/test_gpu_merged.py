"""The aggregate over invocations on the GPU (aiwc_characterize_merged)
against the oracle's concatenation of the same host invocations, element by
element (run with -m gpu)."""
import json

import numpy as np
import pytest

import oracle
from oracle.compare import compare
from helpers import mk, random_trace

pytestmark = pytest.mark.gpu


def on_device(trs):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    keep, hs = [], []
    for tr in trs:
        dev = aiwc.host_to_device(tr, 0)
        keep.append(dev)
        hs.append(aiwc.device_trace(c, dev, tr.table, int(tr.n_sites), int(tr.history_len),
                                    branch_flags=int(getattr(tr, "branch_flags", 0))))
    return c, keep, hs


def check(trs):
    c, keep, hs = on_device(trs)
    m = c.characterize_merged(hs)
    got = m.read()
    mt = oracle.MergedTrace(trs)
    bad = compare(got, oracle.characterize(mt))
    assert not bad, "\n".join(bad[:20])
    for s in (0, 1):
        assert m.spectrum(s) == oracle.spectrum(mt, s, 0), f"spectrum space {s}"
    ncls = int(np.asarray(mt.table)["op_class"].max()) + 1
    assert np.array_equal(m.class_hist(ncls), oracle.class_hist(mt, ncls))
    return got


@pytest.mark.parametrize("seed", range(12))
def test_random_invocation_sets(seed):
    rng = np.random.default_rng(5000 + seed)
    k = int(rng.integers(2, 8))
    m = int(rng.integers(1, 33))
    bits = int(rng.integers(2, 30))
    trs = [random_trace(rng, int(rng.integers(1, 30)), int(rng.integers(0, 2500)),
                        int(rng.integers(1, 400)), m, addr_bits=bits, p_local=float(rng.random()))
           for _ in range(k)]
    print("seed", seed, "invocations", k, [t.opcode.size for t in trs], flush=True)
    check(trs)


def test_one_invocation_equals_the_plain_path():
    from gpu_util import run
    t = random_trace(np.random.default_rng(9), 20, 2000, 50, 8)
    c, keep, hs = on_device([t])
    a = c.characterize_merged(hs).read()
    b = run(t)[0]
    assert json.dumps(a, sort_keys=True) == json.dumps(b, sort_keys=True)


def test_empty_invocations_anywhere():
    rng = np.random.default_rng(17)
    m = 6
    e = mk(np.zeros(0, dtype=np.uint16), [], m=m)
    e2 = mk(np.zeros(0, dtype=np.uint16), [0, 0], m=m)
    a = random_trace(rng, 10, 1500, 30, m)
    b = random_trace(rng, 7, 900, 12, m)
    check([e, a, e2, b, e])
    check([e, e2])


def test_streams_without_memory_or_branches():
    rng = np.random.default_rng(23)
    a = mk(np.zeros(500, dtype=np.uint16), [200, 300], m=4)
    b = random_trace(rng, 5, 800, 9, 4)
    check([a, b, a])


def test_mismatched_invocations_are_rejected():
    import paper_1805_04207_amd as aiwc
    rng = np.random.default_rng(31)
    a = random_trace(rng, 3, 100, 4, 5)
    b = random_trace(rng, 3, 100, 4, 6)
    c, keep, hs = on_device([a, b])
    with pytest.raises(aiwc.AiwcError):
        c.characterize_merged(hs)
    with pytest.raises(aiwc.AiwcError):
        c.characterize_merged([])


def test_merged_with_a_branch_variant():
    rng = np.random.default_rng(41)
    trs = [random_trace(rng, int(rng.integers(1, 20)), 1500, 30, 6) for _ in range(3)]
    for t in trs:
        t.branch_flags = 4 | 8
    check(trs)
