"""Memory streams whose accesses pile onto a few pages (run with -m gpu):
partitions of 2^18 records and more count their candidate pages in
parallel into per-page tables and reduce the rest as usual.  Every case
against the oracle: a produced tiled matrix product (two hot local-memory
tiles), hot global and local pages beside ordinary traffic, more hot
partitions than slots, hot partitions without a candidate page, and
candidate pages with reads and writes."""
import os

import numpy as np
import pytest

import oracle
from oracle.compare import compare
from helpers import mem_trace

pytestmark = pytest.mark.gpu


def check(tr):
    from gpu_util import run
    got = run(tr)[0]
    bad = compare(got, oracle.characterize(tr))
    assert not bad, "\n".join(bad[:20])
    return got


def hot_stream(rng, n, hot_pages, share, local=False):
    """n accesses: a share of them on the given pages (random offsets, 70%
    reads), the rest uniform over 2^26 bytes."""
    k = int(n * share)
    pages = rng.choice(np.asarray(hot_pages, dtype=np.uint64), size=k)
    a_hot = pages * np.uint64(1024) + rng.integers(0, 1024, size=k, dtype=np.uint64)
    a_rest = rng.integers(0, 1 << 26, size=n - k, dtype=np.uint64)
    a = np.concatenate([a_hot, a_rest])
    w = (rng.random(n) < 0.3).astype(np.uint8)
    sp = np.concatenate([np.full(k, 2 if local else 0, np.uint8),
                         ((rng.random(n - k) < 0.1) * 2).astype(np.uint8)])
    order = rng.permutation(n)
    return a[order], (w | sp)[order]


def test_hot_global_pages():
    rng = np.random.default_rng(11)
    a, k = hot_stream(rng, 1500000, [7, 123456, 999], 0.8)
    check(mem_trace(a, k))


def test_hot_local_pages():
    rng = np.random.default_rng(12)
    a, k = hot_stream(rng, 1200000, [0, 1], 0.9, local=True)
    check(mem_trace(a, k))


def test_more_hot_partitions_than_slots():
    rng = np.random.default_rng(13)
    a, k = hot_stream(rng, 6000000, list(range(5000, 5000 + 4096 * 20, 4096)), 0.95)
    check(mem_trace(a, k))


def test_hot_partition_without_candidates(monkeypatch):
    # 16 partitions of ~375K records, each spread over ~19 pages of ~20000
    # records: no page reaches the candidate share of the sample
    monkeypatch.setenv("AIWC_FORCE_PARTITION_LOG2", "4")
    rng = np.random.default_rng(14)
    a, k = hot_stream(rng, 6000000, list(range(300)), 1.0)
    check(mem_trace(a, k))


def test_produced_tiled_matmul():
    import torch
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    from tracegen import kernels as K
    c = ctx()
    L = K.matmul_tiled(64, seed=21)
    p = L.program
    prog = c.program(p.code, p.table, p.n_sites)
    args = []
    for x in L.args:
        if isinstance(x, K.Global):
            args.append((aiwc.aiwc.ARG_GLOBAL, torch.from_numpy(x.array.copy().view(np.uint8)).to("cuda:0")))
        elif isinstance(x, K.Local):
            args.append((aiwc.aiwc.ARG_LOCAL, x.nbytes))
        else:
            args.append((aiwc.aiwc.ARG_SCALAR, x.value))
    produced = prog.produce(L.global_size, L.local_size, args)
    assert produced.desc.n_mem >= 1 << 18
    got = c.characterize(produced.trace()).read()
    want = oracle.characterize(oracle.produce(p, L.global_size, L.local_size, L.fresh_args()))
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])


def test_hot_pages_through_batch_graph_and_stream():
    """The hot-page path in the other entry points: a batch with hot and
    ordinary traces (eager, and a captured graph replayed), a stream of the
    same chunks (one memory stage over the concatenation) and the same stream
    out of core (partition groups, where hot partitions are reduced by the
    ordinary bucket kernel): each equal to the plain path or to the oracle on
    the concatenation."""
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx, same
    from helpers import random_trace
    c = ctx()
    rng = np.random.default_rng(31)
    a0, k0 = hot_stream(rng, 1200000, [0, 1], 0.9, local=True)
    a2, k2 = hot_stream(rng, 700000, [77, 5000], 0.85)
    trs = [mem_trace(a0, k0), random_trace(rng, 64, 3000, 40, 16, addr_bits=20),
           mem_trace(a2, k2)]
    keep, hs = [], []
    for tr in trs:
        dev = aiwc.host_to_device(tr, 0)
        keep.append(dev)
        hs.append(aiwc.device_trace(c, dev, tr.table, int(tr.n_sites), int(tr.history_len)))
    plain = [c.characterize(h).read() for h in hs]
    print("batch, eager", flush=True)
    got = [m.read() for m in c.characterize_batch(hs)]
    for i in range(3):
        assert same(got[i], plain[i]), f"batch, trace {i}"
    print("batch, graph", flush=True)
    for rep in range(3):
        got = [m.read() for m in c.characterize_batch(hs, use_graph=True)]
        for i in range(3):
            assert same(got[i], plain[i]), f"graph replay {rep}, trace {i}"
    # the concatenation (one history length, the largest site count)
    want = oracle.characterize(oracle.MergedTrace(trs))
    for budget in (0, 12 * (sum(t.addr.size for t in trs) // 3)):
        print(f"stream, device budget {budget}", flush=True)
        st = c.stream()
        if budget:
            st.set_device_budget(budget)
        for h in hs:
            st.append(h)
        got = st.finish().read()
        if budget:
            assert st.stats()["groups"] >= 2
        bad = compare(got, want)
        assert not bad, "\n".join(bad[:20])
