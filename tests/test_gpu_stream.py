"""Streaming characterization (aiwc_stream_*) on the GPU: the finished
stream against the oracle on the concatenation of its chunks, element by
element, and against the merged path (run with -m gpu)."""
import numpy as np
import pytest

import oracle
from oracle.compare import compare
from helpers import mem_trace, mk, random_trace

pytestmark = pytest.mark.gpu


def stream_of(trs, hint=False, host=False):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    st = c.stream(sum(t.addr.size for t in trs), sum(t.br_site.size for t in trs),
                  host_retain=host) if hint else c.stream(host_retain=host)
    keep = []
    for tr in trs:
        dev = aiwc.host_to_device(tr, 0)
        keep.append(dev)
        h = aiwc.device_trace(c, dev, tr.table, int(tr.n_sites), int(tr.history_len),
                              branch_flags=int(getattr(tr, "branch_flags", 0)))
        keep.append(h)
        st.append(h)
    m = st.finish()
    return c, m, keep


def check(trs, hint=False, host=False):
    from gpu_util import same
    c, m, keep = stream_of(trs, hint, host)
    got = m.read()
    mt = oracle.MergedTrace(trs)
    bad = compare(got, oracle.characterize(mt))
    assert not bad, "\n".join(bad[:20])
    for s in (0, 1):
        assert m.spectrum(s) == oracle.spectrum(mt, s, 0), f"spectrum space {s}"
    ncls = int(np.asarray(mt.table)["op_class"].max()) + 1
    assert np.array_equal(m.class_hist(ncls), oracle.class_hist(mt, ncls))
    hs = [k for k in keep if hasattr(k, "h")]
    assert same(c.characterize_merged(hs).read(), got)
    return got


@pytest.mark.parametrize("seed", range(8))
def test_random_chunk_sets(seed):
    rng = np.random.default_rng(9000 + seed)
    k = int(rng.integers(1, 9))
    m = int(rng.integers(1, 33))
    trs = [random_trace(rng, int(rng.integers(1, 30)), int(rng.integers(0, 2500)),
                        int(rng.integers(1, 300)), m, addr_bits=int(rng.integers(2, 30)),
                        p_local=float(rng.random())) for _ in range(k)]
    print("seed", seed, "chunks", k, flush=True)
    check(trs)


def test_many_chunks_grow_the_buffers():
    # ~60 chunks of a few thousand memory events: the retained buffers move
    # several times
    rng = np.random.default_rng(77)
    trs = [random_trace(rng, 8, 2000, 50, 10, addr_bits=20) for _ in range(60)]
    print("memory events", sum(t.addr.size for t in trs), flush=True)
    check(trs)
    check(trs, hint=True)


def test_large_values_across_chunks():
    # work-items and barrier segments of >= 2^16 instructions go to the
    # large-value lists, which carry over from chunk to chunk
    from helpers import ID_BARRIER
    trs = []
    for L in (70000, 65536, 90000, 3, 131072):
        op = np.zeros(L, dtype=np.uint16)
        if L > 10:
            op[L // 2] = ID_BARRIER
        trs.append(mk(op, [L]))
    trs.append(mk(np.zeros(200000, dtype=np.uint16), [100000, 100000]))
    check(trs)


def test_empty_and_lopsided_chunks():
    rng = np.random.default_rng(5)
    m = 7
    e = mk(np.zeros(0, dtype=np.uint16), [], m=m)
    e2 = mk(np.zeros(0, dtype=np.uint16), [0, 0, 0], m=m)
    ops_only = mk(np.zeros(900, dtype=np.uint16), [300, 600], m=m)
    a = random_trace(rng, 12, 1800, 40, m)
    check([e, a, e2, ops_only, random_trace(rng, 3, 500, 5, m), e])
    check([e])


def test_branch_variants_through_a_stream():
    rng = np.random.default_rng(13)
    for flags in (2 | 8, 4 | 8, 4 | 2):
        trs = [random_trace(rng, 10, 2000, 60, 9) for _ in range(4)]
        for t in trs:
            t.branch_flags = flags
        print("flags", flags, flush=True)
        check(trs)


def test_stream_errors():
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    rng = np.random.default_rng(3)
    a, b = random_trace(rng, 2, 100, 4, 5), random_trace(rng, 2, 100, 4, 6)
    da, db = aiwc.host_to_device(a, 0), aiwc.host_to_device(b, 0)
    ha = aiwc.device_trace(c, da, a.table, 4, 5)
    hb = aiwc.device_trace(c, db, b.table, 4, 6)
    st = c.stream()
    with pytest.raises(aiwc.AiwcError):
        st.finish()                      # nothing appended
    st.append(ha)
    with pytest.raises(aiwc.AiwcError):
        st.append(hb)                    # another history length
    m = st.finish()
    m.read()
    with pytest.raises(aiwc.AiwcError):
        st.append(ha)                    # finished
    with pytest.raises(aiwc.AiwcError):
        st.finish()
    st.close()


def test_appends_interleaved_with_other_work():
    # the context's scratch arena serves other calls between the appends
    # (and the finish reuses it): the stream's state is its own
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx, run
    c = ctx()
    rng = np.random.default_rng(61)
    trs = [random_trace(rng, 10, 2000, 30, 8, addr_bits=18) for _ in range(3)]
    other = random_trace(rng, 20, 3000, 50, 8, addr_bits=24)
    st = c.stream()
    keep = []
    for t in trs:
        dev = aiwc.host_to_device(t, 0)
        h = aiwc.device_trace(c, dev, t.table, int(t.n_sites), 8)
        keep += [dev, h]
        st.append(h)
        got_other = run(other)[0]
        assert not compare(got_other, oracle.characterize(other))
    got = st.finish().read()
    bad = compare(got, oracle.characterize(oracle.MergedTrace(trs)))
    assert not bad, "\n".join(bad[:20])


@pytest.mark.parametrize("hint", [False, True])
def test_streams_retained_in_host_memory(hint):
    # the memory and branch streams kept in pinned host memory until finish
    rng = np.random.default_rng(83)
    trs = [random_trace(rng, 8, 2000, 40, 12, addr_bits=22) for _ in range(40)]
    trs[3] = mk(np.zeros(0, dtype=np.uint16), [], m=12)
    check(trs, hint=hint, host=True)


def _budget_stream(trs, budget, host):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    st = c.stream(host_retain=host)
    st.set_device_budget(budget)
    keep = []
    for tr in trs:
        dev = aiwc.host_to_device(tr, 0)
        h = aiwc.device_trace(c, dev, tr.table, int(tr.n_sites), int(tr.history_len))
        keep += [dev, h]
        st.append(h)
    m = st.finish()
    return st, m, keep


@pytest.mark.parametrize("host", [False, True])
def test_out_of_core_memory_stage(host):
    # the memory stream reduced one partition group at a time under a device
    # budget of a quarter of its records: identical to the oracle on the
    # concatenation, while the device holds at most a group's records
    rng = np.random.default_rng(4242 + int(host))
    trs = [random_trace(rng, 40, 3000, 400, 16, addr_bits=b, p_local=0.3)
           for b in (12, 20, 28, 34)]
    n_mem = sum(t.addr.size for t in trs)
    st, m, keep = _budget_stream(trs, 12 * (n_mem // 4), host)
    got = m.read()
    s = st.stats()
    print("groups", s["groups"], "device records", s["device_records"], "of", n_mem, flush=True)
    assert s["memory_events"] == n_mem
    assert s["groups"] >= 3 and s["device_records"] < n_mem
    mt = oracle.MergedTrace(trs)
    bad = compare(got, oracle.characterize(mt))
    assert not bad, "\n".join(bad[:20])
    for sp in (0, 1):
        assert m.spectrum(sp) == oracle.spectrum(mt, sp, 0), f"spectrum space {sp}"
    # and the same chunks in one pass give the identical result
    from gpu_util import same
    st1, m1, keep1 = _budget_stream(trs, 0, host)
    assert st1.stats()["groups"] == 1
    assert same(m1.read(), got, drop=("overflow_redos",))


def test_out_of_core_with_a_partition_above_the_budget():
    # one hot page (tens of thousands of accesses to 64 words) holds more
    # records than the budget: its partition is reduced alone, the rest in
    # groups, and the result is still exact
    rng = np.random.default_rng(77)
    hot = mem_trace(np.uint64(0x4000) + 4 * rng.integers(0, 64, size=40000).astype(np.uint64),
                    (rng.random(40000) < 0.5).astype(np.uint8))
    cold = random_trace(rng, 30, 2000, 50, 16, addr_bits=32, p_local=0.2)
    trs = [cold, hot, cold]
    n_mem = sum(t.addr.size for t in trs)
    st, m, keep = _budget_stream(trs, 12 * 2000, True)
    s = st.stats()
    assert s["largest_partition"] >= 40000 and s["device_records"] >= 40000
    assert s["groups"] >= 2 and s["memory_events"] == n_mem
    mt = oracle.MergedTrace(trs)
    bad = compare(m.read(), oracle.characterize(mt))
    assert not bad, "\n".join(bad[:20])
