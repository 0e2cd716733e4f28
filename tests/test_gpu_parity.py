"""HIP path vs the CPU oracle, element by element (run with -m gpu)."""
import os

import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle.compare import compare
from helpers import (BARRIER, BRANCH, COMPUTE, ID_ATOMIC, ID_BARRIER, ID_BRANCH, ID_LOAD,
                     ID_STORE, atomic_trace, branch_trace, mem_trace, mk, random_trace, table)

pytestmark = pytest.mark.gpu


def check(tr, **kw):
    from gpu_util import run
    got, m, t, dev = run(tr, **kw)
    want = oracle.characterize(tr)
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])
    for s in (0, 1):
        assert m.spectrum(s) == oracle.spectrum(tr, s, 0), f"spectrum space {s}"
    ncls = int(np.asarray(tr.table)["op_class"].max()) + 1
    assert np.array_equal(m.class_hist(ncls), oracle.class_hist(tr, ncls))
    return got


def test_config1_full():
    h = tg.generate_host(tg.config1())
    print("config1", h.opcode.size, h.addr.size, h.br_site.size, flush=True)
    got = check(h)
    assert got["total_instructions"] == h.opcode.size


@pytest.mark.parametrize("seed", range(24))
def test_random_small_traces(seed):
    rng = np.random.default_rng(1000 + seed)
    n_wi = int(rng.integers(1, 40))
    tr = random_trace(rng, n_wi, int(rng.integers(0, 3000)), int(rng.integers(1, 600)),
                      int(rng.integers(1, 33)), addr_bits=int(rng.integers(2, 30)),
                      p_local=float(rng.random()))
    print("seed", seed, tr.opcode.size, tr.addr.size, tr.br_site.size, flush=True)
    check(tr)


def test_empty_and_degenerate():
    # no events at all, three empty work-items
    check(mk([], [0, 0, 0]))
    # compute only, no memory and no branches
    check(mk(np.zeros(1000, dtype=np.uint16), [400, 0, 600]))
    # one address accessed 3000 times: counts >= 256 take the sparse spectrum path
    check(mem_trace([0xDEAD_BEE0] * 3000))
    # local-only stream, unaligned byte addresses
    rng = np.random.default_rng(7)
    a = rng.integers(0, 4096, size=20000, dtype=np.uint64)
    check(mem_trace(a, np.full(a.size, 2, dtype=np.uint8)))


def test_branch_edge_cases():
    rng = np.random.default_rng(3)
    # single site (no radix pass), history 1 and 32
    ys = (rng.random(5000) < 0.3).astype(np.uint8)
    check(branch_trace(np.zeros(5000), ys, 1, 1))
    check(branch_trace(np.zeros(5000), ys, 1, 32))
    # many sites: three radix passes (site ids up to 70000)
    s = rng.integers(0, 70000, size=40000).astype(np.uint32)
    check(branch_trace(s, (rng.random(40000) < 0.5).astype(np.uint8), 70000, 4))
    # one hot site with far more distinct histories than the on-chip table
    ys = (rng.random(60000) < 0.5).astype(np.uint8)
    check(branch_trace(np.zeros(60000), ys, 1, 20))


def test_long_segments():
    # ITB values above the LDS range (>= 4096) and above the dense range (>= 65536)
    L = 150_000
    op = np.zeros(L, dtype=np.uint16)
    op[5000] = ID_BARRIER
    op[15000] = ID_BARRIER
    check(mk(op, [70_000, 80_000]))



@pytest.mark.parametrize("n_bar", [0, 1, 2, 3, 5])
def test_barrier_ids(n_bar):
    """Work-item streams long enough for the vectorised chunks, with 0, 1, 2
    (barrier ids compared directly) and 3 or 5 (kinds looked up per event)
    opcode ids of barrier kind."""
    rng = np.random.default_rng(60 + n_bar)
    n_ids = 40
    bars = set(rng.choice(n_ids, size=n_bar, replace=False).tolist())
    tab = table([(i % 7, 1, BARRIER if i in bars else COMPUTE) for i in range(n_ids)])
    lens = rng.integers(0, 6000, size=64)
    op = rng.integers(0, n_ids, size=int(lens.sum())).astype(np.uint16)
    # barriers rare, as in kernels: most drawn barrier ids become other ids
    other = np.asarray([i for i in range(n_ids) if i not in bars], dtype=np.uint16)
    drop = np.isin(op, list(bars)) & (rng.random(op.size) < 0.98)
    op[drop] = rng.choice(other, size=int(drop.sum()))
    check(mk(op, list(lens), tab=tab))


def test_many_opcode_ids_global_path():
    # more than 8192 ids: histogram in global memory
    n = 10000
    tab = table([(i % 5000, 1 + i % 7, COMPUTE) for i in range(n)])
    rng = np.random.default_rng(5)
    op = rng.integers(0, n, size=50000).astype(np.uint16)
    check(mk(op, [25000, 25000], tab=tab))


def test_partition_overflow_redo(monkeypatch):
    # 16 partitions for ~150K distinct pages: every partition holds more pages
    # than one round of the on-chip page table and is split and redone;
    # results must stay exact
    monkeypatch.setenv("AIWC_FORCE_PARTITION_LOG2", "4")
    rng = np.random.default_rng(11)
    a = rng.integers(0, 1 << 28, size=200_000, dtype=np.uint64) * 4
    got = check(mem_trace(a, (rng.random(a.size) < 0.4).astype(np.uint8)))
    assert got["overflow_redos"] > 0


def test_config2_medium_device_generated():
    import torch
    from gpu_util import ctx
    import paper_1805_04207_amd as aiwc
    spec = tg.config2(n_wi=1 << 14)
    h = tg.generate_host(spec)
    d = tg.generate_device(spec, 0)
    for f in ("opcode", "wi_offsets", "addr", "mem_kind", "br_site", "br_taken"):
        a = getattr(h, f)
        b = d[f][:a.size].cpu().numpy().view(a.dtype)
        assert np.array_equal(a, b), f"device generator differs in {f}"
    t = aiwc.device_trace(ctx(), d, h.table, spec.n_sites, spec.history_len, spec.wg_size)
    got = ctx().characterize(t).read()
    bad = compare(got, oracle.characterize(h))
    assert not bad, "\n".join(bad[:20])


def test_atomic_traces():
    # an atomic read-modify-write: one instruction, a read and a write event
    rng = np.random.default_rng(11)
    a = rng.integers(0, 1 << 16, size=3000, dtype=np.uint64) * 4
    got = check(atomic_trace(a, rng.integers(0, 2, size=a.size)))
    assert got["space"][0]["total_reads"] == got["space"][0]["total_writes"]
    # the config1 recipe with a quarter of its memory instructions atomic,
    # generated on the device (identical bytes) and on the host
    import torch
    from gpu_util import ctx
    import paper_1805_04207_amd as aiwc
    spec = tg.config1()
    spec.p_atomic = 0.25
    h = tg.generate_host(spec)
    assert int((h.opcode == tg.ID_ATOMIC).sum()) > 1000
    d = tg.generate_device(spec, 0)
    for f in ("opcode", "wi_offsets", "addr", "mem_kind", "br_site", "br_taken"):
        x = getattr(h, f)
        y = d[f][:x.size].cpu().numpy().view(x.dtype)
        assert np.array_equal(x, y), f"device generator differs in {f}"
    check(h)


def test_atomic_with_one_memory_event_is_inconsistent():
    from gpu_util import run
    import paper_1805_04207_amd as aiwc
    tr = mk([ID_ATOMIC, 0], [2], [256], [0])
    assert not oracle.consistent(tr)
    with pytest.raises(aiwc.AiwcError) as e:
        run(tr)
    assert e.value.status == 2
    with pytest.raises(aiwc.AiwcError) as e:
        run(tr, validate=True)
    assert e.value.status == 2
    # with both of its events it is consistent, on both sides
    ok = mk([ID_ATOMIC, 0], [2], [256, 256], [0, 1])
    assert oracle.consistent(ok)
    check(ok)


def test_determinism_twice():
    from gpu_util import run
    h = tg.generate_host(tg.config2(n_wi=2048))
    a = run(h)[0]
    b = run(h)[0]
    assert a == b or repr(a) == repr(b)


def test_invalid_content_is_reported():
    from gpu_util import run
    import paper_1805_04207_amd as aiwc
    tr = branch_trace([0, 1, 5], [0, 1, 0], 2, 2)     # site 5 >= n_sites
    with pytest.raises(aiwc.AiwcError) as e:
        run(tr, validate=True)
    assert e.value.status == 1
    with pytest.raises(aiwc.AiwcError) as e:
        run(tr)
    assert e.value.status == 1
    # a load opcode without a memory event: inconsistent
    tr = mk([ID_LOAD, 0], [2])
    with pytest.raises(aiwc.AiwcError) as e:
        run(tr)
    assert e.value.status == 2
