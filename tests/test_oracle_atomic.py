"""Pins of the atomic read-modify-write reading (CPU only).

The plugin interface of the paper's Implementation section reports the load
and the store of an atomic through their own callbacks.  Reading: an atomic
RMW is ONE instruction issuing TWO memory events at one address, a read and
then a write.  These checks would fail on the plausible mistakes: counting
an atomic as one memory event, as no instruction, or dropping one half from
the unique read / write counts.
"""
import math

import numpy as np

import oracle
import tracegen as tg
from helpers import ID_ATOMIC, ID_LOAD, ID_STORE, atomic_trace, mk, random_trace


def test_atomics_are_one_instruction_two_events():
    tr = atomic_trace([64, 128, 64 + 4096])
    assert tr.opcode.size == 3 and tr.addr.size == 6
    assert oracle.consistent(tr)
    r = oracle.characterize(tr)
    assert r["total_instructions"] == 3
    g = r["space"][0]
    assert (g["total_reads"], g["total_writes"], g["total_accesses"]) == (3, 3, 6)
    assert (g["unique_reads"], g["unique_writes"], g["footprint"]) == (3, 3, 3)
    assert g["unique_rw_ratio"] == 1.0 and g["reread_ratio"] == 1.0 and g["rewrite_ratio"] == 1.0
    # three addresses accessed twice each: log2(3) bits at skip 0
    assert abs(g["entropy"][0] - math.log2(3)) < 1e-15
    # 6 accesses, 90% of them need ceil(5.4 / 2) = 3 addresses
    assert g["footprint_90"] == 3


def test_atomic_memory_metrics_equal_load_store_pairs():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 1 << 14, size=500, dtype=np.uint64) * 4
    local = rng.integers(0, 2, size=a.size)
    at = atomic_trace(a, local)
    # the same memory stream issued by a load and a store instruction each
    op = np.tile(np.array([ID_LOAD, ID_STORE], dtype=np.uint16), a.size)
    ls = mk(op, [op.size], at.addr, at.mem_kind)
    assert oracle.consistent(at) and oracle.consistent(ls)
    ra, rl = oracle.characterize(at), oracle.characterize(ls)
    assert ra["space"] == rl["space"]
    assert rl["total_instructions"] - ra["total_instructions"] == a.size


def test_atomic_with_one_event_is_inconsistent():
    # an atomic instruction but only its read event
    tr = mk([ID_ATOMIC, 0], [2], [256], [0])
    assert not oracle.consistent(tr)
    # an atomic counted as a plain load would need one event: also caught
    tr2 = mk([ID_ATOMIC, ID_LOAD], [2], [256, 256, 512], [0, 1, 0])
    assert oracle.consistent(tr2)          # 2 + 1 = 3 events
    tr3 = mk([ID_ATOMIC, ID_LOAD], [2], [256, 256], [0, 1])
    assert not oracle.consistent(tr3)


def test_random_traces_with_atomics_are_consistent():
    rng = np.random.default_rng(3)
    seen = 0
    for _ in range(20):
        tr = random_trace(rng, int(rng.integers(1, 20)), 300, 7, 4)
        seen += int((tr.opcode == ID_ATOMIC).sum())
        assert oracle.consistent(tr)
        # each atomic's events: a read then a write of one address
        per = np.where(np.isin(tr.opcode, [ID_LOAD, ID_STORE]), 1,
                       np.where(tr.opcode == ID_ATOMIC, 2, 0))
        first = np.concatenate([[0], np.cumsum(per)[:-1]])
        for i in np.flatnonzero(tr.opcode == ID_ATOMIC):
            e = first[i]
            assert tr.addr[e] == tr.addr[e + 1]
            assert (tr.mem_kind[e] & 1, tr.mem_kind[e + 1] & 1) == (0, 1)
            assert (tr.mem_kind[e] & 2) == (tr.mem_kind[e + 1] & 2)
    assert seen > 100


def test_generated_atomics():
    spec = tg.config1()
    spec.p_atomic = 0.25
    h = tg.generate_host(spec)
    cnt = np.bincount(h.opcode, minlength=tg.N_OPCODE_IDS)
    assert cnt[tg.ID_ATOMIC] > 1000
    assert cnt[tg.ID_LOAD] + cnt[tg.ID_STORE] + 2 * cnt[tg.ID_ATOMIC] == h.addr.size
    assert oracle.consistent(h)
    # the atomic share of memory instructions is close to the requested one
    n_inst = cnt[tg.ID_LOAD] + cnt[tg.ID_STORE] + cnt[tg.ID_ATOMIC]
    assert abs(cnt[tg.ID_ATOMIC] / n_inst - 0.25) < 0.02
    # without atomics the bytes are those of the plain recipe
    plain = tg.generate_host(tg.config1())
    assert tg.config1().p_atomic == 0.0 and oracle.consistent(plain)
    assert int(np.bincount(plain.opcode, minlength=tg.N_OPCODE_IDS)[tg.ID_ATOMIC]) == 0
