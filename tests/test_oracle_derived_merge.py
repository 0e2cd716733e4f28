"""Pins for the oracle's derived parallelism metrics and for its aggregate
over several invocations (the concatenation of their streams).

Derived metrics (LU decomposition analysis of the paper): closed forms on
hand-built traces and the printed needle figure.  Aggregation: relations the
aggregate must satisfy whatever the implementation -- doubled invocations
keep every distribution metric, disjoint address sets obey the grouping
property of entropy, disjoint branch sites average Yokota by windows, a
site's history carries across invocations, pooled medians and extrema."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from helpers import (ID_BARRIER, ID_LOAD, BRANCH, COMPUTE, OPDT, branch_trace, mem_trace, mk,
                     random_trace, table)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def same(a, b):
    return json.dumps(a, sort_keys=True) == json.dumps(b, sort_keys=True)


# ------------------------------------------------------------ derived metrics
def test_needle_mean_itb_golden():
    # a dropped final segment (mean ITB over barriers only) or a ratio over
    # barriers_hit alone would give 10/275, not the printed 0.04
    g = json.load(open(os.path.join(GOLDEN, "needle_mean_itb.json")))
    B, nb, tail, W = (g["barrier_every"], g["barriers_per_workitem"], g["tail_instructions"],
                      g["work_items"])
    wi = [ID_BARRIER if (p % B) == 0 else 0 for p in range(1, B * nb + 1)] + [0] * tail
    r = oracle.characterize(mk(np.array(wi * W, dtype=np.uint16), [len(wi)] * W))
    assert r["barriers_per_instruction"] == g["barriers_per_instruction"]
    assert r["itb_min"] == r["itb_max"] == B


@pytest.mark.parametrize("W", [1, 3, 4, 1000])
def test_granularity_is_inverse_work_items(W):
    r = oracle.characterize(mk(np.zeros(2 * W, dtype=np.uint16), [2] * W))
    assert r["granularity"] == 1.0 / W
    assert r["load_imbalance"] == 0


def test_instructions_per_operand_is_inverse_mean_width():
    # widths 1, 1, 4 and 8: 4 instructions over 14 operands; a reciprocal of
    # the width sum alone would give 1/14
    tab = table([(0, 1, COMPUTE), (1, 4, COMPUTE), (2, 8, COMPUTE)])
    r = oracle.characterize(mk(np.array([0, 0, 1, 2], dtype=np.uint16), [4], tab=tab))
    assert r["instructions_per_operand"] == 4 / 14
    tab4 = table([(0, 4, COMPUTE)])
    r = oracle.characterize(mk(np.zeros(9, dtype=np.uint16), [9], tab=tab4))
    assert r["instructions_per_operand"] == 0.25


def test_barriers_per_instruction_counts_kernel_end():
    # two work-items: 5 instructions with one barrier, 3 without: ITB values
    # {b-segment, rest} + {3}; 3 segments over 8 instructions
    op = np.array([0, ID_BARRIER, 0, 0, 0, 0, 0, 0], dtype=np.uint16)
    r = oracle.characterize(mk(op, [5, 3]))
    assert r["barriers_per_instruction"] == 3 / 8
    assert r["barriers_per_instruction"] == (r["barriers_hit"] + r["work_items"]) / 8


def test_load_imbalance_is_ipt_spread():
    r = oracle.characterize(mk(np.zeros(10, dtype=np.uint16), [0, 3, 7, 0]))
    assert r["load_imbalance"] == 7
    r = oracle.characterize(mk(np.zeros(12, dtype=np.uint16), [2, 9, 1]))
    assert r["load_imbalance"] == 8


def test_derived_of_an_empty_trace_follow_ieee():
    r = oracle.characterize(mk(np.zeros(0, dtype=np.uint16), []))
    assert r["granularity"] == math.inf
    assert math.isnan(r["barriers_per_instruction"]) and math.isnan(r["instructions_per_operand"])
    assert r["load_imbalance"] == 0
    # work-items without instructions: one empty segment each
    r = oracle.characterize(mk(np.zeros(0, dtype=np.uint16), [0, 0]))
    assert r["granularity"] == 0.5 and r["barriers_per_instruction"] == math.inf


# ---------------------------------------------------------------- aggregation
def test_one_invocation_is_itself():
    t = random_trace(np.random.default_rng(5), 6, 80, 3, 4)
    assert same(oracle.characterize_merged([t]), oracle.characterize(t))


def test_split_at_any_points_reassembles():
    # the aggregate of pieces of one trace (work-items split at a boundary,
    # memory and branch streams anywhere) is that trace's metrics
    rng = np.random.default_rng(11)
    t = random_trace(rng, 12, 90, 4, 3)
    w = 5
    e = int(t.wi_offsets[w])
    cm, cb = t.addr.size // 3, (2 * t.br_site.size) // 3
    a = mk(t.opcode[:e], np.diff(t.wi_offsets[:w + 1]).tolist(), t.addr[:cm], t.mem_kind[:cm],
           t.br_site[:cb], t.br_taken[:cb], n_sites=t.n_sites, m=t.history_len)
    b = mk(t.opcode[e:], np.diff(t.wi_offsets[w:]).tolist(), t.addr[cm:], t.mem_kind[cm:],
           t.br_site[cb:], t.br_taken[cb:], n_sites=t.n_sites, m=t.history_len)
    assert same(oracle.characterize_merged([a, b]), oracle.characterize(t))


def test_doubled_invocation_keeps_distributions():
    # every address's count doubles: distinct counts, entropies, 90%
    # footprint and unique counts stay; totals double
    t = random_trace(np.random.default_rng(3), 8, 100, 3, 2, addr_bits=9)
    r1, r2 = oracle.characterize(t), oracle.characterize_merged([t, t])
    for f in ("total_instructions", "barriers_hit", "itb_count", "itb_sum", "work_items",
              "total_branches"):
        assert r2[f] == 2 * r1[f], f
    for f in ("unique_opcodes", "opcodes_90", "simd_max", "simd_mean", "itb_min", "itb_max",
              "itb_median", "ipt_min", "ipt_max", "ipt_median", "unique_branches",
              "branches_90", "barriers_per_instruction", "instructions_per_operand",
              "load_imbalance"):
        assert r2[f] == r1[f], f
    assert r2["granularity"] == 1.0 / (2 * r1["work_items"])
    for s in (0, 1):
        a, b = r1["space"][s], r2["space"][s]
        assert b["total_accesses"] == 2 * a["total_accesses"]
        for f in ("unique_reads", "unique_writes", "footprint", "footprint_90", "distinct"):
            assert b[f] == a[f], (s, f)
        for k in range(11):
            assert math.isclose(b["entropy"][k], a["entropy"][k], rel_tol=1e-13, abs_tol=1e-15)


def test_disjoint_addresses_obey_entropy_grouping():
    # H(A u B) = (N1 H1 + N2 H2) / N + h(N1 / N) for disjoint supports, at
    # every skip (the shift keeps the sets apart after dropping 10 bits)
    rng = np.random.default_rng(8)
    a = mem_trace(rng.integers(0, 1 << 12, size=700, dtype=np.uint64))
    b = mem_trace((rng.integers(0, 1 << 14, size=300, dtype=np.uint64) ** 2 % (1 << 14))
                  + np.uint64(1 << 40))
    ra, rb, r = (oracle.characterize(a), oracle.characterize(b),
                 oracle.characterize_merged([a, b]))
    n1, n2 = 700, 300
    n = n1 + n2
    mix = -(n1 / n) * math.log2(n1 / n) - (n2 / n) * math.log2(n2 / n)
    for k in range(11):
        assert r["space"][0]["distinct"][k] == ra["space"][0]["distinct"][k] + \
            rb["space"][0]["distinct"][k]
        want = (n1 * ra["space"][0]["entropy"][k] + n2 * rb["space"][0]["entropy"][k]) / n + mix
        assert math.isclose(r["space"][0]["entropy"][k], want, rel_tol=1e-12)


def test_shared_addresses_count_once():
    a = mem_trace([16, 32, 48, 48])
    b = mem_trace([48, 64])
    r = oracle.characterize_merged([a, b])
    s = r["space"][0]
    assert s["footprint"] == 4 and s["total_accesses"] == 6
    # counts 1, 1, 3, 1 of 6
    want = -(3 * (1 / 6) * math.log2(1 / 6) + (3 / 6) * math.log2(3 / 6))
    assert math.isclose(s["entropy"][0], want, rel_tol=1e-13)


def test_disjoint_sites_average_yokota_by_windows():
    rng = np.random.default_rng(21)
    m = 3
    sa = rng.integers(0, 4, size=400)
    ya = (rng.random(400) < 0.3).astype(np.uint8)
    sb = rng.integers(0, 5, size=250) + 4
    yb = (rng.random(250) < 0.6).astype(np.uint8)
    a = branch_trace(sa, ya, 9, m)
    b = branch_trace(sb, yb, 9, m)
    ra, rb, r = (oracle.characterize(a), oracle.characterize(b),
                 oracle.characterize_merged([a, b]))
    assert r["n_windows"] == ra["n_windows"] + rb["n_windows"]
    assert r["albe_min_sum"] == ra["albe_min_sum"] + rb["albe_min_sum"]
    assert r["unique_branches"] == ra["unique_branches"] + rb["unique_branches"]
    want = (ra["n_windows"] * ra["yokota_entropy"] + rb["n_windows"] * rb["yokota_entropy"]) / \
        r["n_windows"]
    assert math.isclose(r["yokota_entropy"], want, rel_tol=1e-12)


def test_history_carries_across_invocations():
    # a site's first m outcomes form no window: over the aggregate that is
    # the first m of the whole sequence, not of each invocation
    m = 4
    a = branch_trace([0] * 6 + [1] * 2, [1, 0] * 4, 2, m)
    b = branch_trace([0] * 3 + [1] * 5, [0, 1, 1, 0, 1, 0, 0, 1], 2, m)
    r = oracle.characterize_merged([a, b])
    assert r["n_windows"] == (9 - m) + (7 - m)
    per_invocation = max(0, 6 - m) + max(0, 2 - m) + max(0, 3 - m) + max(0, 5 - m)
    assert r["n_windows"] != per_invocation


def test_pooled_parallelism():
    # invocation A: work-items of 5 and 5; B: 9 and 9 -- each balanced, the
    # aggregate spread 4; ITB values {1, 2, 3} and {10, 20}: pooled median 3
    r = oracle.characterize_merged([mk(np.zeros(10, dtype=np.uint16), [5, 5]),
                                    mk(np.zeros(18, dtype=np.uint16), [9, 9])])
    assert (r["ipt_min"], r["ipt_max"], r["load_imbalance"], r["work_items"]) == (5, 9, 4, 4)
    a = mk(np.array([ID_BARRIER, 0, ID_BARRIER, 0, 0, 0], dtype=np.uint16), [6])
    b = mk(np.array([0] * 9 + [ID_BARRIER] + [0] * 20, dtype=np.uint16), [30])
    r = oracle.characterize_merged([a, b])
    assert r["itb_count"] == 5 and r["itb_median"] == 3.0
    assert (r["itb_min"], r["itb_max"]) == (1, 20)


def test_empty_invocations_change_nothing():
    t = random_trace(np.random.default_rng(2), 5, 60, 2, 2)
    e = mk(np.zeros(0, dtype=np.uint16), [], n_sites=1, m=t.history_len)
    assert same(oracle.characterize_merged([e, t, e]), oracle.characterize(t))


def test_site_space_is_the_largest():
    a = branch_trace([0, 1, 0, 1], [1, 0, 1, 1], 2, 1)
    b = branch_trace([5, 5, 5], [0, 0, 1], 6, 1)
    assert oracle.MergedTrace([a, b]).n_sites == 6
    r = oracle.characterize_merged([a, b])
    assert r["unique_branches"] == 3


def test_mismatched_invocations_are_rejected():
    a = branch_trace([0, 0], [1, 0], 1, 2)
    with pytest.raises(ValueError):
        oracle.MergedTrace([a, branch_trace([0, 0], [1, 0], 1, 3)])
    other = np.array(a.table).copy()
    other[0]["simd_width"] = 2
    b = branch_trace([0], [1], 1, 2)
    b.table = other
    with pytest.raises(ValueError):
        oracle.MergedTrace([a, b])
    with pytest.raises(ValueError):
        oracle.MergedTrace([])
