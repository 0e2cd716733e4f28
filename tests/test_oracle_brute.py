"""The C oracle against a second, independent restatement (oracle/brute.py:
Counter + fractions + 50-digit mpmath) on random tiny traces."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import brute
from helpers import random_trace

INT_FIELDS = ["total_instructions", "unique_opcodes", "opcodes_90", "simd_max", "simd_sum",
              "work_items", "barriers_hit", "itb_count", "itb_sum", "itb_min", "itb_max",
              "ipt_min", "ipt_max", "total_branches", "unique_branches", "branches_90",
              "n_windows", "albe_min_sum", "load_imbalance"]
EXACT_FLOATS = ["simd_mean", "itb_median", "ipt_median", "linear_branch_entropy", "granularity",
                "barriers_per_instruction", "instructions_per_operand"]
SPACE_INTS = ["total_accesses", "total_reads", "total_writes", "unique_reads",
              "unique_writes", "footprint", "footprint_90"]


def _close(a, b, rel=1e-12):
    b = float(b)
    if b == 0.0:
        return a == 0.0
    return abs(a - b) <= rel * abs(b)


def check(tr):
    r = oracle.characterize(tr)
    b = brute.characterize(tr.opcode, tr.wi_offsets, tr.table, tr.addr, tr.mem_kind,
                           tr.br_site, tr.br_taken, tr.n_sites, tr.history_len)
    for f in INT_FIELDS:
        assert r[f] == b[f], f
    assert r["simd_sumsq_lo"] + (r["simd_sumsq_hi"] << 64) == b["simd_sumsq"]
    for f in EXACT_FLOATS:
        assert r[f] == b[f] or (math.isnan(r[f]) and math.isnan(b[f])), f
    assert _close(r["simd_sd"], b["simd_sd"], 1e-15)
    assert _close(r["yokota_entropy"], b["yokota_entropy"])
    for sp in (0, 1):
        rs, bs = r["space"][sp], b["space"][sp]
        for f in SPACE_INTS:
            assert rs[f] == bs[f], (sp, f)
        assert rs["distinct"] == bs["distinct"]
        for k in range(11):
            assert _close(rs["entropy"][k], bs["entropy"][k]), (sp, k)
        assert oracle.spectrum(tr, sp, 0) == bs["spectrum0"]


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(seed=st.integers(0, 2**32 - 1), n_wi=st.integers(1, 6), max_len=st.integers(0, 120),
       n_sites=st.integers(1, 5), m=st.integers(1, 5), bits=st.integers(1, 14))
def test_oracle_matches_bruteforce(seed, n_wi, max_len, n_sites, m, bits):
    rng = np.random.default_rng(seed)
    check(random_trace(rng, n_wi, max_len, n_sites, m, addr_bits=bits))


def test_oracle_matches_bruteforce_larger():
    rng = np.random.default_rng(1234)
    check(random_trace(rng, 20, 300, 7, 6, addr_bits=16))
