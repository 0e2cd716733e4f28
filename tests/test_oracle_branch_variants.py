"""Pins for the oracle's branch-entropy variants: zero-initialised
histories, one global history over all branches, and the pattern form of
Yokota's branch history entropy.  Closed forms on constructed outcome
streams, relations between the variants, and the brute-force restatement
(outcome lists instead of shift registers) on random tiny traces."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import brute
from helpers import branch_trace, random_trace

ZERO, GLOBAL, PATTERN = oracle.BR_ZERO_HISTORY, oracle.BR_GLOBAL_HISTORY, oracle.BR_PATTERN


def run(sites, outcomes, n_sites, m, flags=0):
    t = branch_trace(sites, outcomes, n_sites, m)
    t.branch_flags = flags
    return oracle.characterize(t)


def de_bruijn(m):
    """Binary de Bruijn sequence of order m (every m-bit string once per cycle),
    by the standard Lyndon-word construction."""
    a = [0] * (2 * m)
    seq = []

    def db(t, p):
        if t > m:
            if m % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, 2):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    return seq


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(seed=st.integers(0, 2**32 - 1), n_sites=st.integers(1, 5), m=st.integers(1, 6),
       flags=st.sampled_from([PATTERN, ZERO | PATTERN, GLOBAL | PATTERN, GLOBAL | ZERO | PATTERN,
                              ZERO, GLOBAL]))
def test_variants_match_bruteforce(seed, n_sites, m, flags):
    rng = np.random.default_rng(seed)
    t = random_trace(rng, int(rng.integers(1, 5)), int(rng.integers(0, 120)), n_sites, m)
    t.branch_flags = flags
    r = oracle.characterize(t)
    b = brute.characterize(t.opcode, t.wi_offsets, t.table, t.addr, t.mem_kind, t.br_site,
                           t.br_taken, t.n_sites, m, flags=flags)
    for f in ("n_windows", "albe_min_sum", "total_branches", "unique_branches"):
        assert r[f] == b[f], f
    assert r["linear_branch_entropy"] == b["linear_branch_entropy"]
    assert math.isclose(r["yokota_entropy"], float(b["yokota_entropy"]), rel_tol=1e-12,
                        abs_tol=1e-300)
    if flags & PATTERN:
        assert math.isclose(r["pattern_entropy"], b["pattern_entropy"], rel_tol=1e-12,
                            abs_tol=1e-300)
    else:
        assert math.isnan(r["pattern_entropy"])


def test_zero_history_is_full_history_after_m_not_taken():
    # zero-initialised histories = the default start-up on the stream with m
    # not-taken executions of every site put in front
    rng = np.random.default_rng(4)
    m, ns = 5, 7
    s = rng.integers(0, ns, size=3000)
    y = (rng.random(3000) < 0.35).astype(np.uint8)
    z = run(s, y, ns, m, ZERO)
    pre_s = np.repeat(np.arange(ns), m)
    f = run(np.concatenate([pre_s, s]), np.concatenate([np.zeros(pre_s.size, np.uint8), y]),
            ns, m)
    assert z["n_windows"] == 3000 == f["n_windows"]
    assert z["albe_min_sum"] == f["albe_min_sum"]
    assert math.isclose(z["yokota_entropy"], f["yokota_entropy"], rel_tol=1e-13)


@pytest.mark.parametrize("m", [2, 4, 16])
def test_zero_history_alternation_scores_two_windows(m):
    # 0,1,0,1,...: only the all-not-taken history (before and after the first
    # outcome) is followed by both outcomes, once each
    n = 1000
    r = run([0] * n, [0, 1] * (n // 2), 1, m, ZERO)
    assert r["n_windows"] == n and r["albe_min_sum"] == 1
    assert r["linear_branch_entropy"] == 2 / n
    assert math.isclose(r["yokota_entropy"], 2 / n, rel_tol=1e-14)
    # the default start-up scores the same stream 0
    d = run([0] * n, [0, 1] * (n // 2), 1, m)
    assert d["albe_min_sum"] == 0 and d["yokota_entropy"] == 0.0


@pytest.mark.parametrize("flags", [0, ZERO])
def test_global_history_of_one_site_is_local(flags):
    rng = np.random.default_rng(12)
    y = (rng.random(2000) < 0.6).astype(np.uint8)
    a = run([3] * 2000, y, 4, 6, flags)
    b = run([3] * 2000, y, 4, 6, flags | GLOBAL)
    for f in ("n_windows", "albe_min_sum", "yokota_entropy"):
        assert a[f] == b[f], f


def test_global_history_hand_computed():
    # m = 1, stream (site, outcome): (0,1) (1,0) (0,1) (1,0) (0,0) (1,1)
    s, y = [0, 1, 0, 1, 0, 1], [1, 0, 1, 0, 0, 1]
    g = run(s, y, 2, 1, GLOBAL)
    # windows (site, previous outcome of the stream) -> outcome:
    # (1,1)->0 (0,0)->1 (1,1)->0 (0,0)->0 (1,0)->1: only key (0,0) mixes
    assert g["n_windows"] == 5 and g["albe_min_sum"] == 1
    assert g["linear_branch_entropy"] == 2 / 5
    assert math.isclose(g["yokota_entropy"], 2 / 5, rel_tol=1e-15)
    loc = run(s, y, 2, 1)
    # per site: 0 sees 1,1,0 and 1 sees 0,0,1: keys (0,1) and (1,0) both mix
    assert loc["n_windows"] == 4 and loc["albe_min_sum"] == 2
    assert loc["linear_branch_entropy"] == 1.0


def test_global_history_sees_correlated_branches():
    # site 1 copies the outcome site 0 just had: with the global history
    # every window of site 1 is determined, with its own history it is not
    rng = np.random.default_rng(6)
    a = (rng.random(4000) < 0.5).astype(np.uint8)
    s = np.tile([0, 1], 4000)
    y = np.repeat(a, 2)
    g = run(s, y, 2, 1, GLOBAL | PATTERN)
    one = run(np.zeros(4000, np.int64), a, 1, 1)      # site 0 alone, its own history
    # global keys of site 0 carry site 1's previous outcome = a[k-1]: the
    # same windows as site 0 alone; site 1 adds windows with min 0
    assert g["albe_min_sum"] == one["albe_min_sum"]
    assert g["n_windows"] == 2 * 4000 - 1
    loc = run(s, y, 2, 1)
    assert loc["albe_min_sum"] > 1.8 * one["albe_min_sum"]


@pytest.mark.parametrize("m", [1, 3, 5, 8])
def test_pattern_entropy_of_de_bruijn_is_one(m):
    # every m-bit history exactly R times among the windows: E_m = m
    seq = de_bruijn(m)
    R = 6
    y = seq * R + seq[:m]
    r = run([0] * len(y), y, 1, m, PATTERN)
    assert r["n_windows"] == R * 2 ** m
    assert math.isclose(r["pattern_entropy"], 1.0, rel_tol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 6, 16])
def test_pattern_entropy_closed_forms(m):
    # constant outcomes: one pattern
    assert run([0] * 500, [1] * 500, 1, m, PATTERN)["pattern_entropy"] == 0.0
    # alternation: two patterns, equally often when the window count is even
    n = 2 * 300 + m
    y = [0, 1] * (n // 2) + [0] * (n % 2)
    r = run([0] * n, y, 1, m, PATTERN)
    assert r["n_windows"] == 600
    assert math.isclose(r["pattern_entropy"], 1.0 / m, rel_tol=1e-14)
    # zero-initialised all-not-taken: one pattern again
    assert run([0] * 50, [0] * 50, 1, m, ZERO | PATTERN)["pattern_entropy"] == 0.0


def test_pattern_entropy_of_fair_coin_tends_to_one():
    rng = np.random.default_rng(99)
    y = (rng.random(200000) < 0.5).astype(np.uint8)
    r = run(np.zeros(y.size, np.int64), y, 1, 4, PATTERN)
    assert abs(r["pattern_entropy"] - 1.0) < 1e-3


def test_pattern_entropy_ignores_the_site():
    # the pattern distribution pools the windows of all sites
    y = [0, 0, 1, 1] * 50
    one = run([0] * 200, y, 1, 2, PATTERN)
    two = run([0] * 200 + [1] * 200, y + y, 2, 2, PATTERN)
    assert math.isclose(one["pattern_entropy"], two["pattern_entropy"], rel_tol=1e-15)
