"""Pins for the CPU oracle: closed forms, the paper's one printed figure,
invariants and statistical limits.  Each test would fail on a plausible
slip in the oracle (a dropped term, a wrong shift or index, a swapped
operand); see the comment on each."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from helpers import (BARRIER, BRANCH, COMPUTE, ID_BARRIER, ID_BRANCH, ID_LOAD, ID_RET,
                     branch_trace, mem_trace, mk, table)

pytestmark = pytest.mark.filterwarnings("ignore")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def H2(p):
    return 0.0 if p in (0.0, 1.0) else -(p * math.log2(p) + (1 - p) * math.log2(1 - p))


# ---------------------------------------------------------------- memory
def test_single_address_zero_entropy_everywhere():
    # log1p(0) = 0 exactly: any cancellation error would leave a residue
    r = oracle.characterize(mem_trace([0x1234_5678] * 1000))
    s = r["space"][0]
    assert s["distinct"] == [1] * 11
    assert s["entropy"] == [0.0] * 11
    assert s["footprint_90"] == 1 and s["footprint"] == 1


def test_distinct_each_once_gives_log2_n_at_every_skip():
    # addresses 2 KiB apart stay distinct at every k <= 10
    n = 3000
    r = oracle.characterize(mem_trace([0x7000_0000 + 2048 * i for i in range(n)]))
    s = r["space"][0]
    assert s["distinct"] == [n] * 11
    for h in s["entropy"]:
        assert h == pytest.approx(math.log2(n), rel=1e-14)
    assert s["footprint_90"] == math.ceil(0.9 * n)


@pytest.mark.parametrize("nbits", [8, 12])
def test_dense_byte_sweep_loses_one_bit_per_skip(nbits):
    # aligned sweep of 2^n bytes: distinct_k = 2^(n-k), H_k = n - k exactly;
    # a wrong shift (a >> (k+1)) or a dropped count would break the ladder
    base = 1 << 20
    r = oracle.characterize(mem_trace(np.arange(base, base + (1 << nbits), dtype=np.uint64)))
    s = r["space"][0]
    for k in range(11):
        assert s["distinct"][k] == max(1, 1 << (nbits - k)) if nbits >= k else 1
        assert s["entropy"][k] == pytest.approx(max(0, nbits - k), abs=1e-12)


@pytest.mark.parametrize("j", [2, 5])
def test_power_of_two_stride_sweep(j):
    # stride 2^j over 2^n addresses: flat at n until k = j, then n - (k - j)
    n = 9
    r = oracle.characterize(mem_trace([(1 << 30) + (i << j) for i in range(1 << n)]))
    s = r["space"][0]
    for k in range(11):
        want = n if k <= j else max(0, n - (k - j))
        assert s["entropy"][k] == pytest.approx(want, abs=1e-12)
        assert s["distinct"][k] == 1 << want


def test_doubling_a_sweep_adds_one_bit():
    a = np.arange(0, 4 * 512, 4, dtype=np.uint64)
    b = np.arange(0, 4 * 1024, 4, dtype=np.uint64)
    ha = oracle.characterize(mem_trace(a))["space"][0]["entropy"]
    hb = oracle.characterize(mem_trace(b))["space"][0]["entropy"]
    for k in range(11):
        assert hb[k] - ha[k] == pytest.approx(1.0, abs=1e-12)


def test_entropy_of_known_distribution():
    # counts (4, 2, 1, 1) over 8 accesses: H = 1.75 bits exactly
    addr = [0] * 4 + [4096] * 2 + [8192, 12288]
    s = oracle.characterize(mem_trace(addr))["space"][0]
    assert s["entropy"][0] == pytest.approx(1.75, abs=1e-15)
    # footprint_90: 9*8 = 72 <= 10*cum -> 4,6,7,8 -> need all 4 (cum 7 gives 70)
    assert s["footprint_90"] == 4


def test_permutation_invariance_and_bounds():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 1 << 16, size=5000, dtype=np.uint64) * 3
    r1 = oracle.characterize(mem_trace(a))["space"][0]
    r2 = oracle.characterize(mem_trace(rng.permutation(a)))["space"][0]
    assert r1["distinct"] == r2["distinct"]
    assert r1["entropy"] == pytest.approx(r2["entropy"], rel=1e-15)
    d, h = r1["distinct"], r1["entropy"]
    for k in range(10):
        assert d[k + 1] <= d[k] <= 2 * d[k + 1]
        assert h[k + 1] <= h[k] + 1e-12 and h[k] <= h[k + 1] + 1 + 1e-12
        assert h[k] <= math.log2(d[k]) + 1e-12


def test_uniform_words_miller_madow():
    # N draws uniform over 2^m words: E[H] ~ m - (2^m - 1) / (2 N ln 2)
    rng = np.random.default_rng(11)
    m, N = 8, 200_000
    a = 4 * rng.integers(0, 1 << m, size=N, dtype=np.uint64)
    h = oracle.characterize(mem_trace(a))["space"][0]["entropy"][2]
    want = m - ((1 << m) - 1) / (2 * N * math.log(2))
    assert h == pytest.approx(want, abs=3e-4)


def test_reads_writes_and_spaces():
    # reads {A, B}, writes {B, C}; one local read; ratios are IEEE divisions
    A, B, C = 0x100, 0x200, 0x300
    addr = [A, A, B, B, C, 0x10]
    kinds = [0, 0, 0, 1, 1, 2]
    r = oracle.characterize(mem_trace(addr, kinds))
    g, l = r["space"]
    assert (g["total_reads"], g["total_writes"], g["total_accesses"]) == (3, 2, 5)
    assert (g["unique_reads"], g["unique_writes"], g["footprint"]) == (2, 2, 3)
    assert g["reread_ratio"] == 2 / 3 and g["rewrite_ratio"] == 1.0 and g["unique_rw_ratio"] == 1.0
    assert (l["total_reads"], l["total_writes"], l["footprint"]) == (1, 0, 1)
    assert math.isinf(l["unique_rw_ratio"]) and math.isnan(l["rewrite_ratio"])


def test_spectrum_matches_counts():
    addr = [1] * 5 + [2] * 5 + [3] * 2 + [4]
    assert oracle.spectrum(mem_trace(addr), 0, 0) == [(1, 1), (2, 1), (5, 2)]
    # k = 2: 1,2,3 share bucket 0 and 4 is bucket 1; k = 3: one bucket
    assert oracle.spectrum(mem_trace(addr), 0, 2) == [(1, 1), (12, 1)]
    assert oracle.spectrum(mem_trace(addr), 0, 3) == [(13, 1)]


# --------------------------------------------------------------- compute
@pytest.mark.parametrize("K", [1, 7, 10, 33])
def test_equal_frequency_classes_cover_ceil_point9(K):
    tab = table([(i, 1, COMPUTE) for i in range(K)])
    op = np.tile(np.arange(K, dtype=np.uint16), 5)
    r = oracle.characterize(mk(op, [op.size], tab=tab))
    assert r["unique_opcodes"] == K
    assert r["opcodes_90"] == math.ceil(0.9 * K)


def test_classes_merge_width_variants():
    # ids 0/1 are two widths of one class: the opcode metric counts classes
    tab = table([(0, 1, COMPUTE), (0, 4, COMPUTE), (1, 1, COMPUTE)])
    op = np.array([0] * 50 + [1] * 45 + [2] * 5, dtype=np.uint16)
    r = oracle.characterize(mk(op, [100], tab=tab))
    assert r["unique_opcodes"] == 2 and r["opcodes_90"] == 1
    assert list(oracle.class_hist(mk(op, [100], tab=tab), 3)) == [95, 5, 0]


def test_simd_closed_forms():
    tab = table([(0, 1, COMPUTE), (1, 4, COMPUTE)])
    op = np.array([0, 1] * 50, dtype=np.uint16)
    r = oracle.characterize(mk(op, [100], tab=tab))
    assert (r["simd_max"], r["simd_mean"], r["simd_sd"]) == (4, 2.5, 1.5)
    assert r["simd_sum"] == 250 and r["simd_sumsq_lo"] == 850
    r = oracle.characterize(mk(np.zeros(10, dtype=np.uint16), [10], tab=tab))
    assert (r["simd_max"], r["simd_mean"], r["simd_sd"]) == (1, 1.0, 0.0)


# ----------------------------------------------------------- parallelism
@pytest.mark.parametrize("L,B", [(100, 7), (256, 256), (255, 256), (50, 25), (1, 1)])
def test_itb_closed_form(L, B):
    # barrier at every B-th instruction: floor(L/B) segments of B, then one of L mod B
    op = np.array([ID_BARRIER if (p % B) == 0 else 0 for p in range(1, L + 1)], dtype=np.uint16)
    r = oracle.characterize(mk(op, [L]))
    segs = [B] * (L // B) + [L % B]
    assert r["barriers_hit"] == L // B
    assert r["itb_count"] == len(segs) and r["itb_sum"] == L
    assert (r["itb_min"], r["itb_max"]) == (min(segs), max(segs))
    assert r["itb_median"] == float(np.median(segs))


def test_needle_barriers_per_instruction_golden():
    # Demonstration section: the needle kernels run one barrier per 25
    # instructions, 0.04 barriers per instruction.
    g = json.load(open(os.path.join(GOLDEN, "needle_barriers.json")))
    B, L, W = g["barrier_every"], g["instructions_per_workitem"], g["work_items"]
    op = np.array([ID_BARRIER if (p % B) == 0 else 0 for p in range(1, L + 1)] * W,
                  dtype=np.uint16)
    r = oracle.characterize(mk(op, [L] * W))
    assert r["barriers_hit"] / r["total_instructions"] == g["barriers_per_instruction"]
    assert 1.0 / r["itb_median"] == g["barriers_per_instruction"]


def test_ipt_and_empty_workitems():
    op = np.zeros(10, dtype=np.uint16)
    r = oracle.characterize(mk(op, [0, 3, 7, 0]))
    assert (r["ipt_min"], r["ipt_max"], r["ipt_median"]) == (0, 7, 1.5)
    assert r["itb_count"] == 4 and r["itb_min"] == 0 and r["itb_max"] == 7
    assert r["work_items"] == 4


# --------------------------------------------------------------- control
def test_constant_and_periodic_branches_have_zero_entropy():
    for m in (1, 4, 16):
        for seq in ([1] * 200, [0] * 200, [0, 1] * 100, [1, 1, 0] * 70):
            if m < 2 and seq[:3] == [1, 1, 0]:
                continue  # period 3 is a function of the last 2 outcomes, not 1
            r = oracle.characterize(branch_trace([0] * len(seq), seq, 1, m))
            assert r["yokota_entropy"] == 0.0 and r["linear_branch_entropy"] == 0.0
            assert r["n_windows"] == max(0, len(seq) - m)


def test_deterministic_function_of_history_is_zero():
    # y_t = y_{t-1} xor y_{t-3}: a function of the last 3 outcomes -> 0 at m >= 3
    seq = [1, 0, 0]
    for _ in range(400):
        seq.append(seq[-1] ^ seq[-3])
    r = oracle.characterize(branch_trace([0] * len(seq), seq, 1, 3))
    assert r["yokota_entropy"] == 0.0 and r["albe_min_sum"] == 0
    r = oracle.characterize(branch_trace([0] * len(seq), seq, 1, 2))
    assert r["yokota_entropy"] > 0.1


@pytest.mark.parametrize("p", [0.5, 0.2])
def test_iid_bernoulli_limits(p):
    # m small, long sequence: Yokota -> H2(p), ALBE -> 2 min(p, 1-p)
    rng = np.random.default_rng(5)
    seq = (rng.random(400_000) < p).astype(np.uint8)
    r = oracle.characterize(branch_trace(np.zeros(seq.size), seq, 1, 2))
    assert r["yokota_entropy"] == pytest.approx(H2(p), abs=5e-3)
    assert r["linear_branch_entropy"] == pytest.approx(2 * min(p, 1 - p), abs=5e-3)


def test_branch_invariances():
    rng = np.random.default_rng(9)
    n, S, m = 6000, 5, 4
    sites = rng.integers(0, S, size=n).astype(np.uint32)
    ys = (rng.random(n) < rng.random(S)[sites]).astype(np.uint8)
    base = oracle.characterize(branch_trace(sites, ys, S, m))
    # per-site flip: ALBE bit-identical, Yokota equal up to summation order
    flip = ys ^ (sites % 2 == 0).astype(np.uint8)
    r = oracle.characterize(branch_trace(sites, flip, S, m))
    assert r["albe_min_sum"] == base["albe_min_sum"]
    assert r["linear_branch_entropy"] == base["linear_branch_entropy"]
    assert r["yokota_entropy"] == pytest.approx(base["yokota_entropy"], rel=1e-14)
    # site relabelling (a permutation of ids)
    perm = np.array([3, 0, 4, 1, 2], dtype=np.uint32)
    r = oracle.characterize(branch_trace(perm[sites], ys, S, m))
    assert r["albe_min_sum"] == base["albe_min_sum"]
    assert r["yokota_entropy"] == pytest.approx(base["yokota_entropy"], rel=1e-14)
    # interleaving of different sites does not matter, order within a site does
    order = np.argsort(sites, kind="stable")
    r = oracle.characterize(branch_trace(sites[order], ys[order], S, m))
    assert r["albe_min_sum"] == base["albe_min_sum"]
    assert r["n_windows"] == sum(max(0, int((sites == s).sum()) - m) for s in range(S))


def test_site_coverage_and_counts():
    sites = [0] * 50 + [1] * 30 + [2] * 15 + [3] * 5
    r = oracle.characterize(branch_trace(sites, [0] * 100, 6, 16))
    assert r["unique_branches"] == 4 and r["branches_90"] == 3 and r["total_branches"] == 100


def test_two_by_two_exact_yokota_and_albe():
    # m = 1, site 0: outcomes 0,0,1,0,1,1 -> windows (h=0:y=0),(0:1),(1:0),(0:1),(1:1)
    # key h=0: n0=1,n1=2 ; key h=1: n0=1,n1=1 ; N_w = 5
    r = oracle.characterize(branch_trace([0] * 6, [0, 0, 1, 0, 1, 1], 1, 1))
    want = (3 * H2(2 / 3) + 2 * 1.0) / 5
    assert r["n_windows"] == 5 and r["albe_min_sum"] == 2
    assert r["linear_branch_entropy"] == 0.8
    assert r["yokota_entropy"] == pytest.approx(want, rel=1e-15)
