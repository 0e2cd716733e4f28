"""Vectorised restatement of the Table I metrics for traces too large for the
C oracle (10^9 events) -- TEST INFRASTRUCTURE ONLY.

Same definitions and readings as ``aiwc_oracle.c`` (arXiv 1805.04207, Table I
and the Metrics section), written with numpy primitives (bincount, sort,
unique, reduceat) instead of per-event loops, so that a full-size trace is
checked in about a minute.  It shares no code with the HIP path.  It is
pinned against the C oracle field by field on small traces
(tests/test_oracle_bulk.py); the GPU tests use it for the full-size
workloads.  Only tests may import it.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from typing import Dict

import numpy as np

K_BARRIER = 5        # opcode-table kind of a barrier instruction (as in the C oracle)
LN2 = math.log(2.0)


def _coverage90(counts: np.ndarray, total: int) -> int:
    """Fewest items, most frequent first, whose counts reach 90% of the total
    (10 * cum >= 9 * total in integers); 0 for an empty total."""
    if total == 0:
        return 0
    c = np.sort(np.asarray(counts, dtype=np.uint64))[::-1]
    cum = np.cumsum(c, dtype=np.uint64)          # totals here stay far below 2^60
    idx = np.flatnonzero(cum * np.uint64(10) >= np.uint64(9) * np.uint64(total))
    return int(idx[0]) + 1 if idx.size else int(c.size)


def _median(v: np.ndarray) -> float:
    """Median; the mean of the two middle values for an even count, in double."""
    n = v.size
    if n == 0:
        return 0.0
    if n & 1:
        return float(np.partition(v, n // 2)[n // 2])
    p = np.partition(v, [n // 2 - 1, n // 2])
    return (float(p[n // 2 - 1]) + float(p[n // 2])) * 0.5


def _runs(x: np.ndarray):
    """Distinct values of x and their multiplicities (sort, then run starts)."""
    v = np.sort(x)
    if v.size == 0:
        return v, np.zeros(0, dtype=np.int64)
    first = np.empty(v.size, dtype=bool)
    first[0] = True
    np.not_equal(v[1:], v[:-1], out=first[1:])
    starts = np.flatnonzero(first)
    return v[starts], np.diff(np.append(starts, v.size))


def _bincount(x: np.ndarray, n: int, threads: int) -> np.ndarray:
    """Histogram of small non-negative integers, chunked over threads."""
    if x.size == 0:
        return np.zeros(n, dtype=np.int64)
    chunks = np.array_split(x, max(1, min(threads, x.size // (1 << 20) + 1)))
    with ThreadPoolExecutor(len(chunks)) as ex:
        parts = list(ex.map(lambda c: np.bincount(c, minlength=n), chunks))
    return np.sum(parts, axis=0)


# ----------------------------------------------------------------- compute
def _compute(tr, r: Dict, threads: int) -> None:
    tab = np.asarray(tr.table)
    op = np.asarray(tr.opcode, dtype=np.uint16)
    n = int(op.size)
    ids = _bincount(op, len(tab), threads)                 # executions per opcode id
    cls_of = tab["op_class"].astype(np.int64)
    ncls = int(cls_of.max()) + 1 if len(tab) else 1
    cls = np.zeros(ncls, dtype=np.int64)
    np.add.at(cls, cls_of, ids)
    w = tab["simd_width"].astype(object)
    cnt = ids.astype(object)
    s1 = int(np.sum(cnt * w)) if len(tab) else 0
    s2 = int(np.sum(cnt * w * w)) if len(tab) else 0
    used = ids > 0
    r["total_instructions"] = n
    r["unique_opcodes"] = int(np.count_nonzero(cls))
    r["opcodes_90"] = _coverage90(cls, n)
    r["simd_max"] = int(tab["simd_width"][used].max()) if used.any() else 0
    r["simd_sum"] = s1
    r["simd_sumsq_lo"] = s2 & ((1 << 64) - 1)
    r["simd_sumsq_hi"] = s2 >> 64
    if n:
        r["simd_mean"] = float(s1) / float(n)
        u = n * s2 - s1 * s1                                # exact population variance * N^2
        r["simd_sd"] = math.sqrt(u) / n
    else:
        r["simd_mean"] = r["simd_sd"] = 0.0
    r["_class_hist"] = cls


# ------------------------------------------------------------- parallelism
def _parallelism(tr, r: Dict) -> None:
    """ITB: per work-item segments closed by each barrier (the barrier counts
    in the segment it closes) plus the final segment up to the end; IPT: the
    work-item's length."""
    tab = np.asarray(tr.table)
    op = np.asarray(tr.opcode, dtype=np.uint16)
    off = np.asarray(tr.wi_offsets, dtype=np.int64)
    n_wi = off.size - 1
    bar_ids = np.flatnonzero(tab["kind"] == K_BARRIER)
    if bar_ids.size == 1:
        bpos = np.flatnonzero(op == bar_ids[0])
    elif bar_ids.size:
        bpos = np.flatnonzero(np.isin(op, bar_ids))
    else:
        bpos = np.zeros(0, dtype=np.int64)
    bw = np.searchsorted(off, bpos, side="right") - 1       # work-item of each barrier
    same_prev = np.zeros(bpos.size, dtype=bool)
    same_prev[1:] = bw[1:] == bw[:-1]
    prev_end = np.zeros(bpos.size, dtype=np.int64)
    prev_end[1:] = bpos[:-1] + 1
    seg_start = np.where(same_prev, prev_end, off[bw] if bpos.size else prev_end)
    itb_b = bpos + 1 - seg_start
    nb = np.bincount(bw, minlength=n_wi) if n_wi else np.zeros(0, dtype=np.int64)
    final_start = off[:-1].copy()
    has = nb > 0
    last = np.cumsum(nb) - 1
    final_start[has] = bpos[last[has]] + 1
    itb_f = off[1:] - final_start
    itb = np.concatenate([itb_b, itb_f])
    ipt = np.diff(off)
    r["work_items"] = int(n_wi)
    r["barriers_hit"] = int(bpos.size)
    r["itb_count"] = int(itb.size)
    r["itb_sum"] = int(itb.sum())
    r["itb_min"] = int(itb.min()) if itb.size else 0
    r["itb_max"] = int(itb.max()) if itb.size else 0
    r["itb_median"] = _median(itb)
    r["ipt_min"] = int(ipt.min()) if ipt.size else 0
    r["ipt_max"] = int(ipt.max()) if ipt.size else 0
    r["ipt_median"] = _median(ipt)


# ------------------------------------------------------------------ memory
def _entropy(counts: np.ndarray, N: int) -> float:
    """sum over buckets of (c/N) log2(N/c), evaluated as c log1p((N-c)/c)/ln 2
    per distinct count value (multiplicities grouped, fsum)."""
    if N == 0 or counts.size == 0:
        return 0.0
    top = int(counts.max())
    if top < (1 << 24):
        mult = np.bincount(counts, minlength=top + 1)
        vals = np.flatnonzero(mult)
        mult = mult[vals]
    else:
        vals, mult = _runs(counts)
    terms = [int(m) * (float(c) * math.log1p((N - float(c)) / float(c)) / LN2)
             for c, m in zip(vals.tolist(), mult.tolist())]
    return math.fsum(terms) / N


def _space(addr: np.ndarray, write: np.ndarray) -> Dict:
    n = int(addr.size)
    s = {"total_accesses": n, "total_reads": int(n - np.count_nonzero(write)),
         "total_writes": int(np.count_nonzero(write))}
    if n:
        # one sort of (address, write flag): distinct reads / writes, and the
        # per-address counts from which every coarser level follows
        key = (addr.astype(np.uint64) << np.uint64(1)) | write.astype(np.uint64)
        uk, ck = _runs(key)
        del key
        a = uk >> np.uint64(1)
        s["unique_writes"] = int(np.count_nonzero(uk & np.uint64(1)))
        s["unique_reads"] = int(uk.size - s["unique_writes"])
        first = np.ones(a.size, dtype=bool)
        first[1:] = a[1:] != a[:-1]
        starts = np.flatnonzero(first)
        u0 = a[starts]
        c0 = np.add.reduceat(ck, starts)
        del uk, ck, a, first, starts
    else:
        s["unique_reads"] = s["unique_writes"] = 0
        u0 = np.zeros(0, dtype=np.uint64)
        c0 = np.zeros(0, dtype=np.int64)
    # neighbouring distinct addresses fall in one bucket a >> k exactly when
    # their highest differing bit is below k
    if u0.size > 1:
        x = (u0[1:] ^ u0[:-1]).astype(np.float64)       # exact: addresses < 2^53
        hb = (np.frexp(x)[1] - 1).astype(np.int8)
        del x
    else:
        hb = np.zeros(0, dtype=np.int8)
    C = np.zeros(c0.size + 1, dtype=np.int64)
    np.cumsum(c0, out=C[1:])
    dist, ent = [], []
    for k in range(11):
        if k == 0:
            c = c0
        else:
            st = np.flatnonzero(hb >= k) + 1
            b = np.empty(st.size + 2, dtype=np.int64)
            b[0] = 0
            b[1:-1] = st
            b[-1] = c0.size
            c = C[b[1:]] - C[b[:-1]] if c0.size else c0
        dist.append(int(c.size))
        ent.append(_entropy(c, n))
    s["footprint"] = dist[0]
    s["footprint_90"] = _coverage90(c0, n)
    s["distinct"] = dist
    s["entropy"] = ent
    with np.errstate(divide="ignore", invalid="ignore"):
        s["unique_rw_ratio"] = float(np.float64(s["unique_reads"]) / np.float64(s["unique_writes"]))
        s["reread_ratio"] = float(np.float64(s["unique_reads"]) / np.float64(s["total_reads"]))
        s["rewrite_ratio"] = float(np.float64(s["unique_writes"]) / np.float64(s["total_writes"]))
    s["_counts0"] = c0
    return s


def _memory(tr, r: Dict) -> None:
    addr = np.asarray(tr.addr, dtype=np.uint64)
    kind = np.asarray(tr.mem_kind, dtype=np.uint8)
    space = (kind >> 1) & 1
    r["space"] = []
    for sp in (0, 1):
        sel = space == sp
        r["space"].append(_space(addr[sel], (kind[sel] & 1).astype(bool)))


# ---------------------------------------------------------------- branches
def _branches(tr, r: Dict, threads: int) -> None:
    """Per-site history of the previous m outcomes in stream order; a window
    only once m earlier outcomes of its site exist; per (site, history) the
    outcome counts n0, n1.  Variants (trace attribute branch_flags, same
    values as the C oracle's ORC_BR_*): zero-initialised histories with a
    window at every execution; one global history over all branches; the
    pattern entropy E_m / m over the windows' histories."""
    site = np.asarray(tr.br_site, dtype=np.uint32)
    y = np.asarray(tr.br_taken, dtype=np.uint8).astype(np.uint64) & np.uint64(1)
    m = int(tr.history_len)
    ns = int(tr.n_sites)
    nb = int(site.size)
    flags = int(getattr(tr, "branch_flags", 0))
    zero, glob = bool(flags & 2), bool(flags & 4)
    seen = _bincount(site, ns, threads) if nb else np.zeros(ns, dtype=np.int64)
    r["total_branches"] = nb
    r["unique_branches"] = int(np.count_nonzero(seen))
    r["branches_90"] = _coverage90(seen, nb)
    r["pattern_entropy"] = 0.0 if flags & 8 else float("nan")
    if nb == 0:
        r["n_windows"] = r["albe_min_sum"] = 0
        r["yokota_entropy"] = r["linear_branch_entropy"] = 0.0
        return
    if glob:
        # one register over the stream: no grouping by site before the history
        s_sorted = site.astype(np.uint64)
        y_sorted = y
        pos = np.arange(nb)
    else:
        order = np.argsort(site, kind="stable")
        s_sorted = site[order].astype(np.uint64)
        y_sorted = y[order]
        seg_first = np.ones(nb, dtype=bool)
        seg_first[1:] = s_sorted[1:] != s_sorted[:-1]
        seg_start = np.maximum.accumulate(np.where(seg_first, np.arange(nb), 0))
        pos = np.arange(nb) - seg_start                       # rank within the site
    valid = np.ones(nb, dtype=bool) if zero else pos >= m
    hist = np.zeros(nb, dtype=np.uint64)
    for j in range(1, m + 1):                                 # bit j-1 = outcome j back
        bit = y_sorted[:-j] << np.uint64(j - 1)
        if zero:
            bit = np.where(pos[j:] >= j, bit, np.uint64(0))   # before the start: not taken
        hist[j:] |= bit
    key = (s_sorted[valid] << np.uint64(m)) | hist[valid]
    if flags & 8 and key.size:
        _, pc = np.unique(hist[valid], return_counts=True)
        nwv = int(valid.sum())
        r["pattern_entropy"] = math.fsum(float(c) * math.log2(nwv / float(c))
                                         for c in pc.tolist()) / nwv / m
    kk = (key << np.uint64(1)) | y_sorted[valid]
    uk, ck = _runs(kk)
    kid = uk >> np.uint64(1)
    first = np.ones(kid.size, dtype=bool)
    first[1:] = kid[1:] != kid[:-1]
    starts = np.flatnonzero(first)
    tot = np.add.reduceat(ck, starts) if ck.size else ck
    ones = np.add.reduceat(np.where(uk & np.uint64(1), ck, 0), starts) if ck.size else ck
    n1 = ones.astype(np.int64)
    n0 = tot.astype(np.int64) - n1
    nw = int(valid.sum())
    minsum = int(np.minimum(n0, n1).sum())
    both = (n0 > 0) & (n1 > 0)
    pairs = (n0[both].astype(np.uint64) << np.uint64(32)) | n1[both].astype(np.uint64)
    pv, pm = _runs(pairs)
    terms = []
    for p, mult in zip(pv.tolist(), pm.tolist()):
        a, b = float(p >> 32), float(p & 0xFFFFFFFF)
        terms.append(mult * ((a * math.log1p(b / a) + b * math.log1p(a / b)) / LN2))
    r["n_windows"] = nw
    r["albe_min_sum"] = minsum
    r["yokota_entropy"] = math.fsum(terms) / nw if nw else 0.0
    r["linear_branch_entropy"] = float(2 * minsum) / float(nw) if nw else 0.0


def characterize(tr, threads: int = 16, progress=None) -> Dict:
    """All metrics of one host trace, in the C oracle's result layout (plus
    the class histogram and level-0 counts under private keys).  progress, if
    given, is called with a short message after each part."""
    r: Dict = {}
    say = progress or (lambda msg: None)
    _compute(tr, r, threads)
    say("compute metrics done")
    _parallelism(tr, r)
    say("parallelism metrics done")
    _memory(tr, r)
    say("memory metrics done")
    _branches(tr, r, threads)
    say("branch metrics done")
    _derived(r)
    return r


def _ieee_div(a: int, b: int) -> float:
    """a / b as one IEEE double division (x/0 = inf, 0/0 = NaN)."""
    return float(np.float64(a) / np.float64(b)) if b else (float("inf") if a else float("nan"))


def _derived(r: Dict) -> None:
    """Derived parallelism metrics of the LU decomposition analysis
    (Evaluation section): inverses of work-items, mean ITB and mean SIMD
    width, and load imbalance = max IPT - min IPT."""
    r["granularity"] = _ieee_div(1, r["work_items"])
    r["barriers_per_instruction"] = _ieee_div(r["itb_count"], r["itb_sum"])
    r["instructions_per_operand"] = _ieee_div(r["total_instructions"], r["simd_sum"])
    r["load_imbalance"] = r["ipt_max"] - r["ipt_min"]
