"""Brute-force restatement of the AIWC metrics for tiny traces -- TEST
INFRASTRUCTURE ONLY.

Pure Python: ``collections.Counter`` for every histogram, exact integer and
``fractions`` arithmetic where the definition is rational, and mpmath at 50
significant digits for logarithms.  Used to pin the C oracle; shares nothing
with it beyond reading the same trace arrays.  The definitions and readings
follow arXiv 1805.04207, Table I and the Metrics / Implementation sections
(the same readings as aiwc_oracle.c states).
"""
from __future__ import annotations

from collections import Counter
from fractions import Fraction
from typing import Dict, List

import mpmath

mpmath.mp.dps = 50

BARRIER = 5


def _cover(counts: List[int], total: int) -> int:
    if total == 0:
        return 0
    cum = 0
    for i, c in enumerate(sorted(counts, reverse=True)):
        cum += c
        if Fraction(cum, total) >= Fraction(9, 10):
            return i + 1
    return len(counts)


def _median(v: List[int]) -> float:
    if not v:
        return 0.0
    v = sorted(v)
    n = len(v)
    if n % 2:
        return float(v[n // 2])
    return float(Fraction(v[n // 2 - 1] + v[n // 2], 2))


def _entropy(counter: Counter) -> mpmath.mpf:
    n = sum(counter.values())
    if n == 0:
        return mpmath.mpf(0)
    return mpmath.fsum(mpmath.mpf(c) / n * mpmath.log(mpmath.mpf(n) / c, 2)
                       for c in counter.values())


def characterize(opcode, wi_offsets, table, addr, mem_kind, br_site, br_taken,
                 n_sites: int, m: int, flags: int = 0) -> Dict:
    opcode = [int(x) for x in opcode]
    off = [int(x) for x in wi_offsets]
    cls = [int(table[i]["op_class"]) for i in range(len(table))]
    wid = [int(table[i]["simd_width"]) for i in range(len(table))]
    knd = [int(table[i]["kind"]) for i in range(len(table))]
    r: Dict = {}
    # compute
    ch = Counter(cls[o] for o in opcode)
    N = len(opcode)
    r["total_instructions"] = N
    r["unique_opcodes"] = len(ch)
    r["opcodes_90"] = _cover(list(ch.values()), N)
    ws = [wid[o] for o in opcode]
    r["simd_max"] = max(ws) if ws else 0
    s1, s2 = sum(ws), sum(w * w for w in ws)
    r["simd_sum"], r["simd_sumsq"] = s1, s2
    r["simd_mean"] = float(Fraction(s1, N)) if N else 0.0
    r["simd_sd"] = float(mpmath.sqrt(mpmath.mpf(N * s2 - s1 * s1)) / N) if N else 0.0
    # parallelism
    itb, ipt, nbar = [], [], 0
    for w in range(len(off) - 1):
        seg = 0
        for e in range(off[w], off[w + 1]):
            seg += 1
            if knd[opcode[e]] == BARRIER:
                itb.append(seg)
                seg = 0
                nbar += 1
        itb.append(seg)
        ipt.append(off[w + 1] - off[w])
    r["work_items"] = len(off) - 1
    r["barriers_hit"] = nbar
    r["itb_count"], r["itb_sum"] = len(itb), sum(itb)
    r["itb_min"], r["itb_max"] = (min(itb), max(itb)) if itb else (0, 0)
    r["itb_median"] = _median(itb)
    r["ipt_min"], r["ipt_max"] = (min(ipt), max(ipt)) if ipt else (0, 0)
    r["ipt_median"] = _median(ipt)
    # memory
    spaces = []
    for sp in (0, 1):
        acc = [(int(a), int(k)) for a, k in zip(addr, mem_kind) if (int(k) >> 1) & 1 == sp]
        reads = [a for a, k in acc if not k & 1]
        writes = [a for a, k in acc if k & 1]
        d: Dict = {"total_accesses": len(acc), "total_reads": len(reads),
                   "total_writes": len(writes), "unique_reads": len(set(reads)),
                   "unique_writes": len(set(writes)), "distinct": [], "entropy": []}
        for k in range(11):
            c = Counter(a >> k for a, _ in acc)
            d["distinct"].append(len(c))
            d["entropy"].append(_entropy(c))
            if k == 0:
                d["footprint"] = len(c)
                d["footprint_90"] = _cover(list(c.values()), len(acc))
                d["spectrum0"] = sorted(Counter(c.values()).items())
        spaces.append(d)
    r["space"] = spaces
    # branches
    # histories as outcome lists: per site, or one list shared by every site
    # (flags 4); started with m not-taken outcomes under flags 2, so that
    # every execution then has a full history
    hist: Dict[int, List[int]] = {}
    win = Counter()
    patterns = Counter()
    start = [0] * m if flags & 2 else []
    for s, y in zip(br_site, br_taken):
        s, y = int(s), int(y)
        h = hist.setdefault(-1 if flags & 4 else s, list(start))
        if len(h) >= m:
            win[(s, tuple(h[-m:]), y)] += 1
            patterns[tuple(h[-m:])] += 1
        h.append(y)
    keys = {(s, h) for (s, h, _) in win}
    nw = sum(win.values())
    mins, yok = 0, mpmath.mpf(0)
    for (s, h) in keys:
        n0, n1 = win[(s, h, 0)], win[(s, h, 1)]
        mins += min(n0, n1)
        n = n0 + n1
        for c in (n0, n1):
            if c:
                yok += c * mpmath.log(mpmath.mpf(n) / c, 2)
    sc = Counter(int(s) for s in br_site)
    r["total_branches"] = len(br_site)
    r["unique_branches"] = len(sc)
    r["branches_90"] = _cover(list(sc.values()), len(br_site))
    r["n_windows"] = nw
    r["albe_min_sum"] = mins
    r["yokota_entropy"] = yok / nw if nw else mpmath.mpf(0)
    r["linear_branch_entropy"] = float(Fraction(2 * mins, nw)) if nw else 0.0
    r["pattern_entropy"] = float("nan")
    if flags & 8:
        e = sum((c * mpmath.log(mpmath.mpf(nw) / c, 2) for c in patterns.values()),
                mpmath.mpf(0))
        r["pattern_entropy"] = float(e / nw / m) if nw else 0.0
    # derived parallelism metrics (LU decomposition analysis): exact
    # rationals rounded once, IEEE conventions for a zero denominator
    ratio = lambda a, b: float(Fraction(a, b)) if b else (float("inf") if a else float("nan"))
    r["granularity"] = ratio(1, r["work_items"])
    r["barriers_per_instruction"] = ratio(r["itb_count"], r["itb_sum"])
    r["instructions_per_operand"] = ratio(r["total_instructions"], r["simd_sum"])
    r["load_imbalance"] = r["ipt_max"] - r["ipt_min"]
    return r
