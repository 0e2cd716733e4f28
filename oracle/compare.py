"""Field-by-field comparison of libaiwc results with the oracle's -- TEST
INFRASTRUCTURE ONLY.

Bar: every integer (counts, distinct counts, coverage counts, extrema, the
128-bit SIMD sums, ALBE numerator) bit-exact; every value that is one IEEE
operation on exact integers (means, medians, ratios, ALBE) bit-identical;
the SIMD SD within 1e-15 relative (both take one square root of the same
exact integer, converted to double in different ways); entropies within
1e-9 relative, and exactly 0 where the oracle gives 0.
"""
from __future__ import annotations

import math
from typing import Dict, List

INT_TOP = ["total_instructions", "unique_opcodes", "opcodes_90", "simd_max", "simd_sum",
           "simd_sumsq_lo", "simd_sumsq_hi", "work_items", "barriers_hit", "itb_count",
           "itb_sum", "itb_min", "itb_max", "ipt_min", "ipt_max", "total_branches",
           "unique_branches", "branches_90", "n_windows", "albe_min_sum", "load_imbalance"]
EXACT_TOP = ["simd_mean", "itb_median", "ipt_median", "linear_branch_entropy", "granularity",
             "barriers_per_instruction", "instructions_per_operand"]
INT_SPACE = ["total_accesses", "total_reads", "total_writes", "unique_reads", "unique_writes",
             "footprint", "footprint_90"]
EXACT_SPACE = ["unique_rw_ratio", "reread_ratio", "rewrite_ratio"]
ENTROPY_REL = 1e-9


def _same_float(a: float, b: float) -> bool:
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b


def _rel_ok(a: float, b: float, rel: float) -> bool:
    if b == 0.0:
        return a == 0.0
    return abs(a - b) <= rel * abs(b)


def compare(gpu: Dict, orc: Dict) -> List[str]:
    """List of mismatches (empty when the two agree to the bar above)."""
    bad = []
    for f in INT_TOP:
        if int(gpu[f]) != int(orc[f]):
            bad.append(f"{f}: gpu {gpu[f]} oracle {orc[f]}")
    for f in EXACT_TOP:
        if not _same_float(gpu[f], orc[f]):
            bad.append(f"{f}: gpu {gpu[f]!r} oracle {orc[f]!r}")
    if not _rel_ok(gpu["simd_sd"], orc["simd_sd"], 1e-15):
        bad.append(f"simd_sd: gpu {gpu['simd_sd']!r} oracle {orc['simd_sd']!r}")
    if not _rel_ok(gpu["yokota_entropy"], orc["yokota_entropy"], ENTROPY_REL):
        bad.append(f"yokota: gpu {gpu['yokota_entropy']!r} oracle {orc['yokota_entropy']!r}")
    gp, op = gpu.get("pattern_entropy", math.nan), orc.get("pattern_entropy", math.nan)
    if not ((math.isnan(gp) and math.isnan(op)) or
            (not math.isnan(gp) and not math.isnan(op) and _rel_ok(gp, op, ENTROPY_REL))):
        bad.append(f"pattern_entropy: gpu {gp!r} oracle {op!r}")
    for s in (0, 1):
        g, o = gpu["space"][s], orc["space"][s]
        for f in INT_SPACE:
            if int(g[f]) != int(o[f]):
                bad.append(f"space{s}.{f}: gpu {g[f]} oracle {o[f]}")
        for f in EXACT_SPACE:
            if not _same_float(g[f], o[f]):
                bad.append(f"space{s}.{f}: gpu {g[f]!r} oracle {o[f]!r}")
        for k in range(11):
            if int(g["distinct"][k]) != int(o["distinct"][k]):
                bad.append(f"space{s}.distinct[{k}]: gpu {g['distinct'][k]} oracle {o['distinct'][k]}")
            if not _rel_ok(g["entropy"][k], o["entropy"][k], ENTROPY_REL):
                bad.append(f"space{s}.entropy[{k}]: gpu {g['entropy'][k]!r} oracle {o['entropy'][k]!r}")
    return bad
