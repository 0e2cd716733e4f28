/*
 * aiwc_oracle.h -- CPU oracle for the AIWC metrics (TEST INFRASTRUCTURE).
 *
 * A plain, slow, single-threaded restatement of the metric definitions of
 * Johnston & Milthorpe, "AIWC: OpenCL-based Architecture-Independent Workload
 * Characterization" (arXiv 1805.04207), Table I and the Metrics and
 * Implementation sections.  It exists only to check the HIP implementation:
 * only the tests, the smoke entry point and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or table with the HIP library.
 *
 * Floating-point results accumulate in long double (x87 extended, wider than
 * IEEE binary64) and are returned as double.
 */
#ifndef AIWC_ORACLE_H
#define AIWC_ORACLE_H
#include <stddef.h>
#include <stdint.h>

typedef struct orc_opinfo {
  uint16_t op_class;
  uint8_t simd_width;
  uint8_t kind; /* 0 compute, 1 load, 2 store, 3 atomic rmw, 4 cond branch,
                   5 barrier, 6 other */
} orc_opinfo;

typedef struct orc_trace {
  uint64_t n_events;
  const uint16_t *opcode;
  uint64_t n_wi;
  const uint64_t *wi_offsets; /* [n_wi + 1] */
  uint32_t n_ids;
  uint32_t n_sites;
  const orc_opinfo *table;    /* [n_ids] */
  uint64_t n_mem;
  const uint64_t *addr;
  const uint8_t *mem_kind;    /* bit0 write, bit1 local space */
  uint64_t n_branch;
  const uint32_t *br_site;
  const uint8_t *br_taken;
  uint32_t history_len;       /* m, 1..32 */
  uint32_t flags;             /* ORC_BR_* branch-entropy variants        */
} orc_trace;

/* Branch-entropy variants (Related Work: Yokota's branch history entropy,
 * De Pestel's linear entropy; Implementation: "the full history of combined
 * branch's taken and not-taken").  The default is a per-site history whose
 * windows start once m earlier outcomes exist; these bits select the other
 * readings.  (The values are the interface of the trace flags.)            */
#define ORC_BR_ZERO_HISTORY 2u    /* histories start as m not-taken outcomes;
                                     every branch event forms a window     */
#define ORC_BR_GLOBAL_HISTORY 4u  /* one history of the previous m outcomes
                                     of all branches, keyed with the site  */
#define ORC_BR_PATTERN 8u         /* also report the pattern entropy       */

typedef struct orc_space {
  uint64_t total_accesses, total_reads, total_writes;
  uint64_t unique_reads, unique_writes;
  uint64_t footprint, footprint_90;
  uint64_t distinct[11];
  double entropy[11];
  double unique_rw_ratio, reread_ratio, rewrite_ratio;
} orc_space;

typedef struct orc_result {
  uint64_t total_instructions;
  uint64_t unique_opcodes, opcodes_90;
  uint64_t simd_max, simd_sum, simd_sumsq_lo, simd_sumsq_hi;
  double simd_mean, simd_sd;
  uint64_t work_items, barriers_hit;
  uint64_t itb_count, itb_sum, itb_min, itb_max;
  double itb_median;
  uint64_t ipt_min, ipt_max;
  double ipt_median;
  orc_space space[2];
  uint64_t total_branches, unique_branches, branches_90;
  uint64_t n_windows, albe_min_sum;
  double yokota_entropy, linear_branch_entropy;
  double pattern_entropy;     /* E_m / m with ORC_BR_PATTERN, else NaN      */
  /* derived parallelism metrics (LU decomposition analysis) */
  double granularity, barriers_per_instruction, instructions_per_operand;
  uint64_t load_imbalance;
} orc_result;

/* 0 = ok, 1 = invalid trace, 2 = out of memory */
int orc_characterize(const orc_trace *t, orc_result *out);
/* 1 when #LOAD + #STORE + 2 #ATOMIC_RMW == n_mem and #BRANCH_COND ==
 * n_branch (an atomic is one instruction with a read and a write event),
 * 0 when not, -1 for an invalid trace.                                      */
int orc_kinds_consistent(const orc_trace *t);
/* Per-class instruction counts into out[len] (zeros beyond the classes). */
int orc_class_hist(const orc_trace *t, uint64_t *out, size_t len);
/* Count-of-counts of (space, skip k): ascending f; n_out = number of pairs. */
int orc_spectrum(const orc_trace *t, int space, int k, uint64_t *f, uint64_t *mf,
                 size_t cap, size_t *n_out);

#endif
