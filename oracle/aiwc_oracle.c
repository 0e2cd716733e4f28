/*
 * aiwc_oracle.c -- CPU oracle for the AIWC metrics (TEST INFRASTRUCTURE; see
 * aiwc_oracle.h).  Every function restates one definition of the paper in
 * the most direct form: histograms, qsort, and walks over sorted runs.
 * Readings of points the paper leaves open are marked "Reading:".
 */
#include "aiwc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LN2L 0.693147180559945309417232121458176568L

enum { K_COMPUTE = 0, K_LOAD, K_STORE, K_ATOMIC, K_BRANCH, K_BARRIER, K_OTHER };

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

static int cmp_u64_desc(const void *a, const void *b) { return cmp_u64(b, a); }

/* "# of unique X that cover 90% of Y" (Table I: Opcode, 90% Memory
 * Footprint, 90% Branch Instructions).  Reading: the smallest number of
 * items, taken most frequent first, whose counts sum to at least 90% of the
 * total, tested exactly in integers as 10*cum >= 9*total; 0 when total = 0. */
static uint64_t coverage90(uint64_t *counts, size_t n, uint64_t total) {
  if (total == 0) return 0;
  qsort(counts, n, sizeof(uint64_t), cmp_u64_desc);
  unsigned __int128 cum = 0;
  for (size_t i = 0; i < n; ++i) {
    cum += counts[i];
    if (cum * 10 >= (unsigned __int128)total * 9) return (uint64_t)(i + 1);
  }
  return (uint64_t)n;
}

/* Median of a sample; reading: the mean of the two middle values when the
 * count is even, computed in double. */
static double median_sorted(const uint64_t *v, size_t n) {
  if (n == 0) return 0.0;
  if (n & 1) return (double)v[n / 2];
  return ((double)v[n / 2 - 1] + (double)v[n / 2]) * 0.5;
}

/* ---------------------------------------------------------------- compute
 * Table I, Compute rows, and the Implementation section: each executed
 * instruction increments a map keyed by its LLVM opcode name (here: the
 * op_class of its id); SIMD width is the number of data items of the
 * instruction's result, one value per executed instruction.              */
static int compute_metrics(const orc_trace *t, orc_result *r) {
  uint32_t ncls = 0;
  for (uint32_t i = 0; i < t->n_ids; ++i)
    if ((uint32_t)t->table[i].op_class + 1 > ncls) ncls = t->table[i].op_class + 1u;
  uint64_t *cls = (uint64_t *)calloc(ncls ? ncls : 1, sizeof(uint64_t));
  if (!cls) return 2;
  uint64_t s1 = 0, wmax = 0;
  unsigned __int128 s2 = 0;
  for (uint64_t e = 0; e < t->n_events; ++e) {
    const orc_opinfo *oi = &t->table[t->opcode[e]];
    cls[oi->op_class]++;
    uint64_t w = oi->simd_width;
    s1 += w;
    s2 += (unsigned __int128)(w * w);
    if (w > wmax) wmax = w;
  }
  uint64_t uniq = 0;
  for (uint32_t c = 0; c < ncls; ++c) uniq += cls[c] != 0;
  r->total_instructions = t->n_events;
  r->unique_opcodes = uniq;
  r->opcodes_90 = coverage90(cls, ncls, t->n_events);
  r->simd_max = wmax;
  r->simd_sum = s1;
  r->simd_sumsq_lo = (uint64_t)s2;
  r->simd_sumsq_hi = (uint64_t)(s2 >> 64);
  if (t->n_events) {
    long double n = (long double)t->n_events;
    r->simd_mean = (double)s1 / (double)t->n_events;
    /* population SD (reading: divide by N): sqrt(N*S2 - S1^2) / N */
    unsigned __int128 u = (unsigned __int128)t->n_events * s2 -
                          (unsigned __int128)s1 * (unsigned __int128)s1;
    long double ul = (long double)(uint64_t)(u >> 64) * 18446744073709551616.0L +
                     (long double)(uint64_t)u;
    r->simd_sd = (double)(sqrtl(ul) / n);
  } else {
    r->simd_mean = 0.0;
    r->simd_sd = 0.0;
  }
  free(cls);
  return 0;
}

/* ------------------------------------------------------------ parallelism
 * Metrics section: a running tally of instructions per work-item is saved
 * and reset whenever a barrier is met, and the end of the kernel counts as a
 * final implicit barrier (ITB).  IPT is the tally per work-item until
 * completion.  Reading: the barrier instruction counts inside the segment it
 * closes, so each work-item yields (#barriers + 1) ITB values, the last one
 * possibly 0.  Total Barriers Hit counts explicit barrier instructions.   */
static int parallel_metrics(const orc_trace *t, orc_result *r) {
  uint64_t nbar = 0;
  for (uint64_t e = 0; e < t->n_events; ++e)
    nbar += t->table[t->opcode[e]].kind == K_BARRIER;
  size_t nitb = (size_t)(nbar + t->n_wi);
  uint64_t *itb = (uint64_t *)malloc((nitb ? nitb : 1) * sizeof(uint64_t));
  uint64_t *ipt = (uint64_t *)malloc((t->n_wi ? t->n_wi : 1) * sizeof(uint64_t));
  if (!itb || !ipt) { free(itb); free(ipt); return 2; }
  size_t j = 0;
  uint64_t sum = 0;
  for (uint64_t w = 0; w < t->n_wi; ++w) {
    uint64_t seg = 0;
    for (uint64_t e = t->wi_offsets[w]; e < t->wi_offsets[w + 1]; ++e) {
      seg++;
      if (t->table[t->opcode[e]].kind == K_BARRIER) {
        itb[j++] = seg;
        sum += seg;
        seg = 0;
      }
    }
    itb[j++] = seg;
    sum += seg;
    ipt[w] = t->wi_offsets[w + 1] - t->wi_offsets[w];
  }
  qsort(itb, j, sizeof(uint64_t), cmp_u64);
  qsort(ipt, (size_t)t->n_wi, sizeof(uint64_t), cmp_u64);
  r->work_items = t->n_wi;
  r->barriers_hit = nbar;
  r->itb_count = j;
  r->itb_sum = sum;
  r->itb_min = j ? itb[0] : 0;
  r->itb_max = j ? itb[j - 1] : 0;
  r->itb_median = median_sorted(itb, j);
  r->ipt_min = t->n_wi ? ipt[0] : 0;
  r->ipt_max = t->n_wi ? ipt[t->n_wi - 1] : 0;
  r->ipt_median = median_sorted(ipt, (size_t)t->n_wi);
  free(itb);
  free(ipt);
  return 0;
}

/* ----------------------------------------------------------------- memory */
static size_t distinct_sorted(const uint64_t *v, size_t n) {
  size_t d = 0;
  for (size_t i = 0; i < n; ++i) d += (i == 0 || v[i] != v[i - 1]);
  return d;
}

/* Gather the addresses of one space; sel: 0 = all, 1 = reads, 2 = writes. */
static uint64_t *gather(const orc_trace *t, int space, int sel, size_t *n) {
  size_t c = 0;
  for (uint64_t i = 0; i < t->n_mem; ++i) {
    uint8_t k = t->mem_kind[i];
    if ((int)((k >> 1) & 1u) != space) continue;
    if (sel == 1 && (k & 1u)) continue;
    if (sel == 2 && !(k & 1u)) continue;
    ++c;
  }
  uint64_t *v = (uint64_t *)malloc((c ? c : 1) * sizeof(uint64_t));
  if (!v) return NULL;
  size_t j = 0;
  for (uint64_t i = 0; i < t->n_mem; ++i) {
    uint8_t k = t->mem_kind[i];
    if ((int)((k >> 1) & 1u) != space) continue;
    if (sel == 1 && (k & 1u)) continue;
    if (sel == 2 && !(k & 1u)) continue;
    v[j++] = t->addr[i];
  }
  *n = c;
  return v;
}

/* Table I, Memory rows and the Metrics section.  The addresses of one
 * space, with k least significant bits dropped (k = 0: global memory
 * address entropy; k = 1..10: the local memory address entropy curve), form
 * buckets a >> k.  Distinct_k = number of buckets; entropy_k is Shannon's
 * plug-in entropy in bits of the bucket frequencies,
 *   H_k = sum_b (c_b / N) * log2(N / c_b),
 * evaluated as (c/N) * log1p((N - c) / c) / ln 2 so that c = N gives 0.
 * The total footprint is distinct_0; the 90% footprint covers 90% of the
 * accesses with the most-accessed addresses first.  Unique reads / writes
 * are distinct read / write addresses; the ratios are the IEEE divisions of
 * those integers (reading for zero denominators: inf / NaN).              */
static int space_metrics(const orc_trace *t, int space, orc_space *s) {
  size_t n, nr, nw;
  uint64_t *a = gather(t, space, 0, &n);
  uint64_t *rd = gather(t, space, 1, &nr);
  uint64_t *wr = gather(t, space, 2, &nw);
  uint64_t *counts = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!a || !rd || !wr || !counts) { free(a); free(rd); free(wr); free(counts); return 2; }
  qsort(a, n, sizeof(uint64_t), cmp_u64);
  qsort(rd, nr, sizeof(uint64_t), cmp_u64);
  qsort(wr, nw, sizeof(uint64_t), cmp_u64);
  for (int k = 0; k <= 10; ++k) {
    size_t runs = 0, i = 0;
    long double h = 0.0L, N = (long double)n;
    while (i < n) {
      size_t j = i + 1;
      while (j < n && (a[j] >> k) == (a[i] >> k)) ++j;
      uint64_t c = (uint64_t)(j - i);
      h += ((long double)c / N) * log1pl((N - (long double)c) / (long double)c) / LN2L;
      if (k == 0) counts[runs] = c;
      ++runs;
      i = j;
    }
    s->distinct[k] = runs;
    s->entropy[k] = (double)h;
    if (k == 0) s->footprint_90 = coverage90(counts, runs, n);
  }
  s->total_accesses = n;
  s->total_reads = nr;
  s->total_writes = nw;
  s->unique_reads = distinct_sorted(rd, nr);
  s->unique_writes = distinct_sorted(wr, nw);
  s->footprint = s->distinct[0];
  s->unique_rw_ratio = (double)s->unique_reads / (double)s->unique_writes;
  s->reread_ratio = (double)s->unique_reads / (double)s->total_reads;
  s->rewrite_ratio = (double)s->unique_writes / (double)s->total_writes;
  free(a); free(rd); free(wr); free(counts);
  return 0;
}

/* --------------------------------------------------------------- branches
 * Table I, Control rows, and the Implementation section (per-site outcome
 * histories; branch metrics over 16-outcome history strings).
 * Reading: each site keeps its own history of its previous m outcomes,
 * h <- ((h << 1) | y) mod 2^m, in stream order; an execution forms a window
 * only once m earlier outcomes of its site exist, so N_w = sum_s max(0,
 * n_s - m).  For each key (site, h) let n0 / n1 count the outcomes 0 / 1.
 *   Yokota (Shannon, in [0,1]) = sum_keys [n0 log2(n/n0) + n1 log2(n/n1)] / N_w
 *   average linear branch entropy = sum_keys n * 2 min(p, 1-p) / N_w
 *                                 = 2 sum_keys min(n0, n1) / N_w
 * (De Pestel's linear entropy weighted by pattern frequency); both 0 when
 * N_w = 0.
 * Variants (trace flags):
 *   ORC_BR_ZERO_HISTORY   every history starts as m not-taken outcomes and
 *                         every execution forms a window (N_w = n_branch).
 *   ORC_BR_GLOBAL_HISTORY one history register over all branches in stream
 *                         order (the "combined" history of the Implementation
 *                         section); the key is still (site, h).  Windows
 *                         start once m earlier outcomes of any site exist
 *                         (N_w = max(0, n_branch - m)), or at once with
 *                         ORC_BR_ZERO_HISTORY.
 *   ORC_BR_PATTERN        Yokota's branch history entropy in its pattern
 *                         form: E_m = sum_p c_p log2(N_w / c_p) over the
 *                         m-bit histories p of the windows (whatever their
 *                         site), reported normalised as E_m / m in [0, 1];
 *                         0 when N_w = 0, NaN when not requested.          */
typedef struct { uint64_t key; uint64_t y; } win_t;

static int cmp_win(const void *a, const void *b) {
  const win_t *x = (const win_t *)a, *z = (const win_t *)b;
  if (x->key != z->key) return (x->key > z->key) - (x->key < z->key);
  return (x->y > z->y) - (x->y < z->y);
}

static int branch_metrics(const orc_trace *t, orc_result *r) {
  uint32_t m = t->history_len;
  uint64_t mask = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
  uint64_t *hist = (uint64_t *)calloc(t->n_sites ? t->n_sites : 1, sizeof(uint64_t));
  uint64_t *seen = (uint64_t *)calloc(t->n_sites ? t->n_sites : 1, sizeof(uint64_t));
  win_t *win = (win_t *)malloc((t->n_branch ? t->n_branch : 1) * sizeof(win_t));
  uint64_t *pat = (uint64_t *)malloc((t->n_branch ? t->n_branch : 1) * sizeof(uint64_t));
  if (!hist || !seen || !win || !pat) {
    free(hist); free(seen); free(win); free(pat);
    return 2;
  }
  const int zero = (t->flags & ORC_BR_ZERO_HISTORY) != 0;
  const int glob = (t->flags & ORC_BR_GLOBAL_HISTORY) != 0;
  uint64_t gh = 0, gseen = 0;   /* the one register of the global variant */
  size_t nw = 0;
  for (uint64_t i = 0; i < t->n_branch; ++i) {
    uint32_t s = t->br_site[i];
    uint64_t y = t->br_taken[i];
    uint64_t h = glob ? gh : hist[s];
    uint64_t before = glob ? gseen : seen[s];
    if (zero || before >= m) {
      win[nw].key = ((uint64_t)s << m) | h;
      win[nw].y = y;
      pat[nw] = h;
      ++nw;
    }
    hist[s] = ((hist[s] << 1) | y) & mask;
    seen[s]++;
    gh = ((gh << 1) | y) & mask;
    gseen++;
  }
  uint64_t uniq = 0;
  for (uint32_t s = 0; s < t->n_sites; ++s) uniq += seen[s] != 0;
  r->total_branches = t->n_branch;
  r->unique_branches = uniq;
  r->branches_90 = coverage90(seen, t->n_sites, t->n_branch);
  qsort(win, nw, sizeof(win_t), cmp_win);
  uint64_t minsum = 0;
  long double yok = 0.0L;
  size_t i = 0;
  while (i < nw) {
    size_t j = i;
    uint64_t n0 = 0, n1 = 0;
    while (j < nw && win[j].key == win[i].key) {
      if (win[j].y) ++n1; else ++n0;
      ++j;
    }
    minsum += n0 < n1 ? n0 : n1;
    if (n0 && n1)
      yok += ((long double)n0 * log1pl((long double)n1 / (long double)n0) +
              (long double)n1 * log1pl((long double)n0 / (long double)n1)) / LN2L;
    i = j;
  }
  r->n_windows = nw;
  r->albe_min_sum = minsum;
  r->yokota_entropy = nw ? (double)(yok / (long double)nw) : 0.0;
  r->linear_branch_entropy = nw ? (double)(2 * minsum) / (double)nw : 0.0;
  r->pattern_entropy = NAN;
  if (t->flags & ORC_BR_PATTERN) {
    qsort(pat, nw, sizeof(uint64_t), cmp_u64);
    long double e = 0.0L;
    size_t a = 0;
    while (a < nw) {
      size_t b = a;
      while (b < nw && pat[b] == pat[a]) ++b;
      const long double c = (long double)(b - a);
      e += c * log2l((long double)nw / c);
      a = b;
    }
    r->pattern_entropy = nw ? (double)(e / (long double)nw / (long double)m) : 0.0;
  }
  free(hist); free(seen); free(win); free(pat);
  return 0;
}

/* ---------------------------------------------------------------- derived
 * LU decomposition analysis (Evaluation section): the parallelism spokes of
 * the radar diagram are inverses of collected metrics -- granularity =
 * 1 / work-items, barriers per instruction = 1 / mean ITB, instructions per
 * operand = 1 / (summed SIMD widths) -- and load imbalance = max IPT - min
 * IPT.  Reading: "summed SIMD widths" is taken per instruction, i.e. the
 * mean SIMD width, so instructions per operand = instructions / S1 (the
 * ratio the name states, in (0, 1] like its sibling spokes).  Mean ITB =
 * (sum of ITB values) / (number of ITB values), so its inverse is the single
 * division count / sum.  Divisions by zero follow IEEE (x/0 = inf, 0/0 =
 * NaN), as the other ratios of the result do.                              */
static void derived_metrics(orc_result *r) {
  r->granularity = 1.0 / (double)r->work_items;
  r->barriers_per_instruction = (double)r->itb_count / (double)r->itb_sum;
  r->instructions_per_operand = (double)r->total_instructions / (double)r->simd_sum;
  r->load_imbalance = r->ipt_max - r->ipt_min;
}

static int check_trace(const orc_trace *t) {
  if (!t || t->history_len < 1 || t->history_len > 32) return 1;
  if (t->n_events && (!t->opcode || !t->table)) return 1;
  if (!t->wi_offsets) return 1;
  if (t->wi_offsets[0] != 0 || t->wi_offsets[t->n_wi] != t->n_events) return 1;
  for (uint64_t w = 0; w < t->n_wi; ++w)
    if (t->wi_offsets[w + 1] < t->wi_offsets[w]) return 1;
  for (uint64_t e = 0; e < t->n_events; ++e)
    if (t->opcode[e] >= t->n_ids) return 1;
  if (t->n_mem && (!t->addr || !t->mem_kind)) return 1;
  if (t->n_branch && (!t->br_site || !t->br_taken || !t->n_sites)) return 1;
  for (uint64_t i = 0; i < t->n_branch; ++i)
    if (t->br_site[i] >= t->n_sites || t->br_taken[i] > 1) return 1;
  return 0;
}

int orc_characterize(const orc_trace *t, orc_result *out) {
  if (!out || check_trace(t)) return 1;
  orc_result r;
  memset(&r, 0, sizeof r);
  int rc = compute_metrics(t, &r);
  if (!rc) rc = parallel_metrics(t, &r);
  if (!rc) rc = space_metrics(t, 0, &r.space[0]);
  if (!rc) rc = space_metrics(t, 1, &r.space[1]);
  if (!rc) rc = branch_metrics(t, &r);
  if (!rc) derived_metrics(&r);
  if (!rc) *out = r;
  return rc;
}

/* Whether the opcode kinds announce exactly the memory and branch events the
 * trace carries.  The plugin interface of the Implementation section has
 * separate callbacks for plain loads and stores and for the load and the
 * store of an atomic; reading: an atomic read-modify-write instruction is
 * one instruction with two memory events, a read and a write of one
 * address.  So #LOAD + #STORE + 2 #ATOMIC must equal the memory events and
 * #BRANCH_COND the branch events.  1 = consistent, 0 = not, -1 = invalid.  */
int orc_kinds_consistent(const orc_trace *t) {
  if (check_trace(t)) return -1;
  uint64_t loads = 0, stores = 0, atomics = 0, branches = 0;
  for (uint64_t e = 0; e < t->n_events; ++e) {
    switch (t->table[t->opcode[e]].kind) {
      case K_LOAD: ++loads; break;
      case K_STORE: ++stores; break;
      case K_ATOMIC: ++atomics; break;
      case K_BRANCH: ++branches; break;
      default: break;
    }
  }
  return (loads + stores + 2 * atomics == t->n_mem && branches == t->n_branch) ? 1 : 0;
}

int orc_class_hist(const orc_trace *t, uint64_t *out, size_t len) {
  if (!out || check_trace(t)) return 1;
  memset(out, 0, len * sizeof(uint64_t));
  for (uint64_t e = 0; e < t->n_events; ++e) {
    uint16_t c = t->table[t->opcode[e]].op_class;
    if (c < len) out[c]++;
  }
  return 0;
}

int orc_spectrum(const orc_trace *t, int space, int k, uint64_t *f, uint64_t *mf,
                 size_t cap, size_t *n_out) {
  if (!n_out || check_trace(t) || k < 0 || k > 10 || space < 0 || space > 1) return 1;
  size_t n;
  uint64_t *a = gather(t, space, 0, &n);
  uint64_t *c = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!a || !c) { free(a); free(c); return 2; }
  qsort(a, n, sizeof(uint64_t), cmp_u64);
  size_t runs = 0, i = 0;
  while (i < n) {
    size_t j = i + 1;
    while (j < n && (a[j] >> k) == (a[i] >> k)) ++j;
    c[runs++] = (uint64_t)(j - i);
    i = j;
  }
  qsort(c, runs, sizeof(uint64_t), cmp_u64);
  size_t np = 0;
  i = 0;
  while (i < runs) {
    size_t j = i + 1;
    while (j < runs && c[j] == c[i]) ++j;
    if (np < cap) { f[np] = c[i]; mf[np] = (uint64_t)(j - i); }
    ++np;
    i = j;
  }
  *n_out = np;
  free(a); free(c);
  return 0;
}
