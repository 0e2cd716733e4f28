/*
 * aiwc.h -- C ABI of libaiwc, an MI355X (gfx950) implementation of the
 * data-parallel reduction at the heart of AIWC (Architecture-Independent
 * Workload Characterization, Johnston & Milthorpe, arXiv 1805.04207).
 *
 * A *trace* is the stream of events that an interpreted OpenCL kernel emits
 * to the AIWC plugin (paper, Section "Implementation": instructionExecuted,
 * workItemBegin, memoryLoad/Store/AtomicLoad/AtomicStore, barrier events).
 * libaiwc takes that stream as structure-of-arrays already resident in HBM
 * and reduces it, entirely in HIP kernels, to the metrics of the paper's
 * Table I ("Metrics collected by the AIWC tool ordered by type").
 *
 * Conventions for every entry point:
 *   - Every call returns an aiwc_status.  On anything but AIWC_OK no
 *     out-parameter is written; aiwc_last_error(ctx) holds a message.
 *   - "device pointer" = memory allocated on the context's HIP device
 *     (hipMalloc, a torch CUDA tensor, ...).  It is BORROWED: the caller keeps
 *     it alive and unmodified until the work that reads it has completed
 *     (aiwc_metrics_read returned, or the stream was synchronized).
 *   - "host pointer" = ordinary process memory; it is read (copied) during the
 *     call and may be released when the call returns.
 *   - A stream argument is a hipStream_t passed as void*; NULL = the null stream.
 *   - One context per host thread.  Traces and metrics belong to the context
 *     that created them and must not outlive it.
 */
#ifndef AIWC_H
#define AIWC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef enum aiwc_status {
  AIWC_OK = 0,
  AIWC_ERR_INVALID_ARG = 1,   /* bad pointer, size, flag, or trace content   */
  AIWC_ERR_INCONSISTENT = 2,  /* opcode kinds disagree with stream lengths   */
  AIWC_ERR_OUT_OF_MEMORY = 3, /* device allocation failed / over the cap     */
  AIWC_ERR_HIP = 4,           /* a HIP runtime call failed                   */
  AIWC_ERR_UNSUPPORTED = 5    /* valid request this build does not handle    */
} aiwc_status;

/* ------------------------------------------------------------- opcode kinds
 * The role an opcode plays in the event stream.  COMPUTE/OTHER only feed the
 * opcode and SIMD metrics; LOAD/STORE/ATOMIC_RMW announce memory events;
 * BRANCH_COND announces one branch event; BARRIER closes an
 * instructions-to-barrier segment (Table I, Parallelism rows).              */
enum {
  AIWC_KIND_COMPUTE = 0,
  AIWC_KIND_LOAD = 1,
  AIWC_KIND_STORE = 2,
  AIWC_KIND_ATOMIC_RMW = 3,  /* one instruction = a read and a write event  */
  AIWC_KIND_BRANCH_COND = 4,
  AIWC_KIND_BARRIER = 5,
  AIWC_KIND_OTHER = 6
};

/* mem_kind bits of one memory event.  Bit 0: the event is a write (store, or
 * the store half of an atomic).  Bit 1: the address is in the local (work-group
 * shared) address space; clear = global.  All other bits must be zero.      */
enum { AIWC_MEM_WRITE = 1u, AIWC_MEM_LOCAL = 2u };

/* Per-opcode-id description, indexed by the u16 opcode id of the stream.
 * op_class groups ids into the "unique opcodes" of Table I: the paper counts
 * LLVM opcode *names* (Implementation section, opcode map), so ids that are
 * width variants of one name share a class.  simd_width is the number of
 * data items the instruction's result holds (Implementation section, SIMD
 * paragraph); scalar and void results use 1.                               */
typedef struct aiwc_opcode_info {
  uint16_t op_class;   /* < 65535                                           */
  uint8_t simd_width;  /* >= 1                                              */
  uint8_t kind;        /* AIWC_KIND_*                                       */
} aiwc_opcode_info;

/* trace flags */
enum {
  AIWC_VALIDATE_ON_DEVICE = 1u, /* aiwc_trace_create runs a validation kernel
                                   over every array and synchronizes        */
  /* Branch-entropy variants.  The paper fixes the history length (16) but
   * not the history's scope or start-up, and it cites two entropies
   * (Related Work: Yokota's branch history entropy, De Pestel's linear
   * entropy).  Default: each site keeps its own history of its previous m
   * outcomes, and an execution forms a window once m earlier outcomes of its
   * site exist.                                                            */
  AIWC_BRANCH_ZERO_HISTORY = 2u,    /* histories start as m not-taken outcomes;
                                       every execution forms a window       */
  AIWC_BRANCH_GLOBAL_HISTORY = 4u,  /* one history of the previous m outcomes
                                       of all branches in stream order (the
                                       "combined" history of the
                                       Implementation section), keyed with
                                       the site; needs history_len <= 31    */
  AIWC_BRANCH_PATTERN_ENTROPY = 8u  /* also report pattern_entropy; needs
                                       history_len <= 20                    */
};

/* One kernel launch's event trace (structure of arrays).
 *
 *   opcode[n_events]          device, u16 ids; work-item w's instructions are
 *                             opcode[wi_offsets[w] .. wi_offsets[w+1]) in
 *                             execution order.
 *   wi_offsets[n_workitems+1] device, non-decreasing, [0] = 0,
 *                             [n_workitems] = n_events.
 *   addr[n_mem], mem_kind[n_mem]
 *                             device; the byte address of each memory event
 *                             (its start address) and AIWC_MEM_* bits.  Order
 *                             is free: memory metrics are order independent.
 *                             addr == UINT64_MAX is reserved (rejected).
 *   br_site[n_branch], br_taken[n_branch]
 *                             device; each conditional-branch event's static
 *                             site id (< n_sites) and outcome (0/1), in the
 *                             order the branches executed.  Only the relative
 *                             order of events of the same site matters.
 *   opcode_table[n_opcode_ids] HOST; copied at create time.
 *   history_len               branch history length m, 1..32 (the paper fixes
 *                             16: Metrics section, branch paragraph).
 *   max_lsb_skip              must be 10 (skips 0..10: Table I memory entropy
 *                             rows and the LMAE paragraph of Metrics).
 * Per-trace limits: n_mem < 2^32, n_branch < 2^32, n_sites < 2^31.          */
typedef struct aiwc_trace_desc {
  uint32_t struct_size;   /* = sizeof(aiwc_trace_desc)                       */
  uint32_t flags;         /* AIWC_VALIDATE_ON_DEVICE, ...                    */
  uint64_t n_events;
  const uint16_t *opcode;
  uint64_t n_workitems;
  const uint64_t *wi_offsets;
  uint32_t wg_size;       /* work-group size (informational, sizing feature) */
  uint32_t n_opcode_ids;
  const aiwc_opcode_info *opcode_table;
  uint64_t n_mem;
  const uint64_t *addr;
  const uint8_t *mem_kind;
  uint64_t n_branch;
  const uint32_t *br_site;
  const uint8_t *br_taken;
  uint32_t n_sites;
  uint32_t history_len;
  uint32_t max_lsb_skip;
  uint32_t reserved;
} aiwc_trace_desc;

#define AIWC_NSKIP 11        /* LSB skips 0..10                            */
#define AIWC_SPACE_GLOBAL 0
#define AIWC_SPACE_LOCAL 1

/* Memory metrics of one address space (Table I, Memory rows).  The paper's
 * named scalars refer to the global space; the same set is reported for the
 * local space.  distinct[k] / entropy[k] are taken over the addresses with
 * their k least significant bits dropped (a >> k): k = 0 is the global
 * memory address entropy, k = 1..10 the local (spatial-locality) entropy
 * curve of the Metrics section.  Entropy is Shannon's, base 2, plug-in.    */
typedef struct aiwc_space_metrics {
  uint64_t total_accesses;          /* reads + writes                        */
  uint64_t total_reads;
  uint64_t total_writes;
  uint64_t unique_reads;            /* distinct addresses read               */
  uint64_t unique_writes;           /* distinct addresses written            */
  uint64_t footprint;               /* distinct addresses (= distinct[0])    */
  uint64_t footprint_90;            /* fewest addresses covering 90% of
                                       accesses, most-accessed first          */
  uint64_t distinct[AIWC_NSKIP];
  double entropy[AIWC_NSKIP];
  double unique_rw_ratio;           /* unique_reads / unique_writes          */
  double reread_ratio;              /* unique_reads / total_reads            */
  double rewrite_ratio;             /* unique_writes / total_writes          */
} aiwc_space_metrics;

/* All metrics of one trace.  Ratios are IEEE double divisions of the exact
 * integers (x/0 = +inf, 0/0 = NaN).  Medians of an even count are the mean
 * of the two middle values.                                                 */
typedef struct aiwc_metrics_host {
  uint32_t struct_size;             /* filled by aiwc_metrics_read           */
  uint32_t history_len;
  /* compute (Table I, Compute rows) */
  uint64_t total_instructions;
  uint32_t unique_opcodes;          /* classes executed at least once        */
  uint32_t opcodes_90;              /* fewest classes covering 90% of
                                       dynamic instructions                  */
  uint64_t simd_max;
  uint64_t simd_sum;                /* S1 = sum of widths (exact)            */
  uint64_t simd_sumsq_lo;           /* S2 = sum of squared widths, 128-bit   */
  uint64_t simd_sumsq_hi;
  double simd_mean;                 /* S1 / N                                */
  double simd_sd;                   /* population SD = sqrt(N*S2 - S1^2) / N */
  /* parallelism (Table I, Parallelism rows) */
  uint64_t work_items;
  uint64_t barriers_hit;            /* explicit barrier events               */
  uint64_t itb_count;               /* segments = barriers_hit + work_items  */
  uint64_t itb_sum;                 /* = total_instructions                  */
  uint64_t itb_min, itb_max;
  double itb_median;
  uint64_t ipt_min, ipt_max;
  double ipt_median;
  /* memory */
  aiwc_space_metrics space[2];      /* [AIWC_SPACE_GLOBAL], [AIWC_SPACE_LOCAL] */
  /* control (Table I, Control rows) */
  uint64_t total_branches;
  uint64_t unique_branches;         /* sites executed at least once          */
  uint64_t branches_90;             /* fewest sites covering 90% of branches */
  uint64_t n_windows;               /* history windows: sum_s max(0, n_s - m) */
  uint64_t albe_min_sum;            /* sum over (site, history) of min(n0,n1) */
  double yokota_entropy;            /* H(outcome | site, history), in [0,1]  */
  double linear_branch_entropy;     /* 2 * albe_min_sum / n_windows          */
  double pattern_entropy;           /* with AIWC_BRANCH_PATTERN_ENTROPY:
                                       Yokota's branch history entropy in its
                                       pattern form, E_m / m in [0,1], where
                                       E_m = sum_p c_p log2(N_w / c_p) over
                                       the m-bit histories p of the windows
                                       (any site); 0 when N_w = 0.  NaN when
                                       not requested.                        */
  /* derived parallelism metrics (LU decomposition analysis of the paper:
     the inverted values plotted on the radar diagram, and load imbalance);
     each is one IEEE operation on the exact integers above               */
  double granularity;               /* 1 / work_items                        */
  double barriers_per_instruction;  /* 1 / mean ITB = itb_count / itb_sum    */
  double instructions_per_operand;  /* total_instructions / simd_sum, i.e.
                                       1 / mean SIMD width                   */
  uint64_t load_imbalance;          /* ipt_max - ipt_min                     */
  /* bookkeeping */
  uint32_t overflow_redos;          /* on-chip table overflows redone        */
  uint32_t partitions;              /* memory partitions used (both spaces)  */
} aiwc_metrics_host;

typedef struct aiwc_ctx aiwc_ctx;
typedef struct aiwc_trace aiwc_trace;
typedef struct aiwc_metrics aiwc_metrics;

/* --------------------------------------------------------------- contexts */

/* Create a context on HIP device `hip_device`.  Owns scratch memory, the
 * tuning cache and the sizing network.  Errors: INVALID_ARG (null out, bad
 * device), HIP.                                                            */
aiwc_status aiwc_context_create(int hip_device, aiwc_ctx **out);
/* Destroy a context; waits for its outstanding work.  NULL is a no-op.     */
aiwc_status aiwc_context_destroy(aiwc_ctx *ctx);
/* Last error message of the context ("" if none).  Never NULL.  Valid until
 * the next call on the context.  ctx may be NULL (then: messages of calls
 * that had no context).                                                     */
const char *aiwc_last_error(const aiwc_ctx *ctx);

/* ----------------------------------------------------------------- traces */

/* Describe a trace.  Checks the descriptor on the host (null pointers with
 * non-zero sizes, history_len in 1..32, max_lsb_skip == 10, n_sites >= 1 when
 * n_branch > 0, limits above, opcode table entries) and copies opcode_table
 * to the device.  With AIWC_VALIDATE_ON_DEVICE it also checks the arrays
 * (offsets non-decreasing with [0] = 0 and [n_workitems] = n_events;
 * mem_kind bits; br_taken in {0,1}; br_site < n_sites; addr != UINT64_MAX;
 * opcode ids < n_opcode_ids) and returns INVALID_ARG on the first violation
 * class found, or INCONSISTENT when #LOAD + #STORE + 2 #ATOMIC_RMW != n_mem
 * or #BRANCH_COND != n_branch.  Without the flag those content errors are
 * the caller's responsibility (the consistency check still runs at
 * characterize time).                                                       */
aiwc_status aiwc_trace_create(aiwc_ctx *ctx, const aiwc_trace_desc *desc,
                              aiwc_trace **out);
aiwc_status aiwc_trace_destroy(aiwc_trace *trace);

/* ----------------------------------------------------------- characterize */

/* Enqueue the full reduction of one trace on `stream` (the paper's kernelEnd
 * statistics, Implementation section) and return a metrics handle at once.
 * All arithmetic runs in HIP kernels; nothing is copied to the host until
 * aiwc_metrics_read.  On-chip table overflow is never an error: the kernels
 * redo the affected partition with more rounds (results stay exact).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.                                   */
aiwc_status aiwc_characterize(aiwc_ctx *ctx, const aiwc_trace *trace,
                              void *stream, aiwc_metrics **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * aiwc_characterize without any allocation.  The scratch buffers of every
 * stage (partition records, radix buffers, histograms, accumulators) live in
 * one statically allocated device array of AIWC_STATIC_SCRATCH_BYTES per GPU,
 * held from the library's first context on that GPU until the process ends;
 * the result goes to a caller-owned device block.  The call enqueues the
 * kernels on `stream` (single-stream order) and returns; it calls no
 * hipMalloc / hipFree, creates no event or stream and copies nothing to the
 * host.
 *   dev_result   device pointer, result_bytes long, written by the kernels:
 *                offset 0: aiwc_metrics_host; right after it four uint64
 *                status words: [0] != 0 trace content invalid (the
 *                INVALID_ARG case of aiwc_metrics_read), [1] != 0 kinds
 *                inconsistent with the stream lengths (INCONSISTENT),
 *                [2] spectrum pair counts (not exported here), [3] != 0 an
 *                on-chip round could not be split (UNSUPPORTED); the metrics
 *                are valid only when words 0, 1 and 3 are 0.  At offset
 *                AIWC_STATIC_CLASS_OFFSET: the per-class instruction counts,
 *                uint64[n_classes] with n_classes = 1 + the largest op_class
 *                of the opcode table.  result_bytes must be at least
 *                AIWC_STATIC_RESULT_BYTES(n_classes).
 * Every call on one GPU uses that GPU's one scratch array: calls that
 * overlap on a GPU (other streams, other host threads, other contexts of the
 * process) race and must be serialized by the caller (same stream, or
 * events).  The array keeps the last call's contents; each call clears what
 * it needs zeroed with a kernel.  Limit: traces whose plan needs more than
 * AIWC_STATIC_SCRATCH_BYTES of scratch return UNSUPPORTED before anything
 * is enqueued; use aiwc_characterize for those.  The plan takes 12 B per
 * memory event (partition record and page tag), 8 B more from 2^18 memory
 * events or from 2^12 partitions on (one buffer: the two-level scatter's
 * coarse buckets and the hot partitions' remaining records) with 2.1 MiB of
 * hot-page tables from 2^18 memory events, per-block partition histograms,
 * 8.25 B per branch event (radix buffers and digit counts), 512 KiB per
 * 65536 branch events for hot-site tables (history 16) and ~1.2 MiB of
 * fixed tables: at the 30% memory / 5% branch mix about 3 MiB for 5e5
 * events, 9.4 MiB for 1e6, 48 MiB for 6.7e6, 63.5 MiB for 8.9e6 events
 * (2.7e6 memory events), the largest that fit.
 * Errors: INVALID_ARG (null, foreign trace, result_bytes too small),
 * UNSUPPORTED (over the limit), HIP (launch failure, or the array's address
 * could not be found at context creation).                                  */
#define AIWC_STATIC_SCRATCH_BYTES (64ull << 20)
#define AIWC_STATIC_CLASS_OFFSET ((sizeof(aiwc_metrics_host) + 32 + 255) / 256 * 256)
#define AIWC_STATIC_RESULT_BYTES(n_classes) (AIWC_STATIC_CLASS_OFFSET + 8 * (size_t)(n_classes))
aiwc_status aiwc_characterize_static(aiwc_ctx *ctx, const aiwc_trace *trace, void *stream,
                                     void *dev_result, size_t result_bytes);

/* Metrics of several invocations of one kernel taken together (the paper
 * reports each kernel as the aggregate over all its invocations at a problem
 * size: Evaluation section).  The result is, by definition, that of the one
 * trace formed by concatenating the invocations in the order given: their
 * work-items and instruction streams, memory streams and branch streams.  So
 * counts add up, distinct counts are those of the union of the addresses
 * (an address touched by two invocations counts once, with its accesses
 * summed), entropies and footprints are over the pooled accesses, ITB and
 * IPT statistics over the pooled segments and work-items, and a branch
 * site's history runs on from one invocation into the next.
 *   traces[n]   n >= 1 handles of this context, all with the same opcode
 *               table and history_len.  n_sites of the result is the largest
 *               of theirs.  The summed n_mem and n_branch must stay < 2^32.
 * The concatenation is staged in device memory owned by the returned handle
 * (about 2 B per event + 9 B per memory event + 5 B per branch event + 8 B
 * per work-item), released by aiwc_metrics_destroy.  With n == 1 it is
 * aiwc_characterize.  Errors: INVALID_ARG (null, empty list, foreign handle,
 * tables or history lengths differ, sums over the limits), OUT_OF_MEMORY,
 * HIP.                                                                      */
aiwc_status aiwc_characterize_merged(aiwc_ctx *ctx, const aiwc_trace *const *traces,
                                     size_t n, void *stream, aiwc_metrics **out);

/* ---------------------------------------------------------- streaming
 * A trace that arrives in chunks.  The paper names the memory footprint of
 * full recorded traces as its tool's main limit on large applications
 * (Conclusions; Evaluation: kernels it could not characterize at large
 * sizes).  A chunk is a trace handle holding a run of whole work-items with
 * the memory and branch events they issued, in order.  The result of
 * aiwc_stream_finish is, exactly, that of aiwc_characterize on the
 * concatenation of the chunks (the aggregate of aiwc_characterize_merged).
 * On append, a chunk's instruction stream is reduced into the stream's
 * state (opcodes and work-item offsets are not kept); its memory and branch
 * streams are copied into device buffers the stream owns (9 B per memory
 * event, 5 B per branch event), which finish reduces with the ordinary
 * memory and branch stages.                                                 */
typedef struct aiwc_stream aiwc_stream;
/* stream flags */
enum {
  AIWC_STREAM_HOST_RETAIN = 1u  /* keep the retained memory and branch streams
                                   in pinned host memory until finish (the
                                   paper's remedy for the footprint: keep
                                   the recorded traces out of the working
                                   memory); finish copies them to the device
                                   once.  Appends then hold only the
                                   instruction-stream state on the device.  */
};
/* An empty stream of this context.  mem_hint / branch_hint: expected total
 * memory and branch events (0 = unknown); the retained buffers are reserved
 * for them up front and otherwise grow by doubling (each move copies what
 * is held and synchronizes the stream).  flags: AIWC_STREAM_*.
 * Errors: INVALID_ARG (null, unknown flags), OUT_OF_MEMORY.                 */
aiwc_status aiwc_stream_create(aiwc_ctx *ctx, uint64_t mem_hint, uint64_t branch_hint,
                               uint32_t flags, aiwc_stream **out);
/* Append one chunk, a trace handle of the stream's context.  The first
 * chunk fixes the opcode table, history_len and branch flags; later chunks
 * must match.  Asynchronous on `stream`: the chunk's device arrays are read
 * by work enqueued there, so keep them until that work completes (the chunk
 * handle itself may be destroyed at once).  Errors: INVALID_ARG (null,
 * foreign handle, mismatch, finished stream, summed n_mem or n_branch
 * reaching 2^32), OUT_OF_MEMORY, HIP.                                       */
aiwc_status aiwc_stream_append(aiwc_stream *st, const aiwc_trace *chunk, void *stream);
/* Reduce everything appended and return its metrics handle (as
 * aiwc_characterize does); the stream then takes no more chunks.  Call it on
 * the stream the appends used (or synchronize that stream first): the
 * retained copies are ordered only on it.  The
 * stream must outlive the returned handle's work (aiwc_stream_destroy
 * waits for the device).  Errors: INVALID_ARG (null, nothing appended,
 * already finished), OUT_OF_MEMORY, HIP.                                    */
aiwc_status aiwc_stream_finish(aiwc_stream *st, void *stream, aiwc_metrics **out);
/* Out-of-core memory stage.  Caps the device memory that finish may use for
 * the partitioned memory records (12 B per record: the 8-byte partition
 * record and its 4-byte page tag); 0 = no cap (default).  When the retained
 * memory stream holds more records than the cap allows, finish reduces it
 * one group of partitions at a time: a first sweep over the retained stream
 * counts every partition's records (and each space's reads and writes),
 * then each group sweeps the stream again, keeps only its partitions'
 * records and runs the bucket stage on them.  Partitions hold disjoint 1 KiB
 * pages, so the groups' integer sums are exactly the whole's; the result is
 * identical to the single pass.  With AIWC_STREAM_HOST_RETAIN the sweeps
 * move the retained stream from pinned host memory in chunks of at most
 * 2^22 records, so the device never holds the whole memory stream.  A
 * single partition larger than the cap is reduced alone (the cap is then
 * exceeded by it).  The branch stream is still reduced in one pass.
 * Errors: INVALID_ARG (null, finished stream).                              */
aiwc_status aiwc_stream_set_device_budget(aiwc_stream *st, uint64_t bytes);
typedef struct aiwc_stream_stats {
  uint32_t struct_size;         /* = sizeof(aiwc_stream_stats)               */
  uint32_t groups;              /* partition groups of the last finish (1:
                                   one pass over the whole memory stream)   */
  uint64_t memory_events;       /* retained memory events                    */
  uint64_t device_records;      /* partition records the device held at once */
  uint64_t largest_partition;   /* records of the largest partition         */
} aiwc_stream_stats;
/* Sizes of the last finish of the stream (host struct).  Errors:
 * INVALID_ARG (null, struct_size mismatch, not finished).                   */
aiwc_status aiwc_stream_get_stats(const aiwc_stream *st, aiwc_stream_stats *out);
/* Release the stream's buffers (waits for the device).  NULL is a no-op. */
aiwc_status aiwc_stream_destroy(aiwc_stream *st);

/* Sizing policy for the memory partitions and on-chip tables.             */
typedef enum aiwc_sizing {
  AIWC_SIZING_BOUND = 0,      /* distinct <= accesses: never undersized     */
  AIWC_SIZING_HEURISTIC = 1,  /* extrapolate distinct counts of a prefix    */
  AIWC_SIZING_LEARNED = 2     /* the context's sizing network (MLP)        */
} aiwc_sizing;

typedef enum aiwc_autotune {
  AIWC_AUTOTUNE_OFF = 0,      /* built-in launch shapes                     */
  AIWC_AUTOTUNE_CACHED = 1,   /* use the tuning cache, defaults on a miss   */
  AIWC_AUTOTUNE_SEARCH = 2    /* time candidates on a miss, then cache      */
} aiwc_autotune;

typedef struct aiwc_batch_opts {
  uint32_t struct_size;             /* = sizeof(aiwc_batch_opts)             */
  uint32_t sizing;                  /* aiwc_sizing                           */
  uint32_t autotune;                /* aiwc_autotune                         */
  uint32_t use_graph;               /* capture the batch in a hipGraph       */
  uint64_t admission_cap_bytes;     /* scratch budget per wave; 0 = 200 GiB  */
  uint32_t force_partition_log2;    /* debug: force global partitions 2^x
                                       (undersize => redo path), 0 = off     */
  uint32_t reserved;
} aiwc_batch_opts;

/* Characterize n traces as one batch: the traces are bin-packed into waves
 * whose scratch fits admission_cap_bytes, and each wave's stages run as
 * batch-wide persistent launches over a longest-first work list (optionally
 * replayed from a captured hipGraph).  out[i] receives trace i's metrics.
 * Results are bit-identical to aiwc_characterize on each trace.
 * Errors: INVALID_ARG, OUT_OF_MEMORY (one trace alone exceeds the cap), HIP. */
aiwc_status aiwc_characterize_batch(aiwc_ctx *ctx,
                                    const aiwc_trace *const *traces, size_t n,
                                    const aiwc_batch_opts *opts, void *stream,
                                    aiwc_metrics **out);

/* Statistics of the last aiwc_characterize_batch call of the context.     */
typedef struct aiwc_batch_stats {
  uint32_t struct_size;
  uint32_t waves;                   /* admission waves launched              */
  uint64_t reserved_bytes;          /* peak scratch reserved by a wave       */
  uint64_t redo_partitions;         /* partitions redone after overflow      */
  uint64_t total_partitions;
  double plan_ms;                   /* host planning time                    */
} aiwc_batch_stats;
aiwc_status aiwc_batch_last_stats(const aiwc_ctx *ctx, aiwc_batch_stats *out);

/* Wait for the metrics' work and copy the result to the host (one D2H copy).
 * Errors: INVALID_ARG (null, or trace content found invalid on the device:
 * opcode ids >= n_opcode_ids, sites >= n_sites, outcomes > 1),
 * INCONSISTENT (see aiwc_trace_create), UNSUPPORTED (an internal capacity
 * limit: an on-chip table round could not be split further by hash bits, so
 * the metrics would be incomplete; not a fault of the trace), HIP.          */
aiwc_status aiwc_metrics_read(aiwc_metrics *m, aiwc_metrics_host *out);
/* Per-class instruction counts (index = op_class), len entries (host).     */
aiwc_status aiwc_metrics_class_hist(aiwc_metrics *m, uint64_t *out, size_t len);
/* Count-of-counts spectrum of one space at LSB skip 0: pairs (f, m_f) =
 * "m_f distinct addresses were accessed exactly f times", ascending f.
 * Writes at most cap pairs (host arrays) and the total number of pairs to
 * *n_out.                                                                   */
aiwc_status aiwc_metrics_spectrum(aiwc_metrics *m, int space, uint64_t *f,
                                  uint64_t *mf, size_t cap, size_t *n_out);
aiwc_status aiwc_metrics_destroy(aiwc_metrics *m);

/* ---------------------------------------------------------- instrumentation
 * When enabled, every characterization records a hipEvent on its stream after
 * each kernel launch.  aiwc_profile_read waits for the last one and returns,
 * for the most recent characterization of the context, the per-kernel
 * durations in milliseconds (ms[i] = time from the previous mark to mark i)
 * and their kernel names as one comma-separated string (host buffers).      */
aiwc_status aiwc_profile_enable(aiwc_ctx *ctx, int on);
aiwc_status aiwc_profile_read(aiwc_ctx *ctx, char *names, size_t names_cap,
                              double *ms, size_t max_stages, size_t *n_out);

/* ----------------------------------------------------- learned sizing (MLP)
 * A 40 -> 64 -> 64 -> 64 -> 11 perceptron (exact-erf GELU, bf16 weights,
 * fp32 accumulation) predicts log2 of the global-space distinct counts at
 * skips 0..10 from 40 features of the trace's first 8,192 memory events
 * (exact prefix distinct counts per space and skip, the growth of the
 * distinct count over the prefix, spans, alignment and locality fractions,
 * and the trace's sizes).  The predictions size the memory partitions;
 * overflow is redone, so results never depend on them.  A trace of more
 * than 2^27 memory events gets the most partitions from its record count
 * alone; batched sizing computes no features for it.
 */
#define AIWC_N_FEATURES 40
#define AIWC_N_TARGETS 11
#define AIWC_MLP_HIDDEN 64

/* Features of n traces into dev_out[n][40] (device, fp32, raw = not yet
 * normalized).                                                              */
aiwc_status aiwc_sizer_features(aiwc_ctx *ctx, const aiwc_trace *const *traces,
                                size_t n, void *stream, float *dev_out);

typedef struct aiwc_train_opts {
  uint32_t struct_size;
  uint32_t epochs;
  uint32_t batch;
  uint32_t seed;
  float lr;
  float beta1, beta2, eps;
  uint32_t reserved;
} aiwc_train_opts;

/* Train the context's network on (dev_x[n][40] raw features, dev_y[n][11]
 * log2 targets), device fp32.  Feature/target normalization statistics are
 * taken from this training set.  *loss_out (host, nullable) receives the
 * final epoch's mean squared error (normalized units).                      */
aiwc_status aiwc_sizer_train(aiwc_ctx *ctx, const float *dev_x,
                             const float *dev_y, size_t n,
                             const aiwc_train_opts *opts, void *stream,
                             float *loss_out);
/* Predict log2 distinct counts dev_y[n][11] from raw features dev_x[n][40]. */
aiwc_status aiwc_sizer_predict(aiwc_ctx *ctx, const float *dev_x, size_t n,
                               void *stream, float *dev_y);
/* One forward + backward pass on normalized inputs (device fp32
 * dev_xn[n][40], dev_yn[n][11]) with the current weights; writes the mean
 * squared error to *loss (host) and the gradients of every parameter, in
 * aiwc_sizer_get_params order, to host_grad (fp32, count from
 * aiwc_sizer_num_params).                                                   */
aiwc_status aiwc_sizer_grad(aiwc_ctx *ctx, const float *dev_xn,
                            const float *dev_yn, size_t n, void *stream,
                            float *loss, float *host_grad);
size_t aiwc_sizer_num_params(void);
/* Parameters as fp32 values of the bf16 weights: W1[64][40], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[11][64], b4[11]; then the
 * normalization: x_mean[40], x_std[40], y_mean[11], y_std[11].  set_params
 * rounds weights to bf16 (nearest-even).                                   */
aiwc_status aiwc_sizer_get_params(const aiwc_ctx *ctx, float *host_params);
aiwc_status aiwc_sizer_set_params(aiwc_ctx *ctx, const float *host_params);
aiwc_status aiwc_sizer_save(const aiwc_ctx *ctx, const char *path);
aiwc_status aiwc_sizer_load(aiwc_ctx *ctx, const char *path);
/* Margin (in log2 units) added to predictions before sizing.               */
aiwc_status aiwc_sizer_set_margin(aiwc_ctx *ctx, float margin_log2);

/* ----------------------------------------------------------- trace producer
 * Produces the event arrays of one kernel launch by executing the kernel on
 * the GPU.  The paper obtains its trace by interpreting a kernel's LLVM IR in
 * a simulator that notifies a plugin of every executed instruction, memory
 * access and branch outcome (Implementation section; Methodology, the SPIR
 * paragraph).  Here a kernel is a program of aiwc_insn records (a register
 * machine whose operations carry LLVM's opcode names) that libaiwc
 * interprets with one GPU thread per work-item and one workgroup per
 * work-group, recording the same events:
 *   - every executed instruction appends its opcode id to its work-item's
 *     opcode stream (the instructionExecuted notification);
 *   - LOAD / STORE append one memory event at the access's start address,
 *     ATOMIC a read and then a write event (memoryLoad, memoryStore,
 *     memoryAtomicLoad, memoryAtomicStore);
 *   - BR appends one branch event (site, 1 if the condition held);
 *   - BARRIER ends an instructions-to-barrier segment (its opcode table
 *     entry has AIWC_KIND_BARRIER).
 * Event order follows the paper's schedule: work-groups one after another,
 * and inside a work-group each work-item runs until it reaches a barrier or
 * returns before the next work-item runs.  So the branch stream is ordered
 * by (work-group, barrier interval, local id, execution order).  The opcode
 * stream is work-item major (work-item w = group_linear * wg_size +
 * local_linear), and so are the memory events (their order is free).
 *
 * Machine model.
 *   - AIWC_NREG registers of 64 bits per work-item, zero at start except
 *     r0..r(n_args-1), which hold the kernel arguments.
 *   - Integer operations work on all 64 bits (two's complement; shift counts
 *     taken mod 64; division or remainder by zero gives 0, and so does
 *     INT64_MIN / -1 for its remainder, INT64_MIN for its quotient).
 *   - F-operations work on the binary32 value in the low 32 bits, round to
 *     nearest even, keep subnormals, and write the result's bits
 *     zero-extended; a NaN result is written as 0x7FC00000.  FMIN / FMAX
 *     return the other operand when one is NaN and order -0 below +0.
 *   - width w > 1 applies an operation to w consecutive registers of each
 *     register operand (an immediate operand is shared); a register range of
 *     d must equal or not overlap those of a, b and c.
 *   - Addresses: global argument j (counting global arguments only) is the
 *     buffer whose address is (j + 1) << AIWC_ADDR_TAG_SHIFT; local
 *     arguments are laid out in order, each 16-byte aligned, in the
 *     work-group's local memory, whose addresses are offsets from 0 (tag 0).
 *     The trace records these addresses (global events clear
 *     AIWC_MEM_LOCAL, local events set it).  Local memory starts zeroed in
 *     every work-group.
 *   - An access must lie inside its buffer and be aligned to its element
 *     size; otherwise the launch fails (AIWC_ERR_INVALID_ARG) without doing
 *     the access.
 *
 * Operations (d, a, b, c are registers; "b" is imm instead when
 * flags & AIWC_INSN_IMM_B; LLVM names in brackets are what the opcode table
 * normally gives the id):
 *   RET                      the work-item ends                       [ret]
 *   MOV      d = b                                                    [phi]
 *   ADD SUB MUL SDIV SREM UDIV UREM SHL LSHR ASHR AND OR XOR
 *            d = a op b                                   [add, sub, ...]
 *   ICMP     d = (a mode b) ? 1 : 0, mode AIWC_ICMP_*             [icmp]
 *   FADD FSUB FMUL FDIV d = a op b                  [fadd, fsub, fmul, fdiv]
 *   FCMP     d = (a mode b) ? 1 : 0, mode AIWC_FCMP_* (false if either
 *            is NaN, except UNE)                                  [fcmp]
 *   FMA      d = a * b + c, one rounding                          [call]
 *   FSQRT    d = sqrt(a)                                          [call]
 *   FMIN FMAX d = min / max (a, b)                                [call]
 *   SITOFP   d = float((int32) a)                               [sitofp]
 *   FPTOSI   d = (int64)(int32) trunc(a); NaN -> 0, saturating  [fptosi]
 *   SEXT     d = (int64)(int32) a                                 [sext]
 *   ZEXT     d = a & 0xFFFFFFFF                                   [zext]
 *   SELECT   d = a != 0 ? b : c                                 [select]
 *   GEP      d = a + b * imm (b a register);  with IMM_B: d = a + imm
 *                                                        [getelementptr]
 *   LOAD     d.. = element i at address a + i * size, mode AIWC_LD_*  [load]
 *   STORE    element i of b.. to address a + i * size, mode AIWC_ST_* [store]
 *   ATOMIC   d = old 32-bit value at a, sign-extended; stores
 *            (old mode b), mode AIWC_AT_*                      [atomicrmw]
 *   BR       next = a != 0 ? imm : target2; a branch event of `site` [br]
 *   JMP      next = imm                                          [br]
 *   BARRIER  waits for every work-item of the work-group         [call]
 *   BUILTIN  d = work-item function mode (AIWC_BI_* + dimension)  [call]
 * Falling off the end of the program, or running more than max_steps
 * instructions in one work-item, fails the launch.                         */
#define AIWC_NREG 64
#define AIWC_ADDR_TAG_SHIFT 40
#define AIWC_MAX_KERNEL_ARGS 32
enum {
  AIWC_OP_RET = 0, AIWC_OP_MOV, AIWC_OP_ADD, AIWC_OP_SUB, AIWC_OP_MUL, AIWC_OP_SDIV,
  AIWC_OP_SREM, AIWC_OP_UDIV, AIWC_OP_UREM, AIWC_OP_SHL, AIWC_OP_LSHR, AIWC_OP_ASHR,
  AIWC_OP_AND, AIWC_OP_OR, AIWC_OP_XOR, AIWC_OP_ICMP, AIWC_OP_FADD, AIWC_OP_FSUB,
  AIWC_OP_FMUL, AIWC_OP_FDIV, AIWC_OP_FCMP, AIWC_OP_FMA, AIWC_OP_FSQRT, AIWC_OP_FMIN,
  AIWC_OP_FMAX, AIWC_OP_SITOFP, AIWC_OP_FPTOSI, AIWC_OP_SEXT, AIWC_OP_ZEXT,
  AIWC_OP_SELECT, AIWC_OP_GEP, AIWC_OP_LOAD, AIWC_OP_STORE, AIWC_OP_ATOMIC, AIWC_OP_BR,
  AIWC_OP_JMP, AIWC_OP_BARRIER, AIWC_OP_BUILTIN, AIWC_OP_COUNT
};
enum { AIWC_ICMP_EQ = 0, AIWC_ICMP_NE, AIWC_ICMP_SLT, AIWC_ICMP_SLE, AIWC_ICMP_SGT,
       AIWC_ICMP_SGE, AIWC_ICMP_ULT, AIWC_ICMP_ULE, AIWC_ICMP_UGT, AIWC_ICMP_UGE };
enum { AIWC_FCMP_OEQ = 0, AIWC_FCMP_UNE, AIWC_FCMP_OLT, AIWC_FCMP_OLE, AIWC_FCMP_OGT,
       AIWC_FCMP_OGE };
enum { AIWC_LD_I32 = 0,  /* 4 bytes, sign-extended                            */
       AIWC_LD_U32 = 1,  /* 4 bytes, zero-extended (also binary32 values)     */
       AIWC_LD_64 = 2 }; /* 8 bytes                                           */
enum { AIWC_ST_32 = 0, AIWC_ST_64 = 1 };
enum { AIWC_AT_ADD = 0, AIWC_AT_SUB, AIWC_AT_AND, AIWC_AT_OR, AIWC_AT_XOR, AIWC_AT_MIN,
       AIWC_AT_MAX, AIWC_AT_UMIN, AIWC_AT_UMAX };   /* MIN/MAX signed         */
enum { AIWC_BI_GLOBAL_ID = 0, AIWC_BI_LOCAL_ID = 3, AIWC_BI_GROUP_ID = 6,
       AIWC_BI_GLOBAL_SIZE = 9, AIWC_BI_LOCAL_SIZE = 12, AIWC_BI_NUM_GROUPS = 15 };
enum { AIWC_INSN_IMM_B = 1u };

typedef struct aiwc_insn {
  uint8_t op;        /* AIWC_OP_*                                           */
  uint8_t mode;      /* predicate, load / store / atomic form, builtin      */
  uint8_t width;     /* 1..16; 1 for LOAD/STORE widths above, ATOMIC, BR,
                        JMP, BARRIER, BUILTIN, RET                          */
  uint8_t flags;     /* AIWC_INSN_IMM_B                                     */
  uint8_t d, a, b, c;/* registers < AIWC_NREG                               */
  uint16_t id;       /* opcode id recorded when the instruction executes    */
  uint16_t site;     /* BR: branch site id (< n_sites)                      */
  uint32_t target2;  /* BR: next instruction when the condition is zero     */
  int64_t imm;       /* immediate; BR / JMP: next instruction index         */
} aiwc_insn;         /* 24 bytes                                            */

/* A program: n_insn instructions (host; copied), the opcode table its ids
 * index (host; copied) and its number of branch sites.  The create call
 * checks every field above and that each instruction's id has the kind its
 * operation needs (LOAD -> AIWC_KIND_LOAD, STORE -> STORE, ATOMIC ->
 * ATOMIC_RMW, BR -> BRANCH_COND, BARRIER -> BARRIER, any other -> COMPUTE
 * or OTHER); AIWC_ERR_INVALID_ARG otherwise.                               */
typedef struct aiwc_program_desc {
  uint32_t struct_size;
  uint32_t n_insn;
  const aiwc_insn *code;
  uint32_t n_opcode_ids;
  uint32_t n_sites;
  const aiwc_opcode_info *opcode_table;
} aiwc_program_desc;

enum { AIWC_ARG_GLOBAL = 0,   /* ptr: device buffer of `bytes` bytes (>= 1,
                                 16-byte aligned); read and written in place */
       AIWC_ARG_LOCAL = 1,    /* `bytes` of local memory per work-group      */
       AIWC_ARG_SCALAR = 2 }; /* `value` is the register's 64 bits          */
typedef struct aiwc_kernel_arg {
  uint32_t kind;
  uint32_t reserved;
  void *ptr;
  uint64_t bytes;
  uint64_t value;
} aiwc_kernel_arg;

/* The launch: dims 1..3, global[i] a multiple of local[i], local size
 * product <= 1024, local memory <= 65536 bytes.                             */
typedef struct aiwc_ndrange {
  uint32_t dims;
  uint32_t global[3];
  uint32_t local[3];
  uint32_t reserved;
} aiwc_ndrange;

typedef struct aiwc_program aiwc_program;
typedef struct aiwc_produced aiwc_produced;

aiwc_status aiwc_program_create(aiwc_ctx *ctx, const aiwc_program_desc *desc,
                                aiwc_program **out);
aiwc_status aiwc_program_destroy(aiwc_program *prog);

/* Execute the program over the ND-range and keep its trace.  The kernel runs
 * twice: a counting run sizes every work-item's streams, then the global
 * buffers are restored from a device copy taken before it and a recording
 * run writes the events; the buffers end as the recording run left them.
 * Blocks the calling thread (the trace's sizes decide its allocation).
 * max_steps (1..2^31-1; 0 = 2^20) bounds the instructions of one work-item.
 * Errors: INVALID_ARG for a bad ND-range or argument list, and for a run
 * that accessed memory outside its buffers or misaligned, exceeded
 * max_steps, fell off the program's end, or left some work-items of a
 * work-group waiting at a barrier that others never reached (message names
 * which); UNSUPPORTED when the two runs disagree (control flow that depends
 * on the order in which work-groups ran, e.g. on an atomic's old value);
 * OUT_OF_MEMORY for the snapshot or the trace arrays.                       */
aiwc_status aiwc_produce(aiwc_program *prog, const aiwc_ndrange *nd,
                         const aiwc_kernel_arg *args, uint32_t n_args, uint64_t max_steps,
                         void *stream, aiwc_produced **out);

/* A trace descriptor over the produced arrays: every stream field, the
 * counts, wg_size, n_sites and the program's opcode table (owned by the
 * produced object, valid until it is destroyed), history_len 16,
 * max_lsb_skip 10 and flags 0; the caller may change history_len and flags
 * before aiwc_trace_create.                                                 */
aiwc_status aiwc_produced_desc(const aiwc_produced *p, aiwc_trace_desc *out);
/* Copy the produced arrays to host memory (a NULL pointer skips that array;
 * lengths are those of aiwc_produced_desc: n_events, n_workitems + 1, n_mem,
 * n_mem, n_branch, n_branch).  Synchronous.                                 */
aiwc_status aiwc_produced_to_host(const aiwc_produced *p, uint16_t *opcode, uint64_t *wi_offsets,
                                  uint64_t *addr, uint8_t *mem_kind, uint32_t *br_site,
                                  uint8_t *br_taken);
aiwc_status aiwc_produced_destroy(aiwc_produced *p);

#ifdef __cplusplus
}
#endif
#endif /* AIWC_H */
