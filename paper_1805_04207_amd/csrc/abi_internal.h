// abi_internal.h -- host-side objects behind the opaque handles of aiwc.h.
#pragma once

#include <string>
#include <vector>

#include "common.h"

// Launch-shape knobs the autotuner searches (defaults = built-in shapes).
struct Tune {
  int ops_shift = 0;        // ops task size = default * 2^ops_shift
  u32 hist_blocks = 256;    // max blocks of the partition histogram / scatter
  int part_shift = 0;       // partitions = sized count * 2^part_shift
  bool operator==(const Tune &o) const {
    return ops_shift == o.ops_shift && hist_blocks == o.hist_blocks && part_shift == o.part_shift;
  }
};

struct TracePlan {
  u32 pbits = 4;
  u32 n_hist_blocks = 1;
  u64 hist_chunk = 4;
  u32 sp_cap = 64;
  u32 br_passes = 0;
  u64 br_tiles = 0, br_blocks = 0;
  u64 large_cap = 1;
  u64 ops_task = 4096, ops_tasks = 1;
  // scratch offsets (bytes)
  u64 o_acc = 0, o_id_hist = 0, o_class_hist = 0, o_itb_hist = 0, o_ipt_hist = 0;
  u64 o_sp_f = 0, o_sp_m = 0, o_seg_start = 0, o_seg_end = 0;
  u64 zero_bytes = 0;
  u64 o_itb_large = 0, o_ipt_large = 0, o_part_hist = 0, o_part_off = 0, o_part_rec = 0;
  u64 o_part_order = 0, o_part_tag = 0, o_ops_wlo = 0, o_part_tmp = 0, o_part_cur = 0;
  u64 o_br_a = 0, o_br_b = 0, o_br_cnt = 0, o_scan_tmp = 0, o_pat_hist = 0;
  u64 o_br_hot_list = 0, o_br_hot_tab = 0, o_mem_hot = 0, o_part_cmp = 0;
  u32 br_hot_cap = 0;
  u64 scratch_bytes = 0;
  // result buffer offsets (bytes)
  u64 r_metrics = 0, r_class = 0, r_spec = 0, result_bytes = 0;
  u32 spec_export_cap = 0;
};

struct SizerState;
struct BatchState;

// Per-context stage timer (instrumentation; see aiwc_profile_*).  A stage's
// time runs from the previous mark on the same stream to its own mark, so
// stages on the side stream are timed on their own chain.
struct Profiler : StageMarks {
  bool on = false;
  hipEvent_t start = nullptr;
  struct Mark { std::string name; hipEvent_t end, begin; };
  std::vector<Mark> marks;
  std::vector<std::pair<hipStream_t, hipEvent_t>> last;   // latest mark per stream
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  void begin(hipStream_t s);
  void mark(const char *name, hipStream_t s) override;
  void fork(hipStream_t from, hipStream_t to) override;
  void release();
  hipEvent_t &last_of(hipStream_t s);
};

// A second stream of the context: the instruction and branch stages run on
// it, beside the memory stage, between a fork and a join event.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct aiwc_ctx {
  int device = 0;
  int n_cu = 256;
  std::string arch;
  std::string err;
  char *arena = nullptr;
  u64 arena_bytes = 0;
  hipEvent_t last_done = nullptr;
  SizerState *sizer = nullptr;
  BatchState *batch = nullptr;
  aiwc_batch_stats last_stats{};
  Profiler prof;
  SideStream side;
  bool single_stream = false;      // AIWC_SINGLE_STREAM: no side stream
  std::vector<std::pair<std::string, Tune>> tune_cache;  // class key -> best shape
  bool tune_loaded = false;
  // result blocks and completion events of destroyed metrics handles, kept
  // for the next characterizations (no allocation in a steady loop)
  std::vector<std::pair<u64, void *>> result_pool;      // (bytes, device block)
  std::vector<hipEvent_t> event_pool;
};

struct aiwc_trace {
  aiwc_ctx *ctx = nullptr;
  u64 serial = 0;                 // unique per created trace, never reused
  aiwc_trace_desc d{};
  u32 n_classes = 0;
  std::vector<u32> host_info;
  u32 *dev_info = nullptr;
};

// Device block shared by the metrics handles of one batch call.
struct SharedBuf {
  void *p = nullptr;
  size_t refs = 0;
};

struct aiwc_metrics {
  aiwc_ctx *ctx = nullptr;
  TracePlan plan;
  u32 n_classes = 0;
  void *buf = nullptr;
  u64 buf_bytes = 0;             // size of an owned (pooled) result block
  SharedBuf *shared = nullptr;   // set when buf points into a batch block
  hipEvent_t done = nullptr;
  u32 spec_pairs[2] = {0, 0};
  void *stage = nullptr;         // concatenated trace of a merged call
};

void ctx_error(aiwc_ctx *ctx, const char *fmt, ...);
void plan_trace(const aiwc_trace *t, u32 pbits, TracePlan &p, const Tune *tune = nullptr,
                u64 rec_cap = ~0ull);
u32 bound_pbits(u64 n_mem);
void fill_args(const aiwc_trace *t, const TracePlan &p, char *scratch, char *result,
               TraceArgs &a);
hipError_t enqueue_stages(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                          StageMarks *pm, const SideStream *side = nullptr);
const SideStream *side_stream(aiwc_ctx *ctx);
void add_dims(const aiwc_trace *t, const TracePlan &p, const TraceArgs &a, BatchDims &d);
aiwc_status ensure_arena(aiwc_ctx *ctx, u64 bytes);
aiwc_status new_metrics(aiwc_ctx *ctx, const aiwc_trace *t, const TracePlan &p,
                        aiwc_metrics **out, SharedBuf *shared = nullptr, void *buf = nullptr);
aiwc_status characterize_planned(aiwc_ctx *ctx, const aiwc_trace *t, u32 pbits,
                                 hipStream_t s, aiwc_metrics **out);
aiwc_status validate_on_device(aiwc_ctx *ctx, const aiwc_trace *t);
aiwc_status decode_result(aiwc_ctx *ctx, const char *raw, aiwc_metrics_host *out,
                          u32 spec_pairs[2]);

void sizer_init(aiwc_ctx *ctx);
void sizer_free(aiwc_ctx *ctx);
void batch_free(aiwc_ctx *ctx);
