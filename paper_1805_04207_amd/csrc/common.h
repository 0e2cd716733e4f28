// common.h -- types and device helpers shared by the libaiwc kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aiwc.h"

typedef unsigned long long u64;
typedef unsigned int u32;

#define AIWC_WAVE 64

// ---------------------------------------------------------------- layout
// Accumulators written by the stage kernels and read by the finalize kernel.
// They live at the start of the per-trace zero region (cleared by a fill
// kernel at the start of every characterization).
#define SPEC_DENSE 256       // level-0 spectrum kept densely for f < 256
#define AIWC_STAGE_CAP 16384 // records the bucket kernel stages on chip per round
#define VAL_DENSE 65536      // ITB / IPT value histograms are dense below this
#define TWO_LEVEL_PBITS 12   // partitions from 2^12 on are scattered in two passes
#define AIWC_SORT_CAP 16384  // branch records one windows work block counts on chip
#define AIWC_HOT_MIN 65536   // site segments counted in parallel pieces from this length on
#define AIWC_HOT_PART (1u << 18)  // partitions split into hot-page tables + the rest from this size
#define AIWC_HOT_PMAX 64          // hot partitions per trace
#define AIWC_HOT_CAND 8           // candidate pages per hot partition
#define AIWC_HOT_WORDS (2048 + AIWC_HOT_PMAX * AIWC_HOT_CAND * (1024 + 64))  // u32 words of the state
struct DevAccum {
  u64 itb_min_inv, itb_max, itb_cnt, itb_sum;   // min stored as max of ~v
  u64 ipt_min_inv, ipt_max, ipt_cnt, ipt_sum;
  u64 barriers, bad_ids;
  u64 itb_large_n, ipt_large_n;
  u64 sp_reads[2], sp_writes[2];
  u64 distinct[2][AIWC_NSKIP];
  u64 ent_lo[2][AIWC_NSKIP], ent_hi[2][AIWC_NSKIP];  // fixed point, 2^-64 units
  u64 uniq_r[2], uniq_w[2];
  u64 spec_dense[2][SPEC_DENSE];
  u64 redos;
  u64 mem_queue;
  u64 br_windows, br_minsum, yok_lo, yok_hi;
  u64 br_queue;
  u64 bad_mem;
  u64 pat_lo, pat_hi;        // pattern entropy sum, 2^-64 units
  u64 split_fail;            // on-chip tables that could not be split further
  u64 br_queue2, br_big_n;   // windows ranges left to the hash-table kernel
  u64 br_hot_n, br_piece_q;  // hot site segments registered, their pieces taken
};

// Everything a kernel needs to know about one trace and its scratch.
struct TraceArgs {
  // inputs (device)
  const uint16_t *opcode;
  const u64 *wi_off;
  const u64 *addr;
  const uint8_t *mem_kind;
  const u32 *br_site;
  const uint8_t *br_taken;
  const u32 *op_info;        // per id: kind | width << 8 | class << 16
  u64 n_events, n_wi, n_mem, n_branch;
  u32 n_ids, n_classes, n_sites, m;
  u32 wg_size;
  u32 br_flags;              // AIWC_BRANCH_* variant bits of the trace
  // planning
  u32 pbits;                 // memory partitions P = 2^pbits
  u32 n_hist_blocks;         // blocks of the partition histogram / scatter
  u64 hist_chunk;            // records per histogram block (multiple of 4)
  u32 sp_cap;                // sparse spectrum capacity per space (pow2)
  u32 br_passes;             // radix passes of 8 bits over the site ids
  u64 br_tiles;              // 4096-element tiles of the branch stream
  u64 br_blocks;             // windows work blocks
  u64 large_cap;             // capacity of the ITB / IPT large-value lists
  u64 ops_task;              // events per ops task
  u64 ops_tasks;
  u64 *ops_wlo;              // [ops_tasks + 1] first work-item of each ops task (or null)
  // scratch (device)
  DevAccum *acc;
  u64 *id_hist;              // [n_ids]
  u64 *class_hist;           // [n_classes]
  u64 *itb_hist, *ipt_hist;  // [VAL_DENSE]
  u64 *itb_large, *ipt_large;// [large_cap]
  u64 *sp_f, *sp_m;          // [2][sp_cap] sparse level-0 spectrum (f >= 256)
  u32 *seg_start, *seg_end;  // [n_sites]
  u32 *part_hist;            // [n_hist_blocks][P]
  u32 *part_off;             // [P + 1]
  u32 *part_order;           // [P] bucket-kernel queue order: oversized partitions first
  u32 part_queue;            // entries of part_order the bucket kernel takes (0: all P)
  u32 pad1;
  u64 *part_rec;             // [n_mem]
  u64 *part_tmp;             // [n_mem] coarse-bucket records of the two-level scatter (or null)
  u32 *part_cur;             // [P + 512] fine cursors, coarse cursors, coarse tile starts
  u32 *part_tag;             // [n_mem] page slot and position of each record (bucket kernel)
  u64 *part_cmp;             // [n_mem] hot partitions' records off their candidate pages
  u32 *mem_hot;              // [AIWC_HOT_WORDS] hot partitions, candidate pages, their tables
                             // (null: no hot-page path)
  u32 *br_a, *br_b;          // [n_branch] radix ping-pong
  u32 *br_cnt;               // [256 * br_tiles]; after the sort: (start, end) ranges
                             // left to the hash-table windows kernel
  u32 *br_hot_list;          // [2 * br_hot_cap] (start, end) of hot site segments
  unsigned long long *br_hot_tab; // [br_hot_cap << m] n0 | n1 << 32 per history
  u32 br_hot_cap;            // hot segments with a table (0: none)
  u32 pad2;
  u32 *pat_hist;             // [2^m] windows per history pattern (pattern entropy)
  u32 *scan_tmp;             // block sums for the generic scan
  // result (device)
  aiwc_metrics_host *out;
  u64 *out_class_hist;       // [n_classes]
  u64 *out_spec;             // [2][SPEC_DENSE] then sparse export
  u32 spec_export_cap;       // sparse pairs exported per space
  u32 pad0;
  // batch bookkeeping
  u32 *br_sorted;            // br_a or br_b: where the last radix pass leaves data
  void *zero_base;           // start and size of this trace's zero region
  u64 zero_bytes;
};

// A kernel either serves one trace (arguments by value) or a whole batch
// (grid.y = trace index into a device array of TraceArgs).  Kernels copy the
// result into a local at entry, so that a batch kernel reads its trace's
// arguments from memory once rather than after every store.
template <bool BATCH>
__device__ __forceinline__ const TraceArgs &trace_args(const TraceArgs &A0,
                                                       const TraceArgs *batch) {
  if constexpr (BATCH) return batch[blockIdx.y];
  else return A0;
}

// ------------------------------------------------------------ device math
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Runs of equal keys among neighbouring lanes: the lanes that end a run
// (lane 63 always does).  The next lane's key arrives by a whole-wavefront
// DPP shift (wave_shl:1), which every lane must execute: a lane left out of a
// cross-lane read would hand its neighbour a stale value.
__device__ __forceinline__ u64 run_ends(u64 key) {
  const int lane = lane_id();
  const u32 lo = (u32)__builtin_amdgcn_update_dpp(0, (int)(u32)key, 0x130, 0xF, 0xF, false);
  const u32 hi = (u32)__builtin_amdgcn_update_dpp(0, (int)(u32)(key >> 32), 0x130, 0xF, 0xF,
                                                  false);
  const u64 next = ((u64)hi << 32) | lo;
  return __ballot(lane == 63 || next != key);
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void wave_sum_u128(u64 &lo, u64 &hi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    u64 ol = __shfl_xor(lo, o, 64), oh = __shfl_xor(hi, o, 64);
    u64 nl = lo + ol;
    hi = hi + oh + (nl < lo ? 1ull : 0ull);
    lo = nl;
  }
}

// Exact 128-bit accumulation into a pair of u64 words (global or LDS).
__device__ __forceinline__ void atomic_add_u128(u64 *lo, u64 *hi, u64 vlo, u64 vhi) {
  if (vlo == 0 && vhi == 0) return;
  u64 old = atomicAdd(lo, vlo);
  u64 carry = (old + vlo < old) ? 1ull : 0ull;
  if (vhi + carry) atomicAdd(hi, vhi + carry);
}

// Non-negative double -> unsigned fixed point with 64 fraction bits, as a
// (lo, hi) pair.  Exact for every double below 2^63; bits below 2^-64 are
// truncated.
__device__ __forceinline__ void to_fx64(double d, u64 &lo, u64 &hi) {
  lo = hi = 0;
  if (!(d > 0.0)) return;
  int e;
  double mant = frexp(d, &e);                 // d = mant * 2^e, mant in [0.5,1)
  u64 m53 = (u64)ldexp(mant, 53);             // exact
  int sh = e - 53 + 64;                       // value * 2^64 = m53 * 2^sh
  if (sh >= 128) { lo = hi = ~0ull; return; }
  if (sh >= 64) { hi = m53 << (sh - 64); lo = 0; }
  else if (sh > 0) { lo = m53 << sh; hi = m53 >> (64 - sh); }
  else if (sh == 0) { lo = m53; }
  else if (sh > -64) { lo = m53 >> (-sh); }
}

__host__ __device__ __forceinline__ double fx64_to_double(u64 lo, u64 hi) {
  return ((double)hi * 18446744073709551616.0 + (double)lo) * 5.421010862427522170e-20;
}

// A bijection of the 54-bit page numbers (address >> 10): multiply by odd
// constants and xor-shift inside 54 bits.  Spreads pages over partitions.
#define PAGE_BITS 54
__device__ __forceinline__ u64 mix54(u64 x) {
  const u64 M = (1ull << PAGE_BITS) - 1ull;
  x &= M;
  x = (x * 0x2545F4914F6CDD1Dull) & M;
  x ^= x >> 27;
  x = (x * 0x1D8E4E27C47D124Full) & M;
  x ^= x >> 25;
  x = (x * 0x3C79AC492BA7B653ull) & M;
  x ^= x >> 29;
  return x;
}

__device__ __forceinline__ u32 hash_slot(u64 key, u32 cap) {
  u64 h = key * 0x9E3779B97F4A7C15ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  u32 x = (u32)(h >> 32);
  return (u32)(((u64)x * cap) >> 32);
}

// ---------------------------------------------------------- host helpers
// Optional instrumentation: when set, a hipEvent is recorded on the stream
// after every kernel launch, tagged with the kernel's name.
struct StageMarks {
  virtual void mark(const char *name, hipStream_t s) = 0;
  virtual void fork(hipStream_t from, hipStream_t to) = 0;   // `to` continues from `from`
  virtual ~StageMarks() {}
};

// Launch shapes of a batch: the maxima over its traces (grid.x) and the
// trace count (grid.y).  For one trace, batch == nullptr and n == 1.
struct BatchDims {
  u32 n = 1;
  const TraceArgs *batch = nullptr;   // device array [n], or nullptr
  u64 max_ops_tasks = 0, max_hist_blocks = 0, max_parts = 0, max_tiles = 0;
  u64 max_br_blocks = 0, max_scan_blocks = 0, max_zero16 = 0;
  u32 max_ids = 0, max_passes = 0;
  u64 ops_lds = 0;                    // dynamic LDS of the ops kernel (max over traces)
  u32 ops_max_blocks = 0;             // cap on the ops grid (0 = none)
  bool any_mem = false, any_branch = false;
  bool any_two_level = false, any_one_level = false;   // memory scatter paths in use
  bool any_local = false, any_global = false;   // branch history variants present
  bool any_pattern = false;                     // some trace wants the pattern entropy
  bool any_hot = false;                         // some trace has hot-segment tables
  bool any_hot_mem = false;                     // some trace has the hot-page path
  u32 max_pattern_bins = 0;
  bool vec = true;                    // every address / kind array 16 / 4 B aligned
  bool ops_vec = true;                // every opcode array 16 B aligned
};

namespace aiwc_kernels {
hipError_t launch_zero(const TraceArgs &a, const BatchDims &d, hipStream_t s);
hipError_t launch_ops(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm);
hipError_t launch_mem(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm);
hipError_t launch_mem_partition(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                                StageMarks *pm);
hipError_t launch_mem_bucket(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                             StageMarks *pm);
hipError_t launch_mem_count(const TraceArgs &a, u32 *count, hipStream_t s);
hipError_t launch_mem_scatter_range(const TraceArgs &a, u32 p0, u32 p1, u32 *cursor, u64 *rec,
                                    hipStream_t s);
hipError_t launch_branch(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm);
hipError_t launch_finalize(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm);
u64 scan_blocks_for(u64 n);
size_t ops_lds_bytes(u32 n_ids);
hipError_t launch_merge_offsets(u64 *dst, const u64 *src, u64 n_wi, u64 base, bool first,
                                hipStream_t s);
}  // namespace aiwc_kernels

#define AIWC_MARK(pm, name, s) \
  do { if (pm) (pm)->mark(name, s); } while (0)
