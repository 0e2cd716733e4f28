// abi.hip -- the C ABI of libaiwc: contexts, trace descriptors, the
// per-trace planner (scratch layout and launch shapes) and metrics handles.
// All metric arithmetic runs in the kernels of k_*.hip; this file only
// validates arguments, sizes buffers and enqueues launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "abi_internal.h"

namespace aiwc_kernels {
u64 scan_tmp_elems(u64 n);
u64 br_tiles_for(u64 n);
u64 br_blocks_for(u64 n);
}

static thread_local std::string g_noctx_err;
// Creation serials of traces: a destroyed trace's heap address may be reused
// by the next trace, its serial never is.
static std::atomic<u64> g_trace_serial{0};

void ctx_error(aiwc_ctx *ctx, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf; else g_noctx_err = buf;
}

#define HIP_OR(ctx, call)                                                       \
  do {                                                                          \
    hipError_t e__ = (call);                                                    \
    if (e__ != hipSuccess) {                                                    \
      ctx_error(ctx, "%s failed: %s", #call, hipGetErrorString(e__));           \
      return AIWC_ERR_HIP;                                                      \
    }                                                                           \
  } while (0)

static inline u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }
static inline u32 ceil_log2(u64 x) {
  u32 b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// ------------------------------------------------------------------ plan
// Scratch layout of one trace: a zero region (cleared by a kernel) followed
// by buffers that every stage fully writes before reading.
void plan_trace(const aiwc_trace *t, u32 pbits, TracePlan &p, const Tune *tune, u64 rec_cap) {
  const aiwc_trace_desc &d = t->d;
  const Tune T = tune ? *tune : Tune();
  p = TracePlan();
  int pb = (int)pbits + T.part_shift;
  p.pbits = d.n_mem ? (u32)std::min(15, std::max(4, pb)) : 4;
  const u64 P = 1ull << p.pbits;
  // memory: histogram blocks up to the tuned maximum (more when the
  // partition table is small enough for several blocks per CU), >= 16K
  // records each
  u64 nb = (d.n_mem + 16383) / 16384;
  u64 nbmax = std::max<u32>(1, T.hist_blocks);
  if (P <= 4096) nbmax *= 4; else if (P <= 8192) nbmax *= 2;
  nb = std::max<u64>(1, std::min<u64>(nb, nbmax));
  p.n_hist_blocks = (u32)nb;
  p.hist_chunk = align_up((d.n_mem + nb - 1) / nb, 8);
  if (p.hist_chunk == 0) p.hist_chunk = 8;
  u64 r = (u64)std::sqrt((double)(2 * d.n_mem)) + 2;
  p.sp_cap = (u32)std::max<u64>(64, 1ull << ceil_log2(2 * r));
  // branches
  p.br_passes = 0;
  if (d.n_sites > 1) p.br_passes = (ceil_log2(d.n_sites) + 7) / 8;
  p.br_tiles = aiwc_kernels::br_tiles_for(d.n_branch);
  p.br_blocks = aiwc_kernels::br_blocks_for(d.n_branch);
  // ops
  p.large_cap = d.n_events / 65536 + 1;
  u64 E = std::max<u64>(4096, (d.n_events + 16383) / 16384);
  if (T.ops_shift > 0) E <<= T.ops_shift;
  if (T.ops_shift < 0) E = std::max<u64>(2048, E >> (-T.ops_shift));
  p.ops_task = align_up(E, 512);
  p.ops_tasks = std::max<u64>(1, (d.n_events + p.ops_task - 1) / p.ops_task);

  u64 o = 0;
  auto take = [&](u64 bytes) { u64 at = o; o += align_up(bytes, 256); return at; };
  p.o_acc = take(sizeof(DevAccum));
  p.o_id_hist = take(8ull * d.n_opcode_ids);
  p.o_class_hist = take(8ull * t->n_classes);
  p.o_itb_hist = take(8ull * VAL_DENSE);
  p.o_ipt_hist = take(8ull * VAL_DENSE);
  p.o_sp_f = take(8ull * 2 * p.sp_cap);
  p.o_sp_m = take(8ull * 2 * p.sp_cap);
  p.o_seg_start = take(4ull * std::max<u32>(1, d.n_sites));
  p.o_seg_end = take(4ull * std::max<u32>(1, d.n_sites));
  if (d.flags & AIWC_BRANCH_PATTERN_ENTROPY) p.o_pat_hist = take(4ull << d.history_len);
  p.zero_bytes = o;
  p.o_itb_large = take(8ull * p.large_cap);
  p.o_ipt_large = take(8ull * p.large_cap);
  p.o_part_hist = take(4ull * p.n_hist_blocks * P);
  p.o_part_off = take(4ull * (P + 1));
  p.o_part_order = take(4ull * P);
  // partition records and tags: the whole memory stream, or the largest
  // group of partitions a stream reduces at once
  const u64 nrec = std::max<u64>(1, std::min<u64>(d.n_mem, rec_cap));
  p.o_part_rec = take(8ull * nrec);
  p.o_part_tag = take(4ull * nrec);
  // the two-level scatter: coarse-bucket records and the cursors
  p.o_part_tmp = (d.n_mem && p.pbits >= TWO_LEVEL_PBITS) ? take(8ull * nrec) : 0;
  p.o_part_cur = take(4ull * (P + 512));
  // hot pages: the state and tables, and a buffer for the compacted rest
  // (the coarse-bucket records' buffer when there is one: free by then);
  // not for the partition groups of a stream, reduced without them
  if (d.n_mem >= AIWC_HOT_PART && rec_cap == ~0ull) {
    p.o_mem_hot = take(4ull * AIWC_HOT_WORDS);
    p.o_part_cmp = p.o_part_tmp ? p.o_part_tmp : take(8ull * nrec);
  }
  p.o_ops_wlo = take(8ull * (p.ops_tasks + 1));
  // radix records: site << 1 | outcome (u32), or with the global history
  // site << 33 | history << 1 | outcome (u64)
  const u64 rec = (d.flags & AIWC_BRANCH_GLOBAL_HISTORY) ? 8 : 4;
  p.o_br_a = take(rec * std::max<u64>(1, d.n_branch));
  p.o_br_b = take(rec * std::max<u64>(1, d.n_branch));
  p.o_br_cnt = take(4ull * 256 * std::max<u64>(1, p.br_tiles));
  p.o_scan_tmp = take(4ull * aiwc_kernels::scan_tmp_elems(256 * std::max<u64>(1, p.br_tiles)));
  // hot site segments (at least AIWC_HOT_MIN records, per-site histories of
  // m <= 16): a table of 2^m 64-bit counters each, for up to 64 of them
  // (at most 8 B per branch event)
  p.br_hot_cap = 0;
  if (!(d.flags & AIWC_BRANCH_GLOBAL_HISTORY) && d.history_len <= 16 && d.n_branch >= AIWC_HOT_MIN)
    p.br_hot_cap = (u32)std::min<u64>(64, d.n_branch / AIWC_HOT_MIN);
  p.o_br_hot_list = take(8ull * std::max<u32>(1, p.br_hot_cap));
  p.o_br_hot_tab = take(p.br_hot_cap ? (8ull << d.history_len) * p.br_hot_cap : 8);
  p.scratch_bytes = o;
  p.spec_export_cap = std::min<u32>(p.sp_cap, 65536);
  // result buffer: metrics, 4 status words, class histogram, spectrum pairs
  u64 rb = 0;
  p.r_metrics = rb; rb += align_up(sizeof(aiwc_metrics_host) + 32, 256);
  p.r_class = rb; rb += align_up(8ull * t->n_classes, 256);
  p.r_spec = rb; rb += align_up(8ull * 2 * 2 * p.spec_export_cap, 256);
  p.result_bytes = rb;
}

u32 bound_pbits(u64 n_mem) {
  // pages <= accesses: aim at <= 1024 pages (1 KiB) per partition
  u64 want = (n_mem + 1023) / 1024;
  u32 b = ceil_log2(std::max<u64>(want, 1));
  return std::min<u32>(15, std::max<u32>(4, b));
}

void fill_args(const aiwc_trace *t, const TracePlan &p, char *scratch, char *result,
               TraceArgs &a) {
  const aiwc_trace_desc &d = t->d;
  memset(&a, 0, sizeof a);
  a.opcode = d.opcode;
  a.wi_off = (const u64 *)d.wi_offsets;
  a.addr = (const u64 *)d.addr;
  a.mem_kind = d.mem_kind;
  a.br_site = d.br_site;
  a.br_taken = d.br_taken;
  a.op_info = t->dev_info;
  a.n_events = d.n_events;
  a.n_wi = d.n_workitems;
  a.n_mem = d.n_mem;
  a.n_branch = d.n_branch;
  a.n_ids = d.n_opcode_ids;
  a.n_classes = t->n_classes;
  a.n_sites = d.n_sites;
  a.m = d.history_len;
  a.pbits = p.pbits;
  a.n_hist_blocks = p.n_hist_blocks;
  a.hist_chunk = p.hist_chunk;
  a.sp_cap = p.sp_cap;
  a.br_passes = p.br_passes;
  a.br_tiles = p.br_tiles;
  a.br_blocks = p.br_blocks;
  a.large_cap = p.large_cap;
  a.ops_task = p.ops_task;
  a.ops_tasks = p.ops_tasks;
  a.ops_wlo = (u64 *)(scratch + p.o_ops_wlo);
  a.acc = (DevAccum *)(scratch + p.o_acc);
  a.id_hist = (u64 *)(scratch + p.o_id_hist);
  a.class_hist = (u64 *)(scratch + p.o_class_hist);
  a.itb_hist = (u64 *)(scratch + p.o_itb_hist);
  a.ipt_hist = (u64 *)(scratch + p.o_ipt_hist);
  a.itb_large = (u64 *)(scratch + p.o_itb_large);
  a.ipt_large = (u64 *)(scratch + p.o_ipt_large);
  a.sp_f = (u64 *)(scratch + p.o_sp_f);
  a.sp_m = (u64 *)(scratch + p.o_sp_m);
  a.seg_start = (u32 *)(scratch + p.o_seg_start);
  a.seg_end = (u32 *)(scratch + p.o_seg_end);
  a.part_hist = (u32 *)(scratch + p.o_part_hist);
  a.part_off = (u32 *)(scratch + p.o_part_off);
  a.part_order = (u32 *)(scratch + p.o_part_order);
  a.part_rec = (u64 *)(scratch + p.o_part_rec);
  a.part_tag = (u32 *)(scratch + p.o_part_tag);
  a.part_tmp = p.o_part_tmp ? (u64 *)(scratch + p.o_part_tmp) : nullptr;
  a.part_cur = (u32 *)(scratch + p.o_part_cur);
  a.br_a = (u32 *)(scratch + p.o_br_a);
  a.br_b = (u32 *)(scratch + p.o_br_b);
  a.br_cnt = (u32 *)(scratch + p.o_br_cnt);
  a.mem_hot = p.o_mem_hot ? (u32 *)(scratch + p.o_mem_hot) : nullptr;
  a.part_cmp = p.o_mem_hot ? (u64 *)(scratch + p.o_part_cmp) : nullptr;
  a.br_hot_list = (u32 *)(scratch + p.o_br_hot_list);
  a.br_hot_tab = (unsigned long long *)(scratch + p.o_br_hot_tab);
  a.br_hot_cap = p.br_hot_cap;
  a.pat_hist = (d.flags & AIWC_BRANCH_PATTERN_ENTROPY) ? (u32 *)(scratch + p.o_pat_hist) : nullptr;
  a.br_flags = d.flags & (AIWC_BRANCH_ZERO_HISTORY | AIWC_BRANCH_GLOBAL_HISTORY |
                          AIWC_BRANCH_PATTERN_ENTROPY);
  a.scan_tmp = (u32 *)(scratch + p.o_scan_tmp);
  a.out = (aiwc_metrics_host *)(result + p.r_metrics);
  a.out_class_hist = (u64 *)(result + p.r_class);
  a.out_spec = (u64 *)(result + p.r_spec);
  a.spec_export_cap = p.spec_export_cap;
  a.br_sorted = (p.br_passes & 1) ? a.br_b : a.br_a;
  a.zero_base = scratch + p.o_acc;
  a.zero_bytes = p.zero_bytes;
}

// Fold one trace into the launch shapes of a batch.
void add_dims(const aiwc_trace *t, const TracePlan &p, const TraceArgs &a, BatchDims &d) {
  const aiwc_trace_desc &D = t->d;
  d.max_ops_tasks = std::max<u64>(d.max_ops_tasks, p.ops_tasks);
  d.max_zero16 = std::max<u64>(d.max_zero16, p.zero_bytes / 16);
  d.max_ids = std::max<u32>(d.max_ids, D.n_opcode_ids);
  d.ops_lds = std::max<u64>(d.ops_lds, aiwc_kernels::ops_lds_bytes(D.n_opcode_ids));
  if ((uintptr_t)a.opcode % 16) d.ops_vec = false;
  if (D.n_mem) {
    d.any_mem = true;
    d.max_hist_blocks = std::max<u64>(d.max_hist_blocks, p.n_hist_blocks);
    d.max_parts = std::max<u64>(d.max_parts, 1ull << p.pbits);
    if (a.part_tmp) d.any_two_level = true; else d.any_one_level = true;
    if (a.mem_hot) d.any_hot_mem = true;
    if ((uintptr_t)a.addr % 16 || (uintptr_t)a.mem_kind % 8) d.vec = false;
  }
  if (D.n_branch) {
    d.any_branch = true;
    if (D.flags & AIWC_BRANCH_GLOBAL_HISTORY) d.any_global = true; else d.any_local = true;
    if (p.br_hot_cap) d.any_hot = true;
    if (D.flags & AIWC_BRANCH_PATTERN_ENTROPY) {
      d.any_pattern = true;
      d.max_pattern_bins = std::max<u32>(d.max_pattern_bins, 1u << D.history_len);
    }
    d.max_tiles = std::max<u64>(d.max_tiles, p.br_tiles);
    d.max_passes = std::max<u32>(d.max_passes, p.br_passes);
    d.max_br_blocks = std::max<u64>(d.max_br_blocks, p.br_blocks);
    d.max_scan_blocks = std::max<u64>(d.max_scan_blocks,
                                      aiwc_kernels::scan_blocks_for(256 * p.br_tiles));
  }
}

// The context's side stream, created on first use (default priority,
// non-blocking so that a caller on the null stream does not serialize it).
const SideStream *side_stream(aiwc_ctx *ctx) {
  if (ctx->single_stream) return nullptr;
  SideStream &S = ctx->side;
  if (!S.s) {
    if (hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S.join, hipEventDisableTiming) != hipSuccess) {
      hipGetLastError();
      return nullptr;
    }
  }
  return &S;
}

// The stages of a characterization.  The memory stage and the instruction +
// branch stages touch disjoint data (they meet only in k_finalize), so with
// a side stream the latter run beside the former: the memory kernels are
// bound by latency and the radix passes need little LDS, so they overlap.
hipError_t enqueue_stages(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                          StageMarks *pm, const SideStream *side) {
  hipError_t e = aiwc_kernels::launch_zero(a, d, s);
  AIWC_MARK(pm, "k_zero", s);
  hipStream_t t = s;
  if (e == hipSuccess && side) {
    e = hipEventRecord(side->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
    if (pm) pm->fork(s, side->s);
    t = side->s;
  }
  if (side) {
    // two ops blocks per CU (13 KiB of LDS each) leave room for a partition
    // histogram or scatter block (128 KiB) beside them
    BatchDims ds = d;
    ds.ops_max_blocks = 512;
    if (e == hipSuccess) e = aiwc_kernels::launch_ops(a, ds, t, pm);
  } else if (e == hipSuccess) {
    e = aiwc_kernels::launch_ops(a, d, t, pm);
  }
  if (e == hipSuccess) e = aiwc_kernels::launch_branch(a, d, t, pm);
  if (e == hipSuccess) e = aiwc_kernels::launch_mem_partition(a, d, s, pm);
  // the bucket kernel fills every CU's registers and LDS, so nothing of the
  // side chain could run beside it: it starts once that chain is done
  if (e == hipSuccess && side) {
    e = hipEventRecord(side->join, side->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, side->join, 0);
    AIWC_MARK(pm, "join", s);   // the bucket kernel's span starts after the wait
  }
  if (e == hipSuccess) e = aiwc_kernels::launch_mem_bucket(a, d, s, pm);
  if (e == hipSuccess) e = aiwc_kernels::launch_finalize(a, d, s, pm);
  return e;
}

// ------------------------------------------------------------ profiling
void Profiler::begin(hipStream_t s) {
  used = 0;
  marks.clear();
  last.clear();
  if (!start) hipEventCreate(&start);
  hipEventRecord(start, s);
  last.emplace_back(s, start);
}

hipEvent_t &Profiler::last_of(hipStream_t s) {
  for (auto &l : last)
    if (l.first == s) return l.second;
  last.emplace_back(s, start);
  return last.back().second;
}

void Profiler::mark(const char *name, hipStream_t s) {
  if (used == pool.size()) {
    hipEvent_t e;
    hipEventCreate(&e);
    pool.push_back(e);
  }
  hipEvent_t e = pool[used++];
  hipEventRecord(e, s);
  hipEvent_t &prev = last_of(s);
  marks.push_back({name, e, prev});
  prev = e;
}

void Profiler::fork(hipStream_t from, hipStream_t to) {
  const hipEvent_t e = last_of(from);
  last_of(to) = e;
}

void Profiler::release() {
  if (start) hipEventDestroy(start);
  for (hipEvent_t e : pool) hipEventDestroy(e);
  pool.clear();
  marks.clear();
  start = nullptr;
}

extern "C" aiwc_status aiwc_profile_enable(aiwc_ctx *ctx, int on) {
  if (!ctx) { ctx_error(nullptr, "aiwc_profile_enable: NULL context"); return AIWC_ERR_INVALID_ARG; }
  ctx->prof.on = on != 0;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_profile_read(aiwc_ctx *ctx, char *names, size_t names_cap,
                                         double *ms, size_t max_stages, size_t *n_out) {
  if (!ctx || !n_out) { ctx_error(ctx, "aiwc_profile_read: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  Profiler &P = ctx->prof;
  std::string csv;
  size_t n = 0;
  if (P.start && !P.marks.empty()) {
    for (auto &m : P.marks) HIP_OR(ctx, hipEventSynchronize(m.end));
    for (auto &m : P.marks) {
      float t = 0.f;
      HIP_OR(ctx, hipEventElapsedTime(&t, m.begin, m.end));
      if (n < max_stages && ms) ms[n] = t;
      if (!csv.empty()) csv += ",";
      csv += m.name;
      ++n;
    }
  }
  if (names && names_cap) {
    size_t c = std::min(names_cap - 1, csv.size());
    memcpy(names, csv.data(), c);
    names[c] = 0;
  }
  *n_out = n;
  return AIWC_OK;
}

// ---------------------------------------------------- allocation-free path
// Scratch of aiwc_characterize_static: one array per GPU, allocated with the
// code object.  In host code `scratch` names a host-side stand-in; the
// device address of each GPU's copy is looked up once per device (at
// context creation, with the device current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[AIWC_STATIC_SCRATCH_BYTES];
static std::mutex g_static_mu;
static constexpr int STATIC_MAX_DEVICES = 64;
static void *g_static_ptr[STATIC_MAX_DEVICES];

static hipError_t static_scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (device < 0 || device >= STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
  if (g_static_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_static_ptr[device] = ptr;
  return hipSuccess;
}

static void *static_scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  return (device >= 0 && device < STATIC_MAX_DEVICES) ? g_static_ptr[device] : nullptr;
}

// --------------------------------------------------------------- context
extern "C" aiwc_status aiwc_context_create(int hip_device, aiwc_ctx **out) {
  if (!out) { ctx_error(nullptr, "aiwc_context_create: out is NULL"); return AIWC_ERR_INVALID_ARG; }
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
    ctx_error(nullptr, "aiwc_context_create: no HIP device %d (%d visible)", hip_device, n);
    return AIWC_ERR_INVALID_ARG;
  }
  aiwc_ctx *c = new aiwc_ctx();
  c->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    ctx_error(nullptr, "aiwc_context_create: hipSetDevice(%d) failed", hip_device);
    return AIWC_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
  }
  const hipError_t es = static_scratch_setup(hip_device);
  if (es != hipSuccess) {
    hipGetLastError();
    delete c;
    ctx_error(nullptr, "aiwc_context_create: device %d: address of the static scratch array: %s",
              hip_device, hipGetErrorString(es));
    return AIWC_ERR_HIP;
  }
  // AIWC_SINGLE_STREAM=1: every stage on the caller's stream, one after the
  // other (per-kernel timing without overlap)
  if (const char *e = getenv("AIWC_SINGLE_STREAM")) c->single_stream = atoi(e) != 0;
  sizer_init(c);
  *out = c;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_context_destroy(aiwc_ctx *ctx) {
  if (!ctx) return AIWC_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->arena) hipFree(ctx->arena);
  if (ctx->last_done) hipEventDestroy(ctx->last_done);
  if (ctx->side.s) hipStreamDestroy(ctx->side.s);
  if (ctx->side.fork) hipEventDestroy(ctx->side.fork);
  if (ctx->side.join) hipEventDestroy(ctx->side.join);
  ctx->prof.release();
  sizer_free(ctx);
  batch_free(ctx);
  for (auto &b : ctx->result_pool) hipFree(b.second);
  for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
  delete ctx;
  return AIWC_OK;
}

extern "C" const char *aiwc_last_error(const aiwc_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

// Grow the context's scratch arena (waiting for work that may still use it).
aiwc_status ensure_arena(aiwc_ctx *ctx, u64 bytes) {
  if (ctx->arena_bytes >= bytes) return AIWC_OK;
  if (ctx->arena) {
    if (ctx->last_done) hipEventSynchronize(ctx->last_done);
    hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_bytes = 0;
  }
  u64 want = std::max<u64>(bytes, 1ull << 20);
  void *p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of device memory: scratch of %llu bytes", (unsigned long long)want);
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  ctx->arena = (char *)p;
  ctx->arena_bytes = want;
  return AIWC_OK;
}

// ------------------------------------------------------------------ trace
extern "C" aiwc_status aiwc_trace_create(aiwc_ctx *ctx, const aiwc_trace_desc *d,
                                         aiwc_trace **out) {
  if (!ctx || !d || !out) { ctx_error(ctx, "aiwc_trace_create: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (d->struct_size != sizeof(aiwc_trace_desc)) {
    ctx_error(ctx, "aiwc_trace_create: struct_size %u != %zu", d->struct_size, sizeof(aiwc_trace_desc));
    return AIWC_ERR_INVALID_ARG;
  }
  if (d->history_len < 1 || d->history_len > 32) {
    ctx_error(ctx, "history_len %u outside 1..32", d->history_len);
    return AIWC_ERR_INVALID_ARG;
  }
  if (d->flags & ~(u32)(AIWC_VALIDATE_ON_DEVICE | AIWC_BRANCH_ZERO_HISTORY |
                        AIWC_BRANCH_GLOBAL_HISTORY | AIWC_BRANCH_PATTERN_ENTROPY)) {
    ctx_error(ctx, "unknown trace flag bits 0x%x", d->flags);
    return AIWC_ERR_INVALID_ARG;
  }
  if ((d->flags & AIWC_BRANCH_GLOBAL_HISTORY) && d->history_len > 31) {
    ctx_error(ctx, "the global branch history supports history_len <= 31");
    return AIWC_ERR_UNSUPPORTED;
  }
  if ((d->flags & AIWC_BRANCH_PATTERN_ENTROPY) && d->history_len > 20) {
    ctx_error(ctx, "the pattern entropy supports history_len <= 20");
    return AIWC_ERR_UNSUPPORTED;
  }
  if (d->max_lsb_skip != 10) {
    ctx_error(ctx, "max_lsb_skip must be 10 (got %u)", d->max_lsb_skip);
    return AIWC_ERR_INVALID_ARG;
  }
  if (!d->wi_offsets || (d->n_events && !d->opcode) || (d->n_mem && (!d->addr || !d->mem_kind)) ||
      (d->n_branch && (!d->br_site || !d->br_taken))) {
    ctx_error(ctx, "NULL array with a non-zero length");
    return AIWC_ERR_INVALID_ARG;
  }
  if (d->n_branch && d->n_sites == 0) { ctx_error(ctx, "n_branch > 0 needs n_sites >= 1"); return AIWC_ERR_INVALID_ARG; }
  if (d->n_sites >= (1u << 31)) { ctx_error(ctx, "n_sites must be < 2^31"); return AIWC_ERR_INVALID_ARG; }
  if (d->n_mem >= (1ull << 32) || d->n_branch >= (1ull << 32)) {
    ctx_error(ctx, "n_mem and n_branch must be < 2^32 per trace");
    return AIWC_ERR_INVALID_ARG;
  }
  if (d->n_opcode_ids == 0 || d->n_opcode_ids > 65536 || !d->opcode_table) {
    ctx_error(ctx, "opcode table needs 1..65536 entries");
    return AIWC_ERR_INVALID_ARG;
  }
  u32 ncls = 0;
  std::vector<u32> info(d->n_opcode_ids);
  for (u32 i = 0; i < d->n_opcode_ids; ++i) {
    const aiwc_opcode_info &e = d->opcode_table[i];
    if (e.kind > AIWC_KIND_OTHER || e.simd_width == 0 || e.op_class == 0xFFFF) {
      ctx_error(ctx, "opcode table entry %u is invalid", i);
      return AIWC_ERR_INVALID_ARG;
    }
    ncls = std::max<u32>(ncls, (u32)e.op_class + 1);
    info[i] = (u32)e.kind | ((u32)e.simd_width << 8) | ((u32)e.op_class << 16);
  }
  HIP_OR(ctx, hipSetDevice(ctx->device));
  aiwc_trace *t = new aiwc_trace();
  t->ctx = ctx;
  t->serial = ++g_trace_serial;
  t->d = *d;
  t->d.opcode_table = nullptr;
  t->n_classes = ncls;
  t->host_info = info;
  if (hipMalloc(&t->dev_info, 4ull * info.size()) != hipSuccess) {
    hipGetLastError();
    delete t;
    ctx_error(ctx, "out of device memory for the opcode table");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(t->dev_info, info.data(), 4ull * info.size(), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(t->dev_info);
    delete t;
    ctx_error(ctx, "copying the opcode table failed");
    return AIWC_ERR_HIP;
  }
  if (d->flags & AIWC_VALIDATE_ON_DEVICE) {
    aiwc_status st = validate_on_device(ctx, t);
    if (st != AIWC_OK) { hipFree(t->dev_info); delete t; return st; }
  }
  *out = t;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_trace_destroy(aiwc_trace *t) {
  if (!t) return AIWC_OK;
  if (t->dev_info) hipFree(t->dev_info);
  delete t;
  return AIWC_OK;
}

// ------------------------------------------------------------ characterize
// Result blocks come in power-of-two sizes from 4 KiB, so that a destroyed
// handle's block serves the next call of any trace of the same size class.
static const size_t POOL_MAX = 64;
static u64 result_class(u64 bytes) {
  u64 c = 4096;
  while (c < bytes) c <<= 1;
  return c;
}

aiwc_status new_metrics(aiwc_ctx *ctx, const aiwc_trace *t, const TracePlan &p,
                        aiwc_metrics **out, SharedBuf *shared, void *buf) {
  aiwc_metrics *m = new aiwc_metrics();
  m->ctx = ctx;
  m->plan = p;
  m->n_classes = t->n_classes;
  if (shared) {
    m->shared = shared;
    m->buf = buf;
    shared->refs += 1;
  } else {
    const u64 cls = result_class(p.result_bytes);
    for (size_t i = ctx->result_pool.size(); i-- > 0;) {
      if (ctx->result_pool[i].first == cls) {
        m->buf = ctx->result_pool[i].second;
        ctx->result_pool.erase(ctx->result_pool.begin() + (long)i);
        break;
      }
    }
    if (!m->buf && hipMalloc(&m->buf, cls) != hipSuccess) {
      hipGetLastError();
      delete m;
      ctx_error(ctx, "out of device memory for a result buffer");
      return AIWC_ERR_OUT_OF_MEMORY;
    }
    m->buf_bytes = cls;
  }
  if (!ctx->event_pool.empty()) {
    m->done = ctx->event_pool.back();
    ctx->event_pool.pop_back();
  } else if (hipEventCreateWithFlags(&m->done, hipEventDisableTiming) != hipSuccess) {
    if (!shared) hipFree(m->buf); else shared->refs -= 1;
    delete m;
    ctx_error(ctx, "hipEventCreate failed");
    return AIWC_ERR_HIP;
  }
  *out = m;
  return AIWC_OK;
}

aiwc_status characterize_planned(aiwc_ctx *ctx, const aiwc_trace *t, u32 pbits,
                                 hipStream_t s, aiwc_metrics **out) {
  TracePlan p;
  plan_trace(t, pbits, p);
  aiwc_status st = ensure_arena(ctx, p.scratch_bytes);
  if (st != AIWC_OK) return st;
  aiwc_metrics *m = nullptr;
  st = new_metrics(ctx, t, p, &m);
  if (st != AIWC_OK) return st;
  if (ctx->last_done) HIP_OR(ctx, hipStreamWaitEvent(s, ctx->last_done, 0));
  TraceArgs a;
  fill_args(t, p, ctx->arena, (char *)m->buf, a);
  StageMarks *pm = nullptr;
  if (ctx->prof.on) { ctx->prof.begin(s); pm = &ctx->prof; }
  BatchDims dims;
  add_dims(t, p, a, dims);
  hipError_t e = enqueue_stages(a, dims, s, pm, side_stream(ctx));
  if (e != hipSuccess) {
    ctx_error(ctx, "kernel launch failed: %s", hipGetErrorString(e));
    aiwc_metrics_destroy(m);
    return AIWC_ERR_HIP;
  }
  HIP_OR(ctx, hipEventRecord(m->done, s));
  if (!ctx->last_done) HIP_OR(ctx, hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming));
  HIP_OR(ctx, hipEventRecord(ctx->last_done, s));
  *out = m;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_characterize(aiwc_ctx *ctx, const aiwc_trace *t, void *stream,
                                         aiwc_metrics **out) {
  if (!ctx || !t || !out) { ctx_error(ctx, "aiwc_characterize: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (t->ctx != ctx) { ctx_error(ctx, "trace belongs to another context"); return AIWC_ERR_INVALID_ARG; }
  HIP_OR(ctx, hipSetDevice(ctx->device));
  u32 pbits = bound_pbits(t->d.n_mem);
  // debug knob: force the partition count (undersizing exercises the
  // overflow -> split -> redo path; results must not change)
  if (const char *e = getenv("AIWC_FORCE_PARTITION_LOG2")) {
    int v = atoi(e);
    if (v >= 4 && v <= 15) pbits = (u32)v;
  }
  return characterize_planned(ctx, t, pbits, (hipStream_t)stream, out);
}

// The allocation-free variant: the plan of aiwc_characterize, its scratch in
// the GPU's static array, the result in the caller's block, the single-stream
// stage order (no side stream or events to create).
static_assert(AIWC_STATIC_CLASS_OFFSET == (sizeof(aiwc_metrics_host) + 32 + 255) / 256 * 256,
              "the static result layout follows the metrics handle's result block");
extern "C" aiwc_status aiwc_characterize_static(aiwc_ctx *ctx, const aiwc_trace *t, void *stream,
                                                void *dev_result, size_t result_bytes) {
  if (!ctx || !t || !dev_result) {
    ctx_error(ctx, "aiwc_characterize_static: NULL argument");
    return AIWC_ERR_INVALID_ARG;
  }
  if (t->ctx != ctx) { ctx_error(ctx, "trace belongs to another context"); return AIWC_ERR_INVALID_ARG; }
  const u64 need_out = AIWC_STATIC_RESULT_BYTES(t->n_classes);
  if (result_bytes < need_out) {
    ctx_error(ctx, "aiwc_characterize_static: result block of %zu bytes, %llu needed for %u classes",
              result_bytes, (unsigned long long)need_out, t->n_classes);
    return AIWC_ERR_INVALID_ARG;
  }
  char *ptr = (char *)static_scratch_ptr(ctx->device);
  if (!ptr) {
    ctx_error(ctx, "aiwc_characterize_static: no static scratch address for device %d", ctx->device);
    return AIWC_ERR_HIP;
  }
  TracePlan p;
  plan_trace(t, bound_pbits(t->d.n_mem), p);
  if (p.scratch_bytes > AIWC_STATIC_SCRATCH_BYTES) {
    ctx_error(ctx, "aiwc_characterize_static: the trace needs %llu bytes of scratch, the static "
              "array holds %llu (use aiwc_characterize)", (unsigned long long)p.scratch_bytes,
              (unsigned long long)AIWC_STATIC_SCRATCH_BYTES);
    return AIWC_ERR_UNSUPPORTED;
  }
  p.spec_export_cap = 0;   // the block holds no spectrum pairs
  HIP_OR(ctx, hipSetDevice(ctx->device));
  TraceArgs a;
  fill_args(t, p, ptr, (char *)dev_result, a);
  BatchDims dims;
  add_dims(t, p, a, dims);
  const hipError_t e = enqueue_stages(a, dims, (hipStream_t)stream, nullptr, nullptr);
  if (e != hipSuccess) {
    ctx_error(ctx, "kernel launch failed: %s", hipGetErrorString(e));
    return AIWC_ERR_HIP;
  }
  return AIWC_OK;
}

// Several invocations as one: their streams are concatenated in a staging
// block owned by the metrics handle, then reduced by the ordinary path.
extern "C" aiwc_status aiwc_characterize_merged(aiwc_ctx *ctx, const aiwc_trace *const *traces,
                                                size_t n, void *stream, aiwc_metrics **out) {
  if (!ctx || !traces || !out || n == 0) {
    ctx_error(ctx, "aiwc_characterize_merged: NULL argument or empty list");
    return AIWC_ERR_INVALID_ARG;
  }
  for (size_t i = 0; i < n; ++i)
    if (!traces[i] || traces[i]->ctx != ctx) {
      ctx_error(ctx, "aiwc_characterize_merged: trace %zu is NULL or belongs to another context", i);
      return AIWC_ERR_INVALID_ARG;
    }
  const aiwc_trace *t0 = traces[0];
  if (n == 1) return aiwc_characterize(ctx, t0, stream, out);
  u64 n_ev = 0, n_wi = 0, n_mem = 0, n_br = 0;
  u32 n_sites = 0;
  for (size_t i = 0; i < n; ++i) {
    const aiwc_trace *t = traces[i];
    const u32 variant = ~(u32)AIWC_VALIDATE_ON_DEVICE;
    if (t->d.history_len != t0->d.history_len || t->host_info != t0->host_info ||
        (t->d.flags & variant) != (t0->d.flags & variant)) {
      ctx_error(ctx, "aiwc_characterize_merged: trace %zu has another opcode table, history "
                "length or branch variant than trace 0", i);
      return AIWC_ERR_INVALID_ARG;
    }
    n_ev += t->d.n_events;
    n_wi += t->d.n_workitems;
    n_mem += t->d.n_mem;
    n_br += t->d.n_branch;
    n_sites = std::max(n_sites, t->d.n_sites);
  }
  if (n_mem >= (1ull << 32) || n_br >= (1ull << 32)) {
    ctx_error(ctx, "aiwc_characterize_merged: summed n_mem and n_branch must be < 2^32");
    return AIWC_ERR_INVALID_ARG;
  }
  auto al = [](u64 x) { return (x + 255) & ~255ull; };
  const u64 o_off = al(2 * n_ev), o_addr = o_off + al(8 * (n_wi + 1));
  const u64 o_kind = o_addr + al(8 * n_mem), o_site = o_kind + al(n_mem);
  const u64 o_taken = o_site + al(4 * n_br), total = o_taken + al(n_br);
  HIP_OR(ctx, hipSetDevice(ctx->device));
  char *stage = nullptr;
  if (hipMalloc(&stage, total) != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of device memory: %llu bytes to stage the merged trace",
              (unsigned long long)total);
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  hipStream_t s = (hipStream_t)stream;
  const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
  hipError_t e = hipSuccess;
  u64 ev = 0, wi = 0, mem = 0, br = 0;
  for (size_t i = 0; i < n && e == hipSuccess; ++i) {
    const aiwc_trace_desc &d = traces[i]->d;
    if (d.n_events) e = hipMemcpyAsync(stage + 2 * ev, d.opcode, 2 * d.n_events, D2D, s);
    if (e == hipSuccess)
      e = aiwc_kernels::launch_merge_offsets((u64 *)(stage + o_off) + wi, (const u64 *)d.wi_offsets,
                                             d.n_workitems, ev, i == 0, s);
    if (e == hipSuccess && d.n_mem) e = hipMemcpyAsync(stage + o_addr + 8 * mem, d.addr, 8 * d.n_mem, D2D, s);
    if (e == hipSuccess && d.n_mem) e = hipMemcpyAsync(stage + o_kind + mem, d.mem_kind, d.n_mem, D2D, s);
    if (e == hipSuccess && d.n_branch) e = hipMemcpyAsync(stage + o_site + 4 * br, d.br_site, 4 * d.n_branch, D2D, s);
    if (e == hipSuccess && d.n_branch) e = hipMemcpyAsync(stage + o_taken + br, d.br_taken, d.n_branch, D2D, s);
    ev += d.n_events;
    wi += d.n_workitems;
    mem += d.n_mem;
    br += d.n_branch;
  }
  if (e != hipSuccess) {
    ctx_error(ctx, "staging the merged trace failed: %s", hipGetErrorString(e));
    hipStreamSynchronize(s);
    hipFree(stage);
    return AIWC_ERR_HIP;
  }
  // the concatenation, with the first invocation's opcode table (borrowed)
  aiwc_trace mt;
  mt.ctx = ctx;
  mt.d = t0->d;
  mt.d.flags = t0->d.flags & ~(u32)AIWC_VALIDATE_ON_DEVICE;
  mt.d.n_events = n_ev;
  mt.d.opcode = (const uint16_t *)stage;
  mt.d.n_workitems = n_wi;
  mt.d.wi_offsets = (const uint64_t *)(stage + o_off);
  mt.d.n_mem = n_mem;
  mt.d.addr = (const uint64_t *)(stage + o_addr);
  mt.d.mem_kind = (const uint8_t *)(stage + o_kind);
  mt.d.n_branch = n_br;
  mt.d.br_site = (const uint32_t *)(stage + o_site);
  mt.d.br_taken = (const uint8_t *)(stage + o_taken);
  mt.d.n_sites = n_sites;
  mt.n_classes = t0->n_classes;
  mt.dev_info = t0->dev_info;
  aiwc_metrics *m = nullptr;
  aiwc_status st = characterize_planned(ctx, &mt, bound_pbits(n_mem), s, &m);
  if (st != AIWC_OK) {
    hipStreamSynchronize(s);
    hipFree(stage);
    return st;
  }
  m->stage = stage;
  *out = m;
  return AIWC_OK;
}

// ------------------------------------------------------------------ metrics
// The result block's metrics struct and its status words (written by
// k_finalize): checks the status words and fills *out.
aiwc_status decode_result(aiwc_ctx *ctx, const char *raw, aiwc_metrics_host *out,
                          u32 spec_pairs[2]) {
  aiwc_metrics_host r;
  memcpy(&r, raw, sizeof r);
  u64 status[4];
  memcpy(status, raw + sizeof(aiwc_metrics_host), sizeof status);
  if (spec_pairs) {
    spec_pairs[0] = (u32)(status[2] & 0xFFFFFFFFu);
    spec_pairs[1] = (u32)(status[2] >> 32);
  }
  if (status[0]) {
    ctx_error(ctx, "trace content is invalid (%llu bad opcode ids / sites / outcomes)",
              (unsigned long long)status[0]);
    return AIWC_ERR_INVALID_ARG;
  }
  if (status[1]) {
    ctx_error(ctx, "opcode kinds disagree with the memory / branch stream lengths");
    return AIWC_ERR_INCONSISTENT;
  }
  if (status[3]) {
    ctx_error(ctx, "internal capacity limit: %llu on-chip table rounds could not be split "
              "further (the metrics would be incomplete)", (unsigned long long)status[3]);
    return AIWC_ERR_UNSUPPORTED;
  }
  *out = r;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_metrics_read(aiwc_metrics *m, aiwc_metrics_host *out) {
  if (!m || !out) { ctx_error(m ? m->ctx : nullptr, "aiwc_metrics_read: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  aiwc_ctx *ctx = m->ctx;
  HIP_OR(ctx, hipEventSynchronize(m->done));
  char h[sizeof(aiwc_metrics_host) + 32];
  HIP_OR(ctx, hipMemcpy(h, (char *)m->buf + m->plan.r_metrics, sizeof h, hipMemcpyDeviceToHost));
  return decode_result(ctx, h, out, m->spec_pairs);
}

extern "C" aiwc_status aiwc_metrics_class_hist(aiwc_metrics *m, uint64_t *out, size_t len) {
  if (!m || (!out && len)) { ctx_error(m ? m->ctx : nullptr, "aiwc_metrics_class_hist: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  aiwc_ctx *ctx = m->ctx;
  HIP_OR(ctx, hipEventSynchronize(m->done));
  std::vector<uint64_t> h(m->n_classes);
  if (m->n_classes)
    HIP_OR(ctx, hipMemcpy(h.data(), (char *)m->buf + m->plan.r_class, 8ull * m->n_classes,
                          hipMemcpyDeviceToHost));
  for (size_t i = 0; i < len; ++i) out[i] = i < h.size() ? h[i] : 0;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_metrics_spectrum(aiwc_metrics *m, int space, uint64_t *f,
                                             uint64_t *mf, size_t cap, size_t *n_out) {
  if (!m || !n_out || space < 0 || space > 1 || (cap && (!f || !mf))) {
    ctx_error(m ? m->ctx : nullptr, "aiwc_metrics_spectrum: invalid argument");
    return AIWC_ERR_INVALID_ARG;
  }
  aiwc_ctx *ctx = m->ctx;
  HIP_OR(ctx, hipEventSynchronize(m->done));
  u64 status[4];
  HIP_OR(ctx, hipMemcpy(status, (char *)m->buf + m->plan.r_metrics + sizeof(aiwc_metrics_host),
                        sizeof status, hipMemcpyDeviceToHost));
  u64 n = space ? (status[2] >> 32) : (status[2] & 0xFFFFFFFFu);
  if (n > m->plan.spec_export_cap) {
    ctx_error(ctx, "spectrum has %llu pairs, more than the %u exported",
              (unsigned long long)n, m->plan.spec_export_cap);
    return AIWC_ERR_UNSUPPORTED;
  }
  std::vector<uint64_t> pairs(2 * n);
  if (n)
    HIP_OR(ctx, hipMemcpy(pairs.data(),
                          (char *)m->buf + m->plan.r_spec + 16ull * space * m->plan.spec_export_cap,
                          16 * n, hipMemcpyDeviceToHost));
  std::vector<std::pair<uint64_t, uint64_t>> v(n);
  for (u64 i = 0; i < n; ++i) v[i] = {pairs[2 * i], pairs[2 * i + 1]};
  std::sort(v.begin(), v.end());
  for (u64 i = 0; i < n && i < cap; ++i) { f[i] = v[i].first; mf[i] = v[i].second; }
  *n_out = n;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_metrics_destroy(aiwc_metrics *m) {
  if (!m) return AIWC_OK;
  aiwc_ctx *ctx = m->ctx;
  if (m->done) {
    hipEventSynchronize(m->done);
    if (ctx->event_pool.size() < POOL_MAX) ctx->event_pool.push_back(m->done);
    else hipEventDestroy(m->done);
  }
  if (m->shared) {
    if (--m->shared->refs == 0) {
      hipFree(m->shared->p);
      delete m->shared;
    }
  } else if (m->buf) {
    if (m->buf_bytes && ctx->result_pool.size() < POOL_MAX) ctx->result_pool.push_back({m->buf_bytes, m->buf});
    else hipFree(m->buf);
  }
  if (m->stage) hipFree(m->stage);
  delete m;
  return AIWC_OK;
}
