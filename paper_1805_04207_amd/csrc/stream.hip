// stream.hip -- characterization of a trace that arrives in chunks.
//
// The paper names the memory footprint of full recorded traces as the main
// limit of its tool on large applications (Conclusions) and lists kernels it
// could not characterize at large sizes for that reason (Evaluation).  Here a
// chunk (a run of whole work-items with the memory and branch events they
// issued) is reduced as far as it can be on arrival: its instruction stream
// goes through k_ops into per-stream state (counters, the id histogram, the
// ITB / IPT histograms and large-value lists), so opcodes and work-item
// offsets are never kept; its memory and branch streams are appended to
// device buffers owned by the stream.  aiwc_stream_finish then runs the
// ordinary memory and branch stages and k_finalize over the whole, so the
// result is exactly that of the concatenated trace.
#include <algorithm>
#include <cstring>
#include <vector>

#include "abi_internal.h"

#define ST_HIP_OR(ctx, call)                                                    \
  do {                                                                          \
    hipError_t e__ = (call);                                                    \
    if (e__ != hipSuccess) {                                                    \
      ctx_error(ctx, "%s failed: %s", #call, hipGetErrorString(e__));           \
      return AIWC_ERR_HIP;                                                      \
    }                                                                           \
  } while (0)

namespace {

// A buffer that grows by doubling; `used` bytes survive a move.  It lives in
// device memory, or in pinned host memory for a stream that keeps its
// retained streams off the device until finish.
struct GrowBuf {
  char *p = nullptr;
  u64 cap = 0, used = 0;
  bool host = false;
};

void release(GrowBuf &b) {
  if (b.p) { if (b.host) hipHostFree(b.p); else hipFree(b.p); }
  b.p = nullptr;
  b.cap = b.used = 0;
}

aiwc_status grow(aiwc_ctx *ctx, GrowBuf &b, u64 need, hipStream_t s) {
  if (need <= b.cap) return AIWC_OK;
  const u64 nc = std::max<u64>(need, std::max<u64>(2 * b.cap, 1ull << 16));
  char *np = nullptr;
  const hipError_t e = b.host ? hipHostMalloc((void **)&np, nc, hipHostMallocDefault)
                              : hipMalloc((void **)&np, nc);
  if (e != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of %s memory: a stream buffer of %llu bytes", b.host ? "pinned host" : "device",
              (unsigned long long)nc);
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  if (b.p) {
    if (b.used) ST_HIP_OR(ctx, hipMemcpyAsync(np, b.p, b.used, hipMemcpyDefault, s));
    ST_HIP_OR(ctx, hipStreamSynchronize(s));
    const u64 used = b.used;
    release(b);
    b.used = used;
  }
  b.p = np;
  b.cap = nc;
  return AIWC_OK;
}

aiwc_status append_bytes(aiwc_ctx *ctx, GrowBuf &b, const void *src, u64 bytes, hipStream_t s) {
  if (!bytes) return AIWC_OK;
  aiwc_status st = grow(ctx, b, b.used + bytes, s);
  if (st != AIWC_OK) return st;
  ST_HIP_OR(ctx, hipMemcpyAsync(b.p + b.used, src, bytes, hipMemcpyDefault, s));
  b.used += bytes;
  return AIWC_OK;
}

constexpr u32 VARIANT_FLAGS =
    AIWC_BRANCH_ZERO_HISTORY | AIWC_BRANCH_GLOBAL_HISTORY | AIWC_BRANCH_PATTERN_ENTROPY;

}  // namespace

struct aiwc_stream {
  aiwc_ctx *ctx = nullptr;
  bool started = false, finished = false;
  aiwc_trace proto;                 // opcode table, history length, variant flags
  u64 n_events = 0, n_wi = 0;
  u32 n_sites = 0;
  // instruction-stream state: DevAccum | id_hist | itb_hist | ipt_hist
  char *core = nullptr;
  u64 o_id = 0, o_itb = 0, o_ipt = 0, core_bytes = 0;
  GrowBuf itb_large, ipt_large;     // values >= VAL_DENSE, 8 B each
  GrowBuf addr, kind, site, taken;  // retained memory and branch streams
  GrowBuf staged;                   // device copy of host-held streams at finish
  // out-of-core memory stage
  u64 budget = 0;                   // device bytes for partition records (0: no cap)
  GrowBuf grp;                      // counts | cursors | space totals (device)
  GrowBuf mstage;                   // device chunk of a host-held memory stream
  aiwc_stream_stats stats{};
};

extern "C" aiwc_status aiwc_stream_destroy(aiwc_stream *st);

extern "C" aiwc_status aiwc_stream_create(aiwc_ctx *ctx, uint64_t mem_hint, uint64_t branch_hint,
                                          uint32_t flags, aiwc_stream **out) {
  if (!ctx || !out) { ctx_error(ctx, "aiwc_stream_create: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (flags & ~(u32)AIWC_STREAM_HOST_RETAIN) {
    ctx_error(ctx, "aiwc_stream_create: unknown flag bits 0x%x", flags);
    return AIWC_ERR_INVALID_ARG;
  }
  ST_HIP_OR(ctx, hipSetDevice(ctx->device));
  aiwc_stream *st = new aiwc_stream();
  st->ctx = ctx;
  const bool host = (flags & AIWC_STREAM_HOST_RETAIN) != 0;
  st->addr.host = st->kind.host = st->site.host = st->taken.host = host;
  const u64 mh = std::min<u64>(mem_hint, 1ull << 32), bh = std::min<u64>(branch_hint, 1ull << 32);
  aiwc_status rc = AIWC_OK;
  if (mh && rc == AIWC_OK) rc = grow(ctx, st->addr, 8 * mh, nullptr);
  if (mh && rc == AIWC_OK) rc = grow(ctx, st->kind, mh, nullptr);
  if (bh && rc == AIWC_OK) rc = grow(ctx, st->site, 4 * bh, nullptr);
  if (bh && rc == AIWC_OK) rc = grow(ctx, st->taken, bh, nullptr);
  if (rc != AIWC_OK) {
    aiwc_stream_destroy(st);
    return rc;
  }
  *out = st;
  return AIWC_OK;
}

// The first chunk fixes the table, history length and variant: copy them
// (the chunk's own handle may go away) and set up the zeroed state.
static aiwc_status stream_start(aiwc_stream *st, const aiwc_trace *t, hipStream_t s) {
  aiwc_ctx *ctx = st->ctx;
  st->proto.ctx = ctx;
  st->proto.d = t->d;
  st->proto.d.flags = t->d.flags & VARIANT_FLAGS;
  st->proto.n_classes = t->n_classes;
  st->proto.host_info = t->host_info;
  const u64 ids = t->host_info.size();
  if (hipMalloc(&st->proto.dev_info, 4 * ids) != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of device memory for the stream's opcode table");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(st->proto.dev_info, t->host_info.data(), 4 * ids, hipMemcpyHostToDevice) !=
      hipSuccess) {
    hipFree(st->proto.dev_info);
    st->proto.dev_info = nullptr;
    ctx_error(ctx, "copying the stream's opcode table failed");
    return AIWC_ERR_HIP;
  }
  auto al = [](u64 x) { return (x + 255) & ~255ull; };
  st->o_id = al(sizeof(DevAccum));
  st->o_itb = st->o_id + al(8 * ids);
  st->o_ipt = st->o_itb + al(8ull * VAL_DENSE);
  st->core_bytes = st->o_ipt + al(8ull * VAL_DENSE);
  if (hipMalloc(&st->core, st->core_bytes) != hipSuccess) {
    hipGetLastError();
    hipFree(st->proto.dev_info);
    st->proto.dev_info = nullptr;
    st->core = nullptr;
    ctx_error(ctx, "out of device memory for the stream state");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  TraceArgs z;
  memset(&z, 0, sizeof z);
  z.zero_base = st->core;
  z.zero_bytes = st->core_bytes;
  BatchDims d;
  d.max_zero16 = st->core_bytes / 16;
  ST_HIP_OR(ctx, aiwc_kernels::launch_zero(z, d, s));
  st->started = true;
  return AIWC_OK;
}

// Pointers of the instruction-stream state in a TraceArgs.
static void point_at_state(const aiwc_stream *st, TraceArgs &a) {
  a.acc = (DevAccum *)st->core;
  a.id_hist = (u64 *)(st->core + st->o_id);
  a.itb_hist = (u64 *)(st->core + st->o_itb);
  a.ipt_hist = (u64 *)(st->core + st->o_ipt);
  a.itb_large = (u64 *)st->itb_large.p;
  a.ipt_large = (u64 *)st->ipt_large.p;
  a.large_cap = st->itb_large.cap / 8;
}

extern "C" aiwc_status aiwc_stream_append(aiwc_stream *st, const aiwc_trace *t, void *stream) {
  aiwc_ctx *ctx = st ? st->ctx : nullptr;
  if (!st || !t) { ctx_error(ctx, "aiwc_stream_append: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (t->ctx != ctx) { ctx_error(ctx, "aiwc_stream_append: chunk belongs to another context"); return AIWC_ERR_INVALID_ARG; }
  if (st->finished) { ctx_error(ctx, "aiwc_stream_append: the stream is finished"); return AIWC_ERR_INVALID_ARG; }
  if (st->started && (t->d.history_len != st->proto.d.history_len ||
                      (t->d.flags & VARIANT_FLAGS) != st->proto.d.flags ||
                      t->host_info != st->proto.host_info)) {
    ctx_error(ctx, "aiwc_stream_append: chunk has another opcode table, history length or "
              "branch variant than the stream");
    return AIWC_ERR_INVALID_ARG;
  }
  const aiwc_trace_desc &d = t->d;
  if (st->addr.used / 8 + d.n_mem >= (1ull << 32) || st->taken.used + d.n_branch >= (1ull << 32)) {
    ctx_error(ctx, "aiwc_stream_append: the stream's n_mem and n_branch must stay < 2^32");
    return AIWC_ERR_INVALID_ARG;
  }
  ST_HIP_OR(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  aiwc_status rc = AIWC_OK;
  if (!st->started && (rc = stream_start(st, t, s)) != AIWC_OK) return rc;
  // large ITB / IPT values: at most one per VAL_DENSE instructions, so this
  // capacity can never be exceeded by the stream so far
  // (the device holds the fill counts, so a move copies the whole old list)
  const u64 large = 8 * ((st->n_events + d.n_events) / VAL_DENSE + 1);
  st->itb_large.used = st->itb_large.cap;
  st->ipt_large.used = st->ipt_large.cap;
  if ((rc = grow(ctx, st->itb_large, large, s)) != AIWC_OK) return rc;
  if ((rc = grow(ctx, st->ipt_large, large, s)) != AIWC_OK) return rc;
  // the instruction stream, reduced into the state
  TracePlan p;
  plan_trace(t, 4, p);
  TraceArgs a;
  memset(&a, 0, sizeof a);
  a.opcode = d.opcode;
  a.wi_off = (const u64 *)d.wi_offsets;
  a.op_info = st->proto.dev_info;
  a.n_events = d.n_events;
  a.n_wi = d.n_workitems;
  a.n_ids = d.n_opcode_ids;
  a.ops_task = p.ops_task;
  a.ops_tasks = p.ops_tasks;
  point_at_state(st, a);
  BatchDims dims;
  dims.max_ops_tasks = p.ops_tasks;
  dims.max_ids = d.n_opcode_ids;
  dims.ops_lds = aiwc_kernels::ops_lds_bytes(d.n_opcode_ids);
  dims.ops_vec = ((uintptr_t)d.opcode % 16) == 0;
  ST_HIP_OR(ctx, aiwc_kernels::launch_ops(a, dims, s, nullptr));
  // the memory and branch streams, kept for finish
  if ((rc = append_bytes(ctx, st->addr, d.addr, 8 * d.n_mem, s)) != AIWC_OK) return rc;
  if ((rc = append_bytes(ctx, st->kind, d.mem_kind, d.n_mem, s)) != AIWC_OK) return rc;
  if ((rc = append_bytes(ctx, st->site, d.br_site, 4 * d.n_branch, s)) != AIWC_OK) return rc;
  if ((rc = append_bytes(ctx, st->taken, d.br_taken, d.n_branch, s)) != AIWC_OK) return rc;
  st->n_events += d.n_events;
  st->n_wi += d.n_workitems;
  st->n_sites = std::max(st->n_sites, d.n_sites);
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_stream_set_device_budget(aiwc_stream *st, uint64_t bytes) {
  aiwc_ctx *ctx = st ? st->ctx : nullptr;
  if (!st) { ctx_error(nullptr, "aiwc_stream_set_device_budget: NULL stream"); return AIWC_ERR_INVALID_ARG; }
  if (st->finished) { ctx_error(ctx, "aiwc_stream_set_device_budget: the stream is finished"); return AIWC_ERR_INVALID_ARG; }
  st->budget = bytes;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_stream_get_stats(const aiwc_stream *st, aiwc_stream_stats *out) {
  aiwc_ctx *ctx = st ? st->ctx : nullptr;
  if (!st || !out || out->struct_size != sizeof(aiwc_stream_stats)) {
    ctx_error(ctx, "aiwc_stream_get_stats: NULL argument or struct_size mismatch");
    return AIWC_ERR_INVALID_ARG;
  }
  if (!st->finished) { ctx_error(ctx, "aiwc_stream_get_stats: the stream is not finished"); return AIWC_ERR_INVALID_ARG; }
  *out = st->stats;
  return AIWC_OK;
}

// The memory stage of a finish whose memory stream exceeds the device
// budget: count every partition's records over the retained stream, cut the
// partitions into contiguous groups of at most `cap` records, then per
// group sweep the stream again, scatter the group's records and run the
// bucket kernel over the group's partitions (largest first).  The
// accumulators of all groups add up to those of one pass.
static aiwc_status grouped_memory_stage(aiwc_stream *st, aiwc_trace &mt, u64 cap, hipStream_t s,
                                        aiwc_metrics **out_m, TraceArgs &a, BatchDims &dims) {
  aiwc_ctx *ctx = st->ctx;
  const u64 n_mem = mt.d.n_mem;
  const u32 pbits = bound_pbits(n_mem);
  const u64 P = 1ull << pbits;
  auto al = [](u64 x) { return (x + 255) & ~255ull; };
  const u64 o_cur = al(4 * P), o_tot = o_cur + al(4 * P), gbytes = o_tot + al(sizeof(DevAccum));
  aiwc_status rc = grow(ctx, st->grp, gbytes, s);
  if (rc != AIWC_OK) return rc;
  const bool host = st->addr.host;
  const u64 C = std::min<u64>(n_mem, 1ull << 22);   // records per sweep chunk
  if (host && (rc = grow(ctx, st->mstage, 9 * C, s)) != AIWC_OK) return rc;
  u32 *cnt_d = (u32 *)st->grp.p, *cur_d = (u32 *)(st->grp.p + o_cur);
  DevAccum *tot_d = (DevAccum *)(st->grp.p + o_tot);
  {
    TraceArgs z;
    memset(&z, 0, sizeof z);
    z.zero_base = st->grp.p;
    z.zero_bytes = gbytes;
    BatchDims zd;
    zd.max_zero16 = gbytes / 16;
    ST_HIP_OR(ctx, aiwc_kernels::launch_zero(z, zd, s));
  }
  // one chunk of the retained memory stream as kernel arguments
  auto chunk = [&](u64 i0, TraceArgs &ac) -> hipError_t {
    const u64 n = std::min<u64>(C, n_mem - i0);
    ac.n_mem = n;
    if (!host) {
      ac.addr = (const u64 *)st->addr.p + i0;
      ac.mem_kind = (const uint8_t *)st->kind.p + i0;
      return hipSuccess;
    }
    hipError_t e = hipMemcpyAsync(st->mstage.p, st->addr.p + 8 * i0, 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(st->mstage.p + 8 * C, st->kind.p + i0, n, hipMemcpyHostToDevice, s);
    ac.addr = (const u64 *)st->mstage.p;
    ac.mem_kind = (const uint8_t *)(st->mstage.p + 8 * C);
    return e;
  };
  TraceArgs ac;
  memset(&ac, 0, sizeof ac);
  ac.pbits = pbits;
  ac.acc = tot_d;
  for (u64 i0 = 0; i0 < n_mem; i0 += C) {
    ST_HIP_OR(ctx, chunk(i0, ac));
    ST_HIP_OR(ctx, aiwc_kernels::launch_mem_count(ac, cnt_d, s));
  }
  std::vector<u32> cnt(P);
  ST_HIP_OR(ctx, hipMemcpyAsync(cnt.data(), cnt_d, 4 * P, hipMemcpyDeviceToHost, s));
  ST_HIP_OR(ctx, hipStreamSynchronize(s));
  u64 maxp = 0;
  for (u32 c : cnt) maxp = std::max<u64>(maxp, c);
  const u64 cap_eff = std::max<u64>(cap, maxp);
  std::vector<std::pair<u32, u32>> groups;
  for (u64 p0 = 0, acc = 0, p = 0; p < P; ++p) {
    if (acc + cnt[p] > cap_eff && p > p0) { groups.push_back({(u32)p0, (u32)p}); p0 = p; acc = 0; }
    acc += cnt[p];
    if (p + 1 == P) groups.push_back({(u32)p0, (u32)P});
  }
  // the plan with room for the largest group only
  TracePlan p;
  plan_trace(&mt, pbits, p, nullptr, cap_eff);
  if ((rc = ensure_arena(ctx, p.scratch_bytes)) != AIWC_OK) return rc;
  aiwc_metrics *m = nullptr;
  if ((rc = new_metrics(ctx, &mt, p, &m)) != AIWC_OK) return rc;
  if (ctx->last_done) ST_HIP_OR(ctx, hipStreamWaitEvent(s, ctx->last_done, 0));
  fill_args(&mt, p, ctx->arena, (char *)m->buf, a);
  a.addr = nullptr;        // the memory stream reaches the kernels by chunks only
  a.mem_kind = nullptr;
  a.mem_hot = nullptr;     // groups are reduced without the hot-page path
  a.part_cmp = nullptr;
  point_at_state(st, a);
  add_dims(&mt, p, a, dims);
  hipError_t e = aiwc_kernels::launch_zero(a, dims, s);
  // each space's accesses over the whole stream (the N of every entropy term)
  if (e == hipSuccess)
    e = hipMemcpyAsync(&a.acc->sp_reads[0], &tot_d->sp_reads[0], 4 * sizeof(u64),
                       hipMemcpyDeviceToDevice, s);
  std::vector<u32> off(P + 1), order;
  const u64 zero = 0;
  for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g) {
    const u32 p0 = groups[g].first, p1 = groups[g].second;
    std::fill(off.begin(), off.end(), 0u);
    order.clear();
    u32 run = 0;
    for (u32 q = p0; q < p1; ++q) {
      off[q] = run;
      run += cnt[q];
      if (cnt[q]) order.push_back(q);
    }
    off[p1] = run;
    if (order.empty()) continue;
    std::sort(order.begin(), order.end(), [&](u32 x, u32 y) { return cnt[x] > cnt[y]; });
    // the previous group's kernels read these arrays: wait for them
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(a.part_off, off.data(), 4 * (P + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(a.part_order, order.data(), 4 * order.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(cur_d, off.data(), 4 * P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(&a.acc->mem_queue, &zero, 8, hipMemcpyHostToDevice);
    for (u64 i0 = 0; i0 < n_mem && e == hipSuccess; i0 += C) {
      e = chunk(i0, ac);
      if (e == hipSuccess)
        e = aiwc_kernels::launch_mem_scatter_range(ac, p0, p1, cur_d, a.part_rec, s);
    }
    TraceArgs ag = a;
    ag.part_queue = (u32)order.size();
    if (e == hipSuccess) e = aiwc_kernels::launch_mem_bucket(ag, dims, s, nullptr);
  }
  if (e != hipSuccess) {
    ctx_error(ctx, "the grouped memory stage failed: %s", hipGetErrorString(e));
    hipStreamSynchronize(s);
    aiwc_metrics_destroy(m);
    return AIWC_ERR_HIP;
  }
  st->stats.groups = (u32)groups.size();
  st->stats.device_records = std::min<u64>(n_mem, cap_eff);
  st->stats.largest_partition = maxp;
  *out_m = m;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_stream_finish(aiwc_stream *st, void *stream, aiwc_metrics **out) {
  aiwc_ctx *ctx = st ? st->ctx : nullptr;
  if (!st || !out) { ctx_error(ctx, "aiwc_stream_finish: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (st->finished) { ctx_error(ctx, "aiwc_stream_finish: the stream is finished"); return AIWC_ERR_INVALID_ARG; }
  if (!st->started) { ctx_error(ctx, "aiwc_stream_finish: no chunk was appended"); return AIWC_ERR_INVALID_ARG; }
  ST_HIP_OR(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // the whole trace as the later stages see it: no instruction stream (it
  // is already reduced), the retained memory and branch streams
  aiwc_trace mt;
  mt.ctx = ctx;
  mt.d = st->proto.d;
  mt.d.n_events = st->n_events;
  mt.d.opcode = nullptr;
  mt.d.n_workitems = st->n_wi;
  mt.d.wi_offsets = nullptr;
  mt.d.n_mem = st->kind.used;
  mt.d.addr = (const uint64_t *)st->addr.p;
  mt.d.mem_kind = (const uint8_t *)st->kind.p;
  mt.d.n_branch = st->taken.used;
  mt.d.br_site = (const uint32_t *)st->site.p;
  mt.d.br_taken = (const uint8_t *)st->taken.p;
  st->stats = aiwc_stream_stats{};
  st->stats.struct_size = sizeof(aiwc_stream_stats);
  st->stats.memory_events = mt.d.n_mem;
  const u64 cap = st->budget ? std::max<u64>(1, st->budget / 12) : ~0ull;
  if (mt.d.n_mem > cap) {
    // out of core: the branch stream comes to the device, the memory stream
    // is swept in chunks by the grouped stage
    if (st->site.host) {
      auto al = [](u64 x) { return (x + 255) & ~255ull; };
      const u64 o_taken = al(st->site.used), total = o_taken + al(st->taken.used);
      aiwc_status rc0 = grow(ctx, st->staged, total, s);
      if (rc0 != AIWC_OK) return rc0;
      if (st->site.used)
        ST_HIP_OR(ctx, hipMemcpyAsync(st->staged.p, st->site.p, st->site.used, hipMemcpyHostToDevice, s));
      if (st->taken.used)
        ST_HIP_OR(ctx, hipMemcpyAsync(st->staged.p + o_taken, st->taken.p, st->taken.used,
                                      hipMemcpyHostToDevice, s));
      mt.d.br_site = (const uint32_t *)st->staged.p;
      mt.d.br_taken = (const uint8_t *)(st->staged.p + o_taken);
    }
    mt.d.n_sites = st->n_sites;
    mt.n_classes = st->proto.n_classes;
    mt.dev_info = st->proto.dev_info;
    TraceArgs a;
    BatchDims dims;
    aiwc_metrics *m = nullptr;
    aiwc_status rc = grouped_memory_stage(st, mt, cap, s, &m, a, dims);
    if (rc != AIWC_OK) { mt.dev_info = nullptr; return rc; }
    StageMarks *pm = nullptr;
    if (ctx->prof.on) { ctx->prof.begin(s); pm = &ctx->prof; }
    hipError_t e = aiwc_kernels::launch_branch(a, dims, s, pm);
    if (e == hipSuccess) e = aiwc_kernels::launch_finalize(a, dims, s, pm);
    mt.dev_info = nullptr;
    if (e != hipSuccess) {
      ctx_error(ctx, "kernel launch failed: %s", hipGetErrorString(e));
      aiwc_metrics_destroy(m);
      return AIWC_ERR_HIP;
    }
    ST_HIP_OR(ctx, hipEventRecord(m->done, s));
    if (!ctx->last_done) ST_HIP_OR(ctx, hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming));
    ST_HIP_OR(ctx, hipEventRecord(ctx->last_done, s));
    st->finished = true;
    *out = m;
    return AIWC_OK;
  }
  st->stats.groups = 1;
  st->stats.device_records = mt.d.n_mem;
  if (st->addr.host) {
    // the retained streams come onto the device now, 256-byte aligned
    auto al = [](u64 x) { return (x + 255) & ~255ull; };
    const u64 o_kind = al(st->addr.used), o_site = o_kind + al(st->kind.used);
    const u64 o_taken = o_site + al(st->site.used), total = o_taken + al(st->taken.used);
    aiwc_status rc0 = grow(ctx, st->staged, total, s);
    if (rc0 != AIWC_OK) return rc0;
    char *b = st->staged.p;
    const GrowBuf *src[4] = {&st->addr, &st->kind, &st->site, &st->taken};
    const u64 off[4] = {0, o_kind, o_site, o_taken};
    for (int i = 0; i < 4; ++i)
      if (src[i]->used)
        ST_HIP_OR(ctx, hipMemcpyAsync(b + off[i], src[i]->p, src[i]->used, hipMemcpyHostToDevice, s));
    mt.d.addr = (const uint64_t *)b;
    mt.d.mem_kind = (const uint8_t *)(b + o_kind);
    mt.d.br_site = (const uint32_t *)(b + o_site);
    mt.d.br_taken = (const uint8_t *)(b + o_taken);
  }
  mt.d.n_sites = st->n_sites;
  mt.n_classes = st->proto.n_classes;
  mt.dev_info = st->proto.dev_info;
  TracePlan p;
  plan_trace(&mt, bound_pbits(mt.d.n_mem), p);
  aiwc_status rc = ensure_arena(ctx, p.scratch_bytes);
  if (rc != AIWC_OK) { mt.dev_info = nullptr; return rc; }
  aiwc_metrics *m = nullptr;
  rc = new_metrics(ctx, &mt, p, &m);
  if (rc != AIWC_OK) { mt.dev_info = nullptr; return rc; }
  if (ctx->last_done) ST_HIP_OR(ctx, hipStreamWaitEvent(s, ctx->last_done, 0));
  TraceArgs a;
  fill_args(&mt, p, ctx->arena, (char *)m->buf, a);
  point_at_state(st, a);
  BatchDims dims;
  add_dims(&mt, p, a, dims);
  StageMarks *pm = nullptr;
  if (ctx->prof.on) { ctx->prof.begin(s); pm = &ctx->prof; }
  hipError_t e = aiwc_kernels::launch_zero(a, dims, s);
  if (e == hipSuccess) e = aiwc_kernels::launch_mem(a, dims, s, pm);
  if (e == hipSuccess) e = aiwc_kernels::launch_branch(a, dims, s, pm);
  if (e == hipSuccess) e = aiwc_kernels::launch_finalize(a, dims, s, pm);
  mt.dev_info = nullptr;
  if (e != hipSuccess) {
    ctx_error(ctx, "kernel launch failed: %s", hipGetErrorString(e));
    aiwc_metrics_destroy(m);
    return AIWC_ERR_HIP;
  }
  ST_HIP_OR(ctx, hipEventRecord(m->done, s));
  if (!ctx->last_done) ST_HIP_OR(ctx, hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming));
  ST_HIP_OR(ctx, hipEventRecord(ctx->last_done, s));
  st->finished = true;
  *out = m;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_stream_destroy(aiwc_stream *st) {
  if (!st) return AIWC_OK;
  hipSetDevice(st->ctx->device);
  hipDeviceSynchronize();
  for (GrowBuf *b : {&st->itb_large, &st->ipt_large, &st->addr, &st->kind, &st->site, &st->taken,
                     &st->staged, &st->grp, &st->mstage})
    release(*b);
  if (st->core) hipFree(st->core);
  if (st->proto.dev_info) hipFree(st->proto.dev_info);
  delete st;
  return AIWC_OK;
}
