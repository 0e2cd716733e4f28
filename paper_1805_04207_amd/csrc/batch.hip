// batch.hip -- aiwc_characterize_batch: many traces, few launches.
//
// The traces are planned individually (partition count from the selected
// sizing policy, launch shapes from the tuning cache), bin-packed into
// admission waves whose summed scratch fits the cap (first fit, largest
// first), and each wave runs every stage as ONE batch-wide launch
// (grid.y = trace, longest trace first; the persistent stages pull their
// work from per-trace queues).  With use_graph the wave's launch sequence is
// captured once into a hipGraph and replayed while the same batch is
// characterized again.  Each trace's arithmetic is exactly the single-trace
// path's, so results are bit-identical to aiwc_characterize.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "abi_internal.h"

namespace {

struct Wave {
  std::vector<u32> idx;          // trace indices (caller order) in launch order
  u64 scratch = 0;               // bytes of scratch of this wave
  u64 res_begin = 0, res_end = 0;  // its results in the stable result region
  BatchDims dims;
  TraceArgs *dev_args = nullptr; // [idx.size()]
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void free_waves(std::vector<Wave> &w) {
  for (Wave &x : w) {
    if (x.exec) hipGraphExecDestroy(x.exec);
    if (x.graph) hipGraphDestroy(x.graph);
    if (x.dev_args) hipFree(x.dev_args);
  }
  w.clear();
}

}  // namespace

struct BatchState {
  // cache key of the prepared batch: the traces' creation serials (a trace
  // destroyed and another created at the same address must not match)
  std::vector<u64> key;
  std::vector<u32> key_pbits;
  u64 key_cap = 0;
  bool key_graph = false;
  char *key_arena = nullptr;     // scratch the cached arguments point into
  std::vector<Wave> waves;
  std::vector<TracePlan> plans;
  char *results = nullptr;       // stable result region written by the kernels
  u64 results_bytes = 0;
  std::vector<u64> res_off;      // per trace offset in the result region
  u64 res_total = 0;
  hipStream_t cap_stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<aiwc_metrics *> last_out;
};

void batch_free(aiwc_ctx *ctx) {
  BatchState *b = ctx->batch;
  if (!b) return;
  free_waves(b->waves);
  if (b->results) hipFree(b->results);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  if (b->done) hipEventDestroy(b->done);
  delete b;
  ctx->batch = nullptr;
}

// partition bits chosen by the sizing policy (sizer.hip)
aiwc_status sizer_plan_pbits(aiwc_ctx *ctx, const aiwc_trace *const *traces, size_t n,
                             u32 mode, hipStream_t s, std::vector<u32> &pbits);
// launch-shape tuning (autotune.hip)
aiwc_status tune_plans(aiwc_ctx *ctx, const aiwc_trace *const *traces, size_t n,
                       const std::vector<u32> &pbits, u32 mode, hipStream_t s,
                       std::vector<TracePlan> &plans);

extern "C" aiwc_status aiwc_characterize_batch(aiwc_ctx *ctx, const aiwc_trace *const *traces,
                                               size_t n, const aiwc_batch_opts *opts,
                                               void *stream, aiwc_metrics **out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!ctx || (n && (!traces || !out)) || !opts) {
    ctx_error(ctx, "aiwc_characterize_batch: NULL argument");
    return AIWC_ERR_INVALID_ARG;
  }
  if (opts->struct_size != sizeof(aiwc_batch_opts) || opts->sizing > AIWC_SIZING_LEARNED ||
      opts->autotune > AIWC_AUTOTUNE_SEARCH) {
    ctx_error(ctx, "aiwc_characterize_batch: bad options");
    return AIWC_ERR_INVALID_ARG;
  }
  for (size_t i = 0; i < n; ++i)
    if (!traces[i] || traces[i]->ctx != ctx) {
      ctx_error(ctx, "trace %zu is NULL or belongs to another context", i);
      return AIWC_ERR_INVALID_ARG;
    }
  if (n == 0) return AIWC_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) { ctx_error(ctx, "hipSetDevice failed"); return AIWC_ERR_HIP; }
  hipStream_t s = (hipStream_t)stream;
  if (!ctx->batch) ctx->batch = new BatchState();
  BatchState &B = *ctx->batch;

  // ---- sizing: partition bits per trace
  std::vector<u32> pbits(n);
  if (opts->force_partition_log2) {
    const u32 f = std::min<u32>(15, std::max<u32>(4, opts->force_partition_log2));
    for (size_t i = 0; i < n; ++i) pbits[i] = f;
  } else {
    aiwc_status st = sizer_plan_pbits(ctx, traces, n, opts->sizing, s, pbits);
    if (st != AIWC_OK) return st;
  }
  const u64 cap = opts->admission_cap_bytes ? opts->admission_cap_bytes : (200ull << 30);
  const bool graph = opts->use_graph != 0;

  std::vector<u64> serials(n);
  for (size_t i = 0; i < n; ++i) serials[i] = traces[i]->serial;
  bool same = graph && B.key_graph && B.key_cap == cap && B.key_arena == ctx->arena &&
              B.key == serials && B.key_pbits == pbits;
  if (!same) {
    if (B.done) hipEventSynchronize(B.done);
    free_waves(B.waves);
    B.plans.clear();
    aiwc_status st = tune_plans(ctx, traces, n, pbits, opts->autotune, s, B.plans);
    if (st != AIWC_OK) return st;
    // ---- admission: first fit, largest scratch first
    std::vector<u32> order(n);
    for (u32 i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](u32 a, u32 b) {
      return B.plans[a].scratch_bytes > B.plans[b].scratch_bytes;
    });
    for (u32 i : order) {
      const u64 need = B.plans[i].scratch_bytes;
      if (need > cap) {
        ctx_error(ctx, "trace %u alone needs %llu bytes of scratch, over the cap of %llu", i,
                  (unsigned long long)need, (unsigned long long)cap);
        return AIWC_ERR_OUT_OF_MEMORY;
      }
      Wave *w = nullptr;
      for (Wave &x : B.waves)
        if (x.scratch + need <= cap) { w = &x; break; }
      if (!w) { B.waves.emplace_back(); w = &B.waves.back(); }
      w->idx.push_back(i);
      w->scratch += need;
    }
    // ---- stable result region, laid out in wave order (one copy per wave)
    B.res_off.assign(n, 0);
    u64 rb = 0;
    for (Wave &w : B.waves) {
      w.res_begin = rb;
      for (u32 i : w.idx) { B.res_off[i] = rb; rb += B.plans[i].result_bytes; }
      w.res_end = rb;
    }
    B.res_total = rb;
    if (rb > B.results_bytes) {
      if (B.results) hipFree(B.results);
      B.results = nullptr;
      B.results_bytes = 0;
      if (hipMalloc(&B.results, rb) != hipSuccess) {
        hipGetLastError();
        ctx_error(ctx, "out of device memory for %llu bytes of batch results", (unsigned long long)rb);
        return AIWC_ERR_OUT_OF_MEMORY;
      }
      B.results_bytes = rb;
    }
    u64 max_scratch = 0;
    for (Wave &w : B.waves) max_scratch = std::max(max_scratch, w.scratch);
    aiwc_status st2 = ensure_arena(ctx, max_scratch);
    if (st2 != AIWC_OK) return st2;
    // ---- per-wave argument arrays (device) and launch shapes
    for (Wave &w : B.waves) {
      std::vector<TraceArgs> args(w.idx.size());
      u64 off = 0;
      for (size_t j = 0; j < w.idx.size(); ++j) {
        const u32 i = w.idx[j];
        fill_args(traces[i], B.plans[i], ctx->arena + off, B.results + B.res_off[i], args[j]);
        add_dims(traces[i], B.plans[i], args[j], w.dims);
        off += B.plans[i].scratch_bytes;
      }
      w.dims.n = (u32)w.idx.size();
      if (hipMalloc(&w.dev_args, sizeof(TraceArgs) * args.size()) != hipSuccess ||
          hipMemcpy(w.dev_args, args.data(), sizeof(TraceArgs) * args.size(),
                    hipMemcpyHostToDevice) != hipSuccess) {
        hipGetLastError();
        ctx_error(ctx, "uploading batch arguments failed");
        return AIWC_ERR_OUT_OF_MEMORY;
      }
      w.dims.batch = w.dev_args;
    }
    B.key = serials;
    B.key_pbits = pbits;
    B.key_cap = cap;
    B.key_graph = graph;
    B.key_arena = ctx->arena;
  }

  // ---- metrics handles: views into one device block per call
  SharedBuf *block = new SharedBuf();
  if (hipMalloc(&block->p, B.res_total) != hipSuccess) {
    hipGetLastError();
    delete block;
    ctx_error(ctx, "out of device memory for batch results");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  std::vector<aiwc_metrics *> ms(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    aiwc_status st = new_metrics(ctx, traces[i], B.plans[i], &ms[i], block,
                                 (char *)block->p + B.res_off[i]);
    if (st != AIWC_OK) {
      for (aiwc_metrics *m : ms) aiwc_metrics_destroy(m);
      if (block->refs == 0) { hipFree(block->p); delete block; }
      return st;
    }
  }
  if (ctx->last_done) hipStreamWaitEvent(s, ctx->last_done, 0);
  TraceArgs dummy;
  memset(&dummy, 0, sizeof dummy);
  if (ctx->prof.on && !graph) ctx->prof.begin(s);   // stage marks of this call only
  for (Wave &w : B.waves) {
    if (graph) {
      if (!w.exec) {
        if (!B.cap_stream) hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking);
        hipStreamSynchronize(s);
        if (hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          ctx_error(ctx, "hipStreamBeginCapture failed");
          return AIWC_ERR_HIP;
        }
        // the side stream joins the capture through the fork event and
        // leaves it through the join event, so the graph holds both chains
        hipError_t e = enqueue_stages(dummy, w.dims, B.cap_stream, nullptr, side_stream(ctx));
        hipError_t e2 = hipStreamEndCapture(B.cap_stream, &w.graph);
        if (e != hipSuccess || e2 != hipSuccess ||
            hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0) != hipSuccess) {
          ctx_error(ctx, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
          return AIWC_ERR_HIP;
        }
      }
      if (hipGraphLaunch(w.exec, s) != hipSuccess) { ctx_error(ctx, "hipGraphLaunch failed"); return AIWC_ERR_HIP; }
    } else {
      hipError_t e = enqueue_stages(dummy, w.dims, s, ctx->prof.on ? &ctx->prof : nullptr,
                                    side_stream(ctx));
      if (e != hipSuccess) { ctx_error(ctx, "batch launch failed: %s", hipGetErrorString(e)); return AIWC_ERR_HIP; }
    }
    // this wave's results into the call's block (the stable region is
    // rewritten by the next call)
    if (w.res_end > w.res_begin)
      hipMemcpyAsync((char *)block->p + w.res_begin, B.results + w.res_begin,
                     w.res_end - w.res_begin, hipMemcpyDeviceToDevice, s);
  }
  for (size_t i = 0; i < n; ++i) hipEventRecord(ms[i]->done, s);
  if (!ctx->last_done) hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming);
  hipEventRecord(ctx->last_done, s);
  if (!B.done) hipEventCreateWithFlags(&B.done, hipEventDisableTiming);
  hipEventRecord(B.done, s);
  if (hipGetLastError() != hipSuccess) { ctx_error(ctx, "batch enqueue failed"); return AIWC_ERR_HIP; }

  aiwc_batch_stats &S = ctx->last_stats;
  memset(&S, 0, sizeof S);
  S.struct_size = sizeof S;
  S.waves = (u32)B.waves.size();
  for (Wave &w : B.waves) S.reserved_bytes = std::max<u64>(S.reserved_bytes, w.scratch);
  for (size_t i = 0; i < n; ++i) S.total_partitions += traces[i]->d.n_mem ? (1ull << B.plans[i].pbits) : 0;
  S.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  B.last_out = ms;
  for (size_t i = 0; i < n; ++i) out[i] = ms[i];
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_batch_last_stats(const aiwc_ctx *cctx, aiwc_batch_stats *out) {
  aiwc_ctx *ctx = (aiwc_ctx *)cctx;
  if (!ctx || !out) { ctx_error(ctx, "aiwc_batch_last_stats: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  aiwc_batch_stats s = ctx->last_stats;
  // redone partitions: read back from the last batch's results
  if (ctx->batch && ctx->batch->done) {
    BatchState &B = *ctx->batch;
    hipEventSynchronize(B.done);
    u64 redos = 0;
    for (size_t i = 0; i < B.key.size() && i < B.res_off.size(); ++i) {
      aiwc_metrics_host h;
      if (hipMemcpy(&h, B.results + B.res_off[i] + B.plans[i].r_metrics, sizeof h,
                    hipMemcpyDeviceToHost) == hipSuccess)
        redos += h.overflow_redos;
    }
    s.redo_partitions = redos;
  }
  *out = s;
  return AIWC_OK;
}
