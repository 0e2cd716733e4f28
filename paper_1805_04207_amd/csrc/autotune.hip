// autotune.hip -- launch-shape tuning of the per-trace plans.
//
// Traces are grouped into size classes (log2 of events and of memory
// events).  AUTOTUNE_SEARCH times candidate shapes on the largest trace of
// each class not yet in the cache (coordinate descent over the ops task
// size, the number of histogram / scatter blocks and the partition
// granularity; min of two timed runs each, HIP events), keeps the fastest,
// and stores it under "<gfx arch>/<class>".  AUTOTUNE_CACHED only reads the
// cache; AUTOTUNE_OFF uses the built-in shapes.  The cache persists as JSON
// in the file named by the AIWC_TUNE_CACHE environment variable, if set.
// Shapes never change results, only speed.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "abi_internal.h"

namespace {

int ilog2c(u64 x) {
  int b = 0;
  while ((1ull << b) < x + 1 && b < 63) ++b;
  return b;
}

std::string class_key(const aiwc_ctx *ctx, const aiwc_trace *t) {
  char buf[160];
  snprintf(buf, sizeof buf, "%s/e%d/m%d", ctx->arch.c_str(), ilog2c(t->d.n_events),
           ilog2c(t->d.n_mem));
  return buf;
}

const Tune *lookup(const aiwc_ctx *ctx, const std::string &k) {
  for (auto &e : ctx->tune_cache)
    if (e.first == k) return &e.second;
  return nullptr;
}

void load_cache(aiwc_ctx *ctx) {
  if (ctx->tune_loaded) return;
  ctx->tune_loaded = true;
  const char *path = getenv("AIWC_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  // one entry per line: "key": [ops_shift, hist_blocks, part_shift]
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char key[256];
    int a, b, c;
    const char *q = strchr(line, '"');
    if (!q) continue;
    const char *q2 = strchr(q + 1, '"');
    if (!q2 || q2 - q - 1 >= (long)sizeof key) continue;
    memcpy(key, q + 1, q2 - q - 1);
    key[q2 - q - 1] = 0;
    if (sscanf(q2 + 1, " : [%d, %d, %d]", &a, &b, &c) != 3) continue;
    Tune t;
    t.ops_shift = a;
    t.hist_blocks = (u32)b;
    t.part_shift = c;
    ctx->tune_cache.emplace_back(key, t);
  }
  fclose(f);
}

void save_cache(const aiwc_ctx *ctx) {
  const char *path = getenv("AIWC_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t i = 0; i < ctx->tune_cache.size(); ++i) {
    const auto &e = ctx->tune_cache[i];
    fprintf(f, "  \"%s\": [%d, %u, %d]%s\n", e.first.c_str(), e.second.ops_shift,
            e.second.hist_blocks, e.second.part_shift, i + 1 < ctx->tune_cache.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
}

// Wall time (ms) of one full single-trace characterization with a shape.
float time_shape(aiwc_ctx *ctx, const aiwc_trace *t, u32 pbits, const Tune &tune,
                 hipStream_t s, char *result) {
  TracePlan p;
  plan_trace(t, pbits, p, &tune);
  if (ensure_arena(ctx, p.scratch_bytes) != AIWC_OK) return 1e30f;
  TraceArgs a;
  fill_args(t, p, ctx->arena, result, a);
  BatchDims d;
  add_dims(t, p, a, d);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float best = 1e30f;
  for (int r = 0; r < 3; ++r) {
    hipEventRecord(e0, s);
    enqueue_stages(a, d, s, nullptr);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (r > 0) best = std::min(best, ms);   // first run warms up
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return best;
}

}  // namespace

aiwc_status tune_plans(aiwc_ctx *ctx, const aiwc_trace *const *traces, size_t n,
                       const std::vector<u32> &pbits, u32 mode, hipStream_t s,
                       std::vector<TracePlan> &plans) {
  plans.resize(n);
  if (mode != AIWC_AUTOTUNE_OFF) load_cache(ctx);
  if (mode == AIWC_AUTOTUNE_SEARCH) {
    // representative (largest) trace of each class missing from the cache
    std::vector<std::pair<std::string, size_t>> todo;
    for (size_t i = 0; i < n; ++i) {
      const std::string k = class_key(ctx, traces[i]);
      if (lookup(ctx, k)) continue;
      auto it = std::find_if(todo.begin(), todo.end(), [&](auto &e) { return e.first == k; });
      if (it == todo.end()) todo.emplace_back(k, i);
      else if (traces[i]->d.n_events > traces[it->second]->d.n_events) it->second = i;
    }
    if (!todo.empty()) {
      if (ctx->last_done) hipEventSynchronize(ctx->last_done);
      char *result = nullptr;
      TracePlan big;
      u64 rbytes = 0;
      for (auto &e : todo) {
        plan_trace(traces[e.second], pbits[e.second], big);
        rbytes = std::max(rbytes, big.result_bytes);
      }
      if (hipMalloc(&result, rbytes) != hipSuccess) {
        hipGetLastError();
        ctx_error(ctx, "out of device memory for tuning");
        return AIWC_ERR_OUT_OF_MEMORY;
      }
      for (auto &e : todo) {
        const aiwc_trace *t = traces[e.second];
        Tune best;
        float best_ms = time_shape(ctx, t, pbits[e.second], best, s, result);
        const int ops_c[] = {-1, 1};
        const u32 hb_c[] = {128, 512};
        const int ps_c[] = {-1, 1};
        for (int c : ops_c) {
          Tune x = best; x.ops_shift = c;
          float ms = time_shape(ctx, t, pbits[e.second], x, s, result);
          if (ms < best_ms) { best_ms = ms; best = x; }
        }
        for (u32 c : hb_c) {
          Tune x = best; x.hist_blocks = c;
          float ms = time_shape(ctx, t, pbits[e.second], x, s, result);
          if (ms < best_ms) { best_ms = ms; best = x; }
        }
        for (int c : ps_c) {
          Tune x = best; x.part_shift = c;
          float ms = time_shape(ctx, t, pbits[e.second], x, s, result);
          if (ms < best_ms) { best_ms = ms; best = x; }
        }
        ctx->tune_cache.emplace_back(e.first, best);
      }
      hipStreamSynchronize(s);
      hipFree(result);
      save_cache(ctx);
    }
  }
  for (size_t i = 0; i < n; ++i) {
    const Tune *t = mode == AIWC_AUTOTUNE_OFF ? nullptr : lookup(ctx, class_key(ctx, traces[i]));
    plan_trace(traces[i], pbits[i], plans[i], t);
  }
  return AIWC_OK;
}
