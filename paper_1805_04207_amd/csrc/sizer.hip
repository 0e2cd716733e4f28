// sizer.hip -- the learned sizing part: prefix features, a small MLP with
// hand-written forward / backward / Adam kernels, and the sizing policies
// that turn predicted distinct-address counts into partition counts.
//
// Network: 40 -> 64 -> 64 -> 64 -> 11, exact (erf) GELU on the hidden
// layers, weights stored as bf16 (fp32 master copy for Adam), activations
// and accumulation in fp32.  Inputs are z-scored features of the first
// memory events of a trace; outputs are z-scored log2(1 + distinct_k) of
// the global address space, k = 0..10.  Predictions only size partitions;
// an undersized partition is split and redone by the memory kernels, so the
// metrics never depend on the network.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "abi_internal.h"

namespace {

constexpr int NF = AIWC_N_FEATURES;   // 40
constexpr int NT = AIWC_N_TARGETS;    // 11
constexpr int NH = AIWC_MLP_HIDDEN;   // 64
// parameter layout (fp32 view, in this order)
constexpr int O_W1 = 0, O_B1 = O_W1 + NH * NF;
constexpr int O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH;
constexpr int O_W3 = O_B2 + NH, O_B3 = O_W3 + NH * NH;
constexpr int O_W4 = O_B3 + NH, O_B4 = O_W4 + NT * NH;
constexpr int NPARAM = O_B4 + NT;     // 11659
constexpr int NNORM = 2 * NF + 2 * NT;
constexpr int PREFIX = 8192;          // memory events used for the features
constexpr u32 FT_SLOTS = 16384;       // LDS table for the prefix distinct counts

// ------------------------------------------------------------- bf16 helpers
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(r >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// ------------------------------------------------------------------ features
struct FeatShared {
  u64 key[FT_SLOTS];
  u32 claimed;
  u32 red[32];
  u64 mn[2], mx[2];
};

__device__ void ft_insert(FeatShared &S, u64 key) {
  u32 slot = hash_slot(key, FT_SLOTS);
  while (true) {
    u64 w = S.key[slot];
    if (w == key) return;
    if (w == ~0ull) {
      u64 old = atomicCAS(&S.key[slot], ~0ull, key);
      if (old == ~0ull) { atomicAdd(&S.claimed, 1u); return; }
      if (old == key) return;
    }
    slot = (slot + 1 == FT_SLOTS) ? 0 : slot + 1;
  }
}

__device__ float flog2p1(double x) { return (float)log2(1.0 + x); }

// One block per trace: raw features into out[40].
// One block per trace (blockIdx.x) and per (skip, space) pair of the prefix
// distinct counts (blockIdx.y = 2 * skip + space): the 22 counts are
// independent, so they run side by side; block y = 0 also takes the scalar
// counts and the growth curve.
__global__ void __launch_bounds__(1024) k_features(const TraceArgs *batch, float *out) {
  __shared__ FeatShared S;
  const TraceArgs &A = batch[blockIdx.x];
  float *f = out + (u64)blockIdx.x * NF;
  const int tid = threadIdx.x;
  const u32 np = (u32)(A.n_mem < PREFIX ? A.n_mem : PREFIX);
  const int k = (int)blockIdx.y >> 1, sp = (int)blockIdx.y & 1;
  const bool first = blockIdx.y == 0;
  if (first) {
    // scalar counts of the prefix
    u32 nloc = 0, nwr = 0, nal = 0, near = 0;
    u64 mn0 = ~0ull, mx0 = 0, mn1 = ~0ull, mx1 = 0;
    for (u32 i = tid; i < np; i += 1024) {
      const u64 a = A.addr[i];
      const uint8_t kd = A.mem_kind[i];
      nloc += (kd >> 1) & 1u;
      nwr += kd & 1u;
      nal += (a & 3ull) == 0;
      if (i > 0) {
        const u64 b = A.addr[i - 1];
        const u64 d = a > b ? a - b : b - a;
        near += d <= 256;
      }
      if (kd & 2u) { mn1 = a < mn1 ? a : mn1; mx1 = a > mx1 ? a : mx1; }
      else { mn0 = a < mn0 ? a : mn0; mx0 = a > mx0 ? a : mx0; }
    }
    if (tid < 2) { S.mn[tid] = ~0ull; S.mx[tid] = 0; }
    if (tid < 32) S.red[tid] = 0;
    __syncthreads();
    u32 v4[4] = {nloc, nwr, nal, near};
    for (int j = 0; j < 4; ++j) {
      u32 x = (u32)wave_sum_u64(v4[j]);
      if (lane_id() == 0 && x) atomicAdd(&S.red[j], x);
    }
    if (mn0 != ~0ull) { atomicMin(&S.mn[0], mn0); atomicMax(&S.mx[0], mx0); }
    if (mn1 != ~0ull) { atomicMin(&S.mn[1], mn1); atomicMax(&S.mx[1], mx1); }
    __syncthreads();
  }
  // the distinct count of this block's (skip, space) over the prefix; the
  // growth curve at skip 0 in space 0
  float grow[4];
  for (u32 i = tid; i < FT_SLOTS; i += 1024) S.key[i] = ~0ull;
  if (tid == 0) S.claimed = 0;
  __syncthreads();
  const u32 stops[4] = {1024, 2048, 4096, 8192};
  u32 done = 0;
  for (int g = 0; g < 4; ++g) {
    const u32 end = stops[g] < np ? stops[g] : np;
    for (u32 i = done + tid; i < end; i += 1024) {
      const uint8_t kk = A.mem_kind[i];
      if ((int)((kk >> 1) & 1u) != sp) continue;
      ft_insert(S, A.addr[i] >> k);
    }
    done = end > done ? end : done;
    __syncthreads();
    if (first) grow[g] = flog2p1((double)S.claimed);
    __syncthreads();
  }
  const float dist = flog2p1((double)S.claimed);
  if (tid != 0) return;
  f[(sp ? 19 : 8) + k] = dist;
  if (!first) return;
  const double npd = np ? (double)np : 1.0;
  f[0] = flog2p1((double)A.n_events);
  f[1] = flog2p1((double)A.n_mem);
  f[2] = flog2p1((double)A.n_wi);
  f[3] = flog2p1((double)A.wg_size);
  f[4] = flog2p1((double)A.n_branch);
  f[5] = flog2p1((double)A.n_sites);
  f[6] = (float)(S.red[0] / npd);
  f[7] = (float)(S.red[1] / npd);
  for (int g = 0; g < 4; ++g) f[30 + g] = grow[g];
  f[34] = flog2p1(npd);
  f[35] = S.mx[0] >= S.mn[0] && S.mn[0] != ~0ull ? flog2p1((double)(S.mx[0] - S.mn[0])) : 0.f;
  f[36] = S.mx[1] >= S.mn[1] && S.mn[1] != ~0ull ? flog2p1((double)(S.mx[1] - S.mn[1])) : 0.f;
  f[37] = (float)(S.red[2] / npd);
  f[38] = (float)(S.red[3] / npd);
  f[39] = (float)log2((double)(A.n_mem ? A.n_mem : 1) / npd);
}

// --------------------------------------------------------------- MLP kernels
__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// Activation cache per sample: z1,a1,z2,a2,z3,a3 (64 each) then out (11).
constexpr int ACT = 6 * NH + NT;

// Forward: one 64-thread block per sample.  x: [n][NF] normalized input;
// wb: bf16 weights in the fp32 layout order.
__global__ void __launch_bounds__(64) k_mlp_fwd(const float *x, const uint16_t *wb, u64 n,
                                                float *act, float *yout) {
  __shared__ float in[NH];
  __shared__ float h[NH];
  const u64 s = blockIdx.x;
  if (s >= n) return;
  const int j = threadIdx.x;
  float *A = act ? act + s * ACT : nullptr;
  if (j < NF) in[j] = x[s * NF + j];
  __syncthreads();
  // layer 1
  float z = bf16_to_f32(wb[O_B1 + j]);
  for (int i = 0; i < NF; ++i) z += bf16_to_f32(wb[O_W1 + j * NF + i]) * in[i];
  float a = gelu(z);
  if (A) { A[j] = z; A[NH + j] = a; }
  h[j] = a;
  __syncthreads();
  // layers 2, 3
  for (int l = 0; l < 2; ++l) {
    const int ow = l == 0 ? O_W2 : O_W3, ob = l == 0 ? O_B2 : O_B3;
    float zz = bf16_to_f32(wb[ob + j]);
    for (int i = 0; i < NH; ++i) zz += bf16_to_f32(wb[ow + j * NH + i]) * h[i];
    const float aa = gelu(zz);
    __syncthreads();
    h[j] = aa;
    if (A) { A[(2 + 2 * l) * NH + j] = zz; A[(3 + 2 * l) * NH + j] = aa; }
    __syncthreads();
  }
  if (j < NT) {
    float o = bf16_to_f32(wb[O_B4 + j]);
    for (int i = 0; i < NH; ++i) o += bf16_to_f32(wb[O_W4 + j * NH + i]) * h[i];
    if (A) A[6 * NH + j] = o;
    if (yout) yout[s * NT + j] = o;
  }
}

// Backward deltas per sample (loss = mean over n * NT of squared error):
// writes d4[NT], d3[NH], d2[NH], d1[NH] into dl[s][..] and the squared error.
constexpr int DL = 3 * NH + NT;
__global__ void __launch_bounds__(64) k_mlp_bwd(const float *y, const uint16_t *wb, u64 n,
                                                const float *act, float *dl, float *sqerr) {
  __shared__ float d[NH];
  __shared__ float dn[NH];
  const u64 s = blockIdx.x;
  if (s >= n) return;
  const int j = threadIdx.x;
  const float *A = act + s * ACT;
  float *D = dl + s * DL;
  const float scale = 2.0f / (float)(n * NT);
  if (j < NT) {
    const float e = A[6 * NH + j] - y[s * NT + j];
    d[j] = scale * e;
    D[3 * NH + j] = d[j];
    sqerr[s * NT + j] = e * e;
  }
  __syncthreads();
  // layer 3 delta = (W4^T d4) * gelu'(z3)
  float g = 0.f;
  for (int o = 0; o < NT; ++o) g += bf16_to_f32(wb[O_W4 + o * NH + j]) * d[o];
  g *= gelu_grad(A[4 * NH + j]);
  __syncthreads();
  dn[j] = g;
  D[2 * NH + j] = g;
  __syncthreads();
  for (int l = 1; l >= 0; --l) {           // deltas of layers 2 then 1
    const int ow = l == 1 ? O_W3 : O_W2;
    float gg = 0.f;
    for (int o = 0; o < NH; ++o) gg += bf16_to_f32(wb[ow + o * NH + j]) * dn[o];
    gg *= gelu_grad(A[(2 * l) * NH + j]);
    __syncthreads();
    dn[j] = gg;
    D[l * NH + j] = gg;
    __syncthreads();
  }
}

// Parameter gradients: one thread per parameter, sum over the batch in a
// fixed order (deterministic).
__global__ void k_mlp_wgrad(const float *x, const float *act, const float *dl, u64 n,
                            float *grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  int layer, j, i = -1, fan;
  if (p < O_B1) { layer = 0; j = p / NF; i = p % NF; fan = NF; }
  else if (p < O_W2) { layer = 0; j = p - O_B1; fan = NF; }
  else if (p < O_B2) { layer = 1; j = (p - O_W2) / NH; i = (p - O_W2) % NH; fan = NH; }
  else if (p < O_W3) { layer = 1; j = p - O_B2; fan = NH; }
  else if (p < O_B3) { layer = 2; j = (p - O_W3) / NH; i = (p - O_W3) % NH; fan = NH; }
  else if (p < O_W4) { layer = 2; j = p - O_B3; fan = NH; }
  else if (p < O_B4) { layer = 3; j = (p - O_W4) / NH; i = (p - O_W4) % NH; fan = NH; }
  else { layer = 3; j = p - O_B4; fan = NH; }
  (void)fan;
  float g = 0.f;
  for (u64 s = 0; s < n; ++s) {
    const float *D = dl + s * DL;
    const float dj = layer == 3 ? D[3 * NH + j] : D[layer * NH + j];
    float in = 1.f;
    if (i >= 0) in = layer == 0 ? x[s * NF + i] : act[s * ACT + (2 * layer - 1) * NH + i];
    g += dj * in;
  }
  grad[p] = g;
}

__global__ void k_adam(float *master, uint16_t *wb, float *m, float *v, const float *g,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float w = master[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
  master[p] = w;
  wb[p] = f32_to_bf16(w);
}

// z-score statistics of the columns of x[n][c] (population SD, floored).
__global__ void k_colstats(const float *x, u64 n, int c, float *mean, float *sd) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c) return;
  double s = 0.0, q = 0.0;
  for (u64 r = 0; r < n; ++r) { const double v = x[r * c + j]; s += v; q += v * v; }
  const double mu = s / (double)n;
  double var = q / (double)n - mu * mu;
  mean[j] = (float)mu;
  sd[j] = (float)sqrt(var > 1e-8 ? var : 1e-8);
}

__global__ void k_normalize(const float *x, u64 n, int c, const float *mean, const float *sd,
                            float *out) {
  const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * c) return;
  const int j = (int)(i % c);
  out[i] = (x[i] - mean[j]) / sd[j];
}

__global__ void k_denormalize(float *y, u64 n, const float *mean, const float *sd) {
  const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * NT) return;
  const int j = (int)(i % NT);
  y[i] = y[i] * sd[j] + mean[j];
}

__global__ void k_gather(const float *src, const u32 *idx, u64 n, int c, float *dst) {
  const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * c) return;
  dst[i] = src[(u64)idx[i / c] * c + (i % c)];
}

__global__ void k_sum(const float *x, u64 n, float *out) {
  __shared__ double part[256];
  double s = 0.0;
  for (u64 i = threadIdx.x; i < n; i += 256) s += x[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)part[0];
}

}  // namespace

// ---------------------------------------------------------------- host side
struct SizerState {
  std::vector<float> master;      // fp32 master weights
  std::vector<float> norm;        // x_mean, x_std, y_mean, y_std
  float margin = 0.5f;            // log2 units added before sizing
  bool trained = false;
  // device copies
  float *d_master = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
  uint16_t *d_wb = nullptr;
  float *d_norm = nullptr;
  bool dirty = true;              // host params newer than device
};

static void sizer_default_init(SizerState &S, u32 seed) {
  S.master.assign(NPARAM, 0.f);
  std::mt19937 rng(seed);
  auto fill = [&](int off, int fan_out, int fan_in) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.0f / (float)fan_in));
    for (int k = 0; k < fan_out * fan_in; ++k) S.master[off + k] = nd(rng);
  };
  fill(O_W1, NH, NF);
  fill(O_W2, NH, NH);
  fill(O_W3, NH, NH);
  fill(O_W4, NT, NH);
  for (int k = 0; k < NPARAM; ++k) S.master[k] = bf16_to_f32(f32_to_bf16(S.master[k]));
  S.norm.assign(NNORM, 0.f);
  for (int j = 0; j < NF; ++j) S.norm[NF + j] = 1.f;
  for (int j = 0; j < NT; ++j) S.norm[2 * NF + NT + j] = 1.f;
  S.dirty = true;
}

void sizer_init(aiwc_ctx *ctx) {
  ctx->sizer = new SizerState();
  sizer_default_init(*ctx->sizer, 1234u);
}

void sizer_free(aiwc_ctx *ctx) {
  SizerState *S = ctx->sizer;
  if (!S) return;
  hipFree(S->d_master); hipFree(S->d_m); hipFree(S->d_v); hipFree(S->d_g);
  hipFree(S->d_wb); hipFree(S->d_norm);
  delete S;
  ctx->sizer = nullptr;
}

static aiwc_status sizer_upload(aiwc_ctx *ctx) {
  SizerState &S = *ctx->sizer;
  if (!S.d_master) {
    if (hipMalloc(&S.d_master, 4 * NPARAM) != hipSuccess || hipMalloc(&S.d_m, 4 * NPARAM) != hipSuccess ||
        hipMalloc(&S.d_v, 4 * NPARAM) != hipSuccess || hipMalloc(&S.d_g, 4 * NPARAM) != hipSuccess ||
        hipMalloc(&S.d_wb, 2 * NPARAM) != hipSuccess || hipMalloc(&S.d_norm, 4 * NNORM) != hipSuccess) {
      hipGetLastError();
      ctx_error(ctx, "out of device memory for the sizing network");
      return AIWC_ERR_OUT_OF_MEMORY;
    }
  }
  if (S.dirty) {
    std::vector<uint16_t> wb(NPARAM);
    for (int k = 0; k < NPARAM; ++k) wb[k] = f32_to_bf16(S.master[k]);
    hipMemcpy(S.d_master, S.master.data(), 4 * NPARAM, hipMemcpyHostToDevice);
    hipMemcpy(S.d_wb, wb.data(), 2 * NPARAM, hipMemcpyHostToDevice);
    hipMemcpy(S.d_norm, S.norm.data(), 4 * NNORM, hipMemcpyHostToDevice);
    S.dirty = false;
  }
  return AIWC_OK;
}

static aiwc_status sizer_download(aiwc_ctx *ctx) {
  SizerState &S = *ctx->sizer;
  if (!S.d_master || S.dirty) return AIWC_OK;
  hipMemcpy(S.master.data(), S.d_master, 4 * NPARAM, hipMemcpyDeviceToHost);
  hipMemcpy(S.norm.data(), S.d_norm, 4 * NNORM, hipMemcpyDeviceToHost);
  return AIWC_OK;
}

// Device features of n traces into dev_out[n][40].
static aiwc_status features_impl(aiwc_ctx *ctx, const aiwc_trace *const *traces, size_t n,
                                 hipStream_t s, float *dev_out) {
  std::vector<TraceArgs> args(n);
  for (size_t i = 0; i < n; ++i) {
    TracePlan p;
    plan_trace(traces[i], 4, p);
    fill_args(traces[i], p, nullptr, nullptr, args[i]);
    args[i].wg_size = traces[i]->d.wg_size;
  }
  TraceArgs *d = nullptr;
  if (hipMalloc(&d, sizeof(TraceArgs) * n) != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of device memory for feature arguments");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  hipMemcpy(d, args.data(), sizeof(TraceArgs) * n, hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_features, dim3((unsigned)n, 2 * AIWC_NSKIP), dim3(1024), 0, s, d, dev_out);
  hipError_t e = hipStreamSynchronize(s);
  hipFree(d);
  if (e != hipSuccess || hipGetLastError() != hipSuccess) {
    ctx_error(ctx, "feature kernel failed");
    return AIWC_ERR_HIP;
  }
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_features(aiwc_ctx *ctx, const aiwc_trace *const *traces,
                                           size_t n, void *stream, float *dev_out) {
  if (!ctx || (n && (!traces || !dev_out))) { ctx_error(ctx, "aiwc_sizer_features: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  for (size_t i = 0; i < n; ++i)
    if (!traces[i] || traces[i]->ctx != ctx) { ctx_error(ctx, "bad trace %zu", i); return AIWC_ERR_INVALID_ARG; }
  if (n == 0) return AIWC_OK;
  hipSetDevice(ctx->device);
  return features_impl(ctx, traces, n, (hipStream_t)stream, dev_out);
}

extern "C" size_t aiwc_sizer_num_params(void) { return NPARAM + NNORM; }

extern "C" aiwc_status aiwc_sizer_get_params(const aiwc_ctx *cctx, float *host) {
  aiwc_ctx *ctx = (aiwc_ctx *)cctx;
  if (!ctx || !host) { ctx_error(ctx, "aiwc_sizer_get_params: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  sizer_download(ctx);
  SizerState &S = *ctx->sizer;
  for (int k = 0; k < NPARAM; ++k) host[k] = bf16_to_f32(f32_to_bf16(S.master[k]));
  memcpy(host + NPARAM, S.norm.data(), 4 * NNORM);
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_set_params(aiwc_ctx *ctx, const float *host) {
  if (!ctx || !host) { ctx_error(ctx, "aiwc_sizer_set_params: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  SizerState &S = *ctx->sizer;
  for (int k = 0; k < NPARAM; ++k) S.master[k] = bf16_to_f32(f32_to_bf16(host[k]));
  memcpy(S.norm.data(), host + NPARAM, 4 * NNORM);
  S.dirty = true;
  S.trained = true;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_set_margin(aiwc_ctx *ctx, float margin) {
  if (!ctx || !(margin > -8.f && margin < 8.f)) { ctx_error(ctx, "bad margin"); return AIWC_ERR_INVALID_ARG; }
  ctx->sizer->margin = margin;
  return AIWC_OK;
}

// forward (+ backward) on normalized data already on the device
static aiwc_status run_fwd_bwd(aiwc_ctx *ctx, const float *xn, const float *yn, u64 n,
                               hipStream_t s, float *act, float *dl, float *sq, bool grads) {
  SizerState &S = *ctx->sizer;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)n), dim3(64), 0, s, xn, S.d_wb, n, act, nullptr);
  if (grads) {
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)n), dim3(64), 0, s, yn, S.d_wb, n, act, dl, sq);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((NPARAM + 255) / 256), dim3(256), 0, s, xn, act, dl, n,
                       S.d_g);
  }
  return hipGetLastError() == hipSuccess ? AIWC_OK : AIWC_ERR_HIP;
}

extern "C" aiwc_status aiwc_sizer_grad(aiwc_ctx *ctx, const float *dev_xn, const float *dev_yn,
                                       size_t n, void *stream, float *loss, float *host_grad) {
  if (!ctx || !dev_xn || !dev_yn || !n || !loss || !host_grad) { ctx_error(ctx, "aiwc_sizer_grad: bad argument"); return AIWC_ERR_INVALID_ARG; }
  hipSetDevice(ctx->device);
  aiwc_status st = sizer_upload(ctx);
  if (st != AIWC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  float *act = nullptr, *dl = nullptr, *sq = nullptr, *tot = nullptr;
  if (hipMalloc(&act, 4 * n * ACT) != hipSuccess || hipMalloc(&dl, 4 * n * DL) != hipSuccess ||
      hipMalloc(&sq, 4 * n * NT) != hipSuccess || hipMalloc(&tot, 4) != hipSuccess) {
    hipGetLastError();
    hipFree(act); hipFree(dl); hipFree(sq);
    ctx_error(ctx, "out of device memory");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  run_fwd_bwd(ctx, dev_xn, dev_yn, n, s, act, dl, sq, true);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, sq, (u64)n * NT, tot);
  float t = 0.f;
  hipStreamSynchronize(s);
  hipMemcpy(&t, tot, 4, hipMemcpyDeviceToHost);
  hipMemcpy(host_grad, ctx->sizer->d_g, 4 * NPARAM, hipMemcpyDeviceToHost);
  hipFree(act); hipFree(dl); hipFree(sq); hipFree(tot);
  *loss = t / (float)(n * NT);
  return hipGetLastError() == hipSuccess ? AIWC_OK : AIWC_ERR_HIP;
}

extern "C" aiwc_status aiwc_sizer_train(aiwc_ctx *ctx, const float *dev_x, const float *dev_y,
                                        size_t n, const aiwc_train_opts *o, void *stream,
                                        float *loss_out) {
  if (!ctx || !dev_x || !dev_y || n < 2 || !o || o->struct_size != sizeof(aiwc_train_opts) ||
      o->batch == 0 || o->epochs == 0) {
    ctx_error(ctx, "aiwc_sizer_train: bad argument");
    return AIWC_ERR_INVALID_ARG;
  }
  hipSetDevice(ctx->device);
  SizerState &S = *ctx->sizer;
  sizer_default_init(S, o->seed);
  aiwc_status st = sizer_upload(ctx);
  if (st != AIWC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const u64 B = std::min<u64>(o->batch, n);
  float *xn = nullptr, *yn = nullptr, *bx = nullptr, *by = nullptr, *act = nullptr, *dl = nullptr,
        *sq = nullptr, *tot = nullptr;
  u32 *idx = nullptr;
  bool ok = hipMalloc(&xn, 4 * n * NF) == hipSuccess && hipMalloc(&yn, 4 * n * NT) == hipSuccess &&
            hipMalloc(&bx, 4 * B * NF) == hipSuccess && hipMalloc(&by, 4 * B * NT) == hipSuccess &&
            hipMalloc(&act, 4 * B * ACT) == hipSuccess && hipMalloc(&dl, 4 * B * DL) == hipSuccess &&
            hipMalloc(&sq, 4 * B * NT) == hipSuccess && hipMalloc(&tot, 4) == hipSuccess &&
            hipMalloc(&idx, 4 * n) == hipSuccess;
  auto cleanup = [&]() {
    hipFree(xn); hipFree(yn); hipFree(bx); hipFree(by); hipFree(act); hipFree(dl);
    hipFree(sq); hipFree(tot); hipFree(idx);
  };
  if (!ok) { hipGetLastError(); cleanup(); ctx_error(ctx, "out of device memory for training"); return AIWC_ERR_OUT_OF_MEMORY; }
  // normalization statistics of this training set, then z-scored copies
  float *nm = S.d_norm;
  hipLaunchKernelGGL(k_colstats, dim3(1), dim3(64), 0, s, dev_x, (u64)n, NF, nm, nm + NF);
  hipLaunchKernelGGL(k_colstats, dim3(1), dim3(64), 0, s, dev_y, (u64)n, NT, nm + 2 * NF,
                     nm + 2 * NF + NT);
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n * NF + 255) / 256)), dim3(256), 0, s, dev_x,
                     (u64)n, NF, nm, nm + NF, xn);
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n * NT + 255) / 256)), dim3(256), 0, s, dev_y,
                     (u64)n, NT, nm + 2 * NF, nm + 2 * NF + NT, yn);
  hipMemsetAsync(S.d_m, 0, 4 * NPARAM, s);
  hipMemsetAsync(S.d_v, 0, 4 * NPARAM, s);
  std::mt19937 rng(o->seed ^ 0x5EEDu);
  std::vector<u32> perm(n);
  for (u32 i = 0; i < n; ++i) perm[i] = i;
  const float lr = o->lr > 0 ? o->lr : 1e-3f, b1 = o->beta1 > 0 ? o->beta1 : 0.9f;
  const float b2 = o->beta2 > 0 ? o->beta2 : 0.999f, eps = o->eps > 0 ? o->eps : 1e-8f;
  u64 step = 0;
  double last_loss = 0.0;
  for (u32 ep = 0; ep < o->epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    hipMemcpyAsync(idx, perm.data(), 4 * n, hipMemcpyHostToDevice, s);
    hipStreamSynchronize(s);
    double ep_sum = 0.0;
    u64 ep_cnt = 0;
    for (u64 b0 = 0; b0 + B <= n; b0 += B) {
      hipLaunchKernelGGL(k_gather, dim3((unsigned)((B * NF + 255) / 256)), dim3(256), 0, s, xn,
                         idx + b0, B, NF, bx);
      hipLaunchKernelGGL(k_gather, dim3((unsigned)((B * NT + 255) / 256)), dim3(256), 0, s, yn,
                         idx + b0, B, NT, by);
      run_fwd_bwd(ctx, bx, by, B, s, act, dl, sq, true);
      ++step;
      const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
      hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, S.d_master, S.d_wb,
                         S.d_m, S.d_v, S.d_g, lr, b1, b2, eps, c1, c2);
      if (ep + 1 == o->epochs) {
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, sq, B * NT, tot);
        float t = 0.f;
        hipMemcpyAsync(&t, tot, 4, hipMemcpyDeviceToHost, s);
        hipStreamSynchronize(s);
        ep_sum += t;
        ep_cnt += B * NT;
      }
    }
    if (ep_cnt) last_loss = ep_sum / (double)ep_cnt;
  }
  hipError_t e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess || hipGetLastError() != hipSuccess) { ctx_error(ctx, "training kernels failed"); return AIWC_ERR_HIP; }
  S.trained = true;
  sizer_download(ctx);
  if (loss_out) *loss_out = (float)last_loss;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_predict(aiwc_ctx *ctx, const float *dev_x, size_t n,
                                          void *stream, float *dev_y) {
  if (!ctx || !dev_x || !dev_y) { ctx_error(ctx, "aiwc_sizer_predict: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (n == 0) return AIWC_OK;
  hipSetDevice(ctx->device);
  aiwc_status st = sizer_upload(ctx);
  if (st != AIWC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  SizerState &S = *ctx->sizer;
  float *xn = nullptr;
  if (hipMalloc(&xn, 4 * n * NF) != hipSuccess) { hipGetLastError(); ctx_error(ctx, "out of device memory"); return AIWC_ERR_OUT_OF_MEMORY; }
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n * NF + 255) / 256)), dim3(256), 0, s, dev_x,
                     (u64)n, NF, S.d_norm, S.d_norm + NF, xn);
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)n), dim3(64), 0, s, xn, S.d_wb, (u64)n, nullptr, dev_y);
  hipLaunchKernelGGL(k_denormalize, dim3((unsigned)((n * NT + 255) / 256)), dim3(256), 0, s, dev_y,
                     (u64)n, S.d_norm + 2 * NF, S.d_norm + 2 * NF + NT);
  hipError_t e = hipStreamSynchronize(s);
  hipFree(xn);
  if (e != hipSuccess) { ctx_error(ctx, "prediction kernels failed"); return AIWC_ERR_HIP; }
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_save(const aiwc_ctx *cctx, const char *path) {
  aiwc_ctx *ctx = (aiwc_ctx *)cctx;
  if (!ctx || !path) { ctx_error(ctx, "aiwc_sizer_save: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  sizer_download(ctx);
  FILE *f = fopen(path, "wb");
  if (!f) { ctx_error(ctx, "cannot write %s", path); return AIWC_ERR_INVALID_ARG; }
  const char magic[8] = {'A', 'I', 'W', 'C', 'M', 'L', 'P', '1'};
  const u32 np = NPARAM, nn = NNORM;
  SizerState &S = *ctx->sizer;
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 && fwrite(&nn, 4, 1, f) == 1 &&
            fwrite(S.master.data(), 4, NPARAM, f) == (size_t)NPARAM &&
            fwrite(S.norm.data(), 4, NNORM, f) == (size_t)NNORM && fwrite(&S.margin, 4, 1, f) == 1;
  fclose(f);
  if (!ok) { ctx_error(ctx, "short write to %s", path); return AIWC_ERR_INVALID_ARG; }
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_sizer_load(aiwc_ctx *ctx, const char *path) {
  if (!ctx || !path) { ctx_error(ctx, "aiwc_sizer_load: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  FILE *f = fopen(path, "rb");
  if (!f) { ctx_error(ctx, "cannot read %s", path); return AIWC_ERR_INVALID_ARG; }
  char magic[8];
  u32 np = 0, nn = 0;
  SizerState &S = *ctx->sizer;
  std::vector<float> w(NPARAM), nm(NNORM);
  float margin = 0.f;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "AIWCMLP1", 8) == 0 &&
            fread(&np, 4, 1, f) == 1 && fread(&nn, 4, 1, f) == 1 && np == NPARAM && nn == NNORM &&
            fread(w.data(), 4, NPARAM, f) == (size_t)NPARAM &&
            fread(nm.data(), 4, NNORM, f) == (size_t)NNORM && fread(&margin, 4, 1, f) == 1;
  fclose(f);
  if (!ok) { ctx_error(ctx, "%s is not a sizing network file", path); return AIWC_ERR_INVALID_ARG; }
  S.master = w;
  S.norm = nm;
  S.margin = margin;
  S.dirty = true;
  S.trained = true;
  return AIWC_OK;
}

// ------------------------------------------------------------ sizing policy
// Partitions so that one holds about 1024 pages (1 KiB address blocks).
// Partitions for an expected page count: ~1024 pages per partition (the
// bucket kernel's page table holds 1536), and on average no more than half
// the records the kernel stages on chip per round, so that most partitions
// take a single round.
static u32 pbits_for_pages(double pages, double records) {
  double want = std::ceil(std::max(1.0, pages) / 1024.0);
  want = std::max(want, std::ceil(records / (double)(AIWC_STAGE_CAP / 2)));
  u32 b = 0;
  while ((double)(1ull << b) < want) ++b;
  return std::min<u32>(15, std::max<u32>(4, b));
}

aiwc_status sizer_plan_pbits(aiwc_ctx *ctx, const aiwc_trace *const *traces, size_t n,
                             u32 mode, hipStream_t s, std::vector<u32> &pbits) {
  if (mode == AIWC_SIZING_BOUND) {
    for (size_t i = 0; i < n; ++i) pbits[i] = bound_pbits(traces[i]->d.n_mem);
    return AIWC_OK;
  }
  if (mode == AIWC_SIZING_LEARNED && !ctx->sizer->trained) {
    ctx_error(ctx, "LEARNED sizing needs a trained or loaded sizing network");
    return AIWC_ERR_INVALID_ARG;
  }
  // a trace whose record count alone asks for the most partitions gets them
  // whatever its page count: its features would not change the answer
  std::vector<const aiwc_trace *> sub;
  std::vector<size_t> idx;
  for (size_t i = 0; i < n; ++i) {
    if (pbits_for_pages(1.0, (double)traces[i]->d.n_mem) >= 15) {
      pbits[i] = 15;
    } else {
      sub.push_back(traces[i]);
      idx.push_back(i);
    }
  }
  const size_t m = sub.size();
  if (m == 0) return AIWC_OK;
  float *feat = nullptr, *pred = nullptr;
  if (hipMalloc(&feat, 4 * m * NF) != hipSuccess || hipMalloc(&pred, 4 * m * NT) != hipSuccess) {
    hipGetLastError();
    hipFree(feat);
    ctx_error(ctx, "out of device memory for sizing");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  aiwc_status st = features_impl(ctx, sub.data(), m, s, feat);
  if (st == AIWC_OK && mode == AIWC_SIZING_LEARNED) st = aiwc_sizer_predict(ctx, feat, m, s, pred);
  std::vector<float> hf(m * NF), hp(m * NT);
  if (st == AIWC_OK) {
    hipMemcpy(hf.data(), feat, 4 * m * NF, hipMemcpyDeviceToHost);
    if (mode == AIWC_SIZING_LEARNED) hipMemcpy(hp.data(), pred, 4 * m * NT, hipMemcpyDeviceToHost);
  }
  hipFree(feat);
  hipFree(pred);
  if (st != AIWC_OK) return st;
  for (size_t k = 0; k < m; ++k) {
    const size_t i = idx[k];
    const float *f = &hf[k * NF];
    const double nmem = (double)traces[i]->d.n_mem;
    const double npref = std::exp2((double)f[34]) - 1.0;
    const double scale = npref > 0 ? nmem / npref : 1.0;
    // pages (distinct at skip 10).  Local space: the prefix's local pages
    // extrapolated linearly (an upper estimate); global space: the network's
    // prediction plus the margin, or the prefix extrapolated linearly.
    const double loc = std::min(nmem, (std::exp2((double)f[29]) - 1.0) * scale);
    double glob;
    if (mode == AIWC_SIZING_LEARNED)
      glob = std::exp2((double)hp[k * NT + 10] + ctx->sizer->margin) - 1.0;
    else
      glob = (std::exp2((double)f[18]) - 1.0) * scale;
    glob = std::min(glob, nmem);
    pbits[i] = pbits_for_pages(glob + loc, nmem);
  }
  return AIWC_OK;
}
