// k_ops.hip -- the instruction stream pass (compute and parallelism metrics).
//
// One pass over the u16 opcode stream produces
//  * the per-id instruction histogram (Table I, Compute rows: opcode counts;
//    the SIMD width statistics follow from it exactly, since a width is a
//    property of the id), and
//  * the instructions-to-barrier and instructions-per-thread samples (Table I,
//    Parallelism rows; Metrics section: a per-work-item tally saved and reset
//    at each barrier, the end of the kernel being a final implicit barrier).
//
// Work decomposition: the stream is cut into tasks of ~ops_task events whose
// boundaries are snapped to work-item boundaries (binary search in
// wi_offsets), so no ITB segment crosses a task.  A wavefront owns a task and
// walks it in 512-event chunks: 8 coalesced u16 loads per lane, barrier
// positions gathered with ballots, and the (rare) barrier and work-item end
// markers walked in wave-uniform scalar code.  Histogram increments go to
// LDS copies (lane % ncopies) to spread same-id conflicts of the Zipf-like
// opcode mix.
#include "common.h"

namespace {

constexpr int OPS_BLOCK = 256;
constexpr int OPS_WAVES = OPS_BLOCK / AIWC_WAVE;
constexpr u32 LDS_VALS = 1024;   // ITB / IPT values below this counted in LDS
                                  // (13 KiB per block: two fit beside a 128 KiB
                                  // partition-histogram block)
constexpr u32 KIND_BARRIER = AIWC_KIND_BARRIER;

__device__ __forceinline__ u64 lower_bound(const u64 *a, u64 n, u64 x) {
  // first i in [0, n) with a[i] >= x (n if none)
  u64 lo = 0, hi = n;
  while (lo < hi) {
    u64 mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct WaveStats {
  u64 itb_min, itb_max, itb_cnt, itb_sum;
  u64 ipt_min, ipt_max, ipt_cnt, ipt_sum;
  u64 barriers, bad;
};

__device__ __forceinline__ void record_value(u64 v, u32 *lds_hist, u64 *g_hist,
                                             u64 *g_large, u64 *g_large_n, u64 cap,
                                             int lane) {
  if (lane == 0) {
    if (v < LDS_VALS) atomicAdd(&lds_hist[v], 1u);
    else if (v < VAL_DENSE) atomicAdd(&g_hist[v], 1ull);
    else {
      u64 i = atomicAdd(g_large_n, 1ull);
      if (i < cap) g_large[i] = v;
    }
  }
}

__host__ __device__ __forceinline__ u32 ops_copies(u32 nid) {
  u32 nc = 1;
  while (nc < 16 && (nc * 2) * nid * 4 <= 32768u) nc *= 2;
  return nc;
}

// First work-item of every ops task (the binary searches of all tasks at
// once, so that no wavefront of k_ops waits on a chain of dependent loads).
template <bool BATCH>
__global__ void k_ops_bounds(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!A.ops_wlo) return;
  const u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > A.ops_tasks) return;
  A.ops_wlo[t] = (t == A.ops_tasks) ? A.n_wi : lower_bound(A.wi_off, A.n_wi + 1, t * A.ops_task);
}

template <bool LDS_IDS, bool BATCH, bool VEC>
__global__ void __launch_bounds__(OPS_BLOCK) k_ops(TraceArgs A0, const TraceArgs *batch) {
  extern __shared__ u32 lds[];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  const u32 nid = A.n_ids;
  const u32 ncopies = LDS_IDS ? ops_copies(nid) : 1u;
  WaveStats *ws = (WaveStats *)lds;                   // [OPS_WAVES]
  u32 *itbh = lds + OPS_WAVES * sizeof(WaveStats) / 4; // [LDS_VALS]
  u32 *ipth = itbh + LDS_VALS;                        // [LDS_VALS]
  u32 *hist = ipth + LDS_VALS;                        // [ncopies][nid]
  u32 *info = hist + (LDS_IDS ? ncopies * nid : 0);   // [nid]

  // the wave index is uniform: the task walk below then keeps its state in
  // scalar registers (the barrier and work-item-end walk is wave-uniform)
  const int tid = threadIdx.x, lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(tid / AIWC_WAVE);
  if (LDS_IDS) {
    for (u32 i = tid; i < ncopies * nid; i += OPS_BLOCK) hist[i] = 0;
    for (u32 i = tid; i < nid; i += OPS_BLOCK) info[i] = A.op_info[i];
  }
  for (u32 i = tid; i < 2 * LDS_VALS; i += OPS_BLOCK) itbh[i] = 0;
  __syncthreads();

  const u32 copy = LDS_IDS ? (u32)lane & (ncopies - 1u) : 0u;
  WaveStats st;
  st.itb_min = st.ipt_min = ~0ull;
  st.itb_max = st.itb_cnt = st.itb_sum = 0;
  st.ipt_max = st.ipt_cnt = st.ipt_sum = 0;
  st.barriers = st.bad = 0;

  const u64 nwaves = (u64)gridDim.x * OPS_WAVES;
  for (u64 t = (u64)blockIdx.x * OPS_WAVES + wave; t < A.ops_tasks; t += nwaves) {
    u64 w_lo, w_hi;
    if (A.ops_wlo) {
      w_lo = A.ops_wlo[t];
      w_hi = A.ops_wlo[t + 1];
    } else {
      w_lo = lower_bound(A.wi_off, A.n_wi + 1, t * A.ops_task);
      w_hi = (t + 1 == A.ops_tasks) ? A.n_wi
                                    : lower_bound(A.wi_off, A.n_wi + 1, (t + 1) * A.ops_task);
    }
    if (w_lo > A.n_wi) w_lo = A.n_wi;
    if (w_hi > A.n_wi) w_hi = A.n_wi;
    if (w_hi <= w_lo) continue;
    // clamp to the stream so malformed offsets cannot read past it
    const u64 e1 = A.wi_off[w_hi] < A.n_events ? A.wi_off[w_hi] : A.n_events;
    const u64 e0 = A.wi_off[w_lo] < e1 ? A.wi_off[w_lo] : e1;
    u64 cur_w = w_lo, cur_begin = e0, seg_start = e0;
    u64 cur_end = A.wi_off[cur_w + 1];

    // 512-event chunks: lane l holds events [cb + 8l, cb + 8l + 8) (one
    // 16-byte load when aligned), barrier positions as per-lane bit masks.
    for (u64 cb0 = e0 & ~7ull; cb0 < e1; cb0 += 4 * 8 * AIWC_WAVE) {
      // four chunks' loads in flight before any is used
      uint4 pre[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u64 i0 = cb0 + (u64)q * 8 * AIWC_WAVE + 8ull * lane;
        pre[q] = (VEC && i0 >= e0 && i0 + 8 <= e1)
                     ? *reinterpret_cast<const uint4 *>(A.opcode + i0)
                     : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
      const u64 cb = cb0 + (u64)q * 8 * AIWC_WAVE;
      if (cb >= e1) break;
      const u64 i0 = cb + 8ull * lane;
      u32 ids[8];
      if (VEC && i0 >= e0 && i0 + 8 <= e1) {
        const uint4 v = pre[q];
        ids[0] = v.x & 0xFFFFu; ids[1] = v.x >> 16; ids[2] = v.y & 0xFFFFu; ids[3] = v.y >> 16;
        ids[4] = v.z & 0xFFFFu; ids[5] = v.z >> 16; ids[6] = v.w & 0xFFFFu; ids[7] = v.w >> 16;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const u64 i = i0 + j;
          ids[j] = (i >= e0 && i < e1) ? (u32)A.opcode[i] : 0xFFFFFFFFu;
        }
      }
      u32 bm = 0;
      // whole-wavefront fast path: every lane holds 8 valid ids, so the
      // table loads and the counting atomics are issued back to back
      bool fast = false;
      if (LDS_IDS && VEC && i0 >= e0 && i0 + 8 <= e1) {
        u32 mx = ids[0];
#pragma unroll
        for (int j = 1; j < 8; ++j) mx = ids[j] > mx ? ids[j] : mx;
        fast = mx < nid;
      }
      if (LDS_IDS && __ballot(!fast) == 0) {
        u32 in[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) in[j] = info[ids[j]];
#pragma unroll
        for (int j = 0; j < 8; ++j) atomicAdd(&hist[copy * nid + ids[j]], 1u);
#pragma unroll
        for (int j = 0; j < 8; ++j) bm |= ((in[j] & 0xFFu) == KIND_BARRIER ? 1u : 0u) << j;
      } else
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const u32 id = ids[j];
        if (id == 0xFFFFFFFFu) continue;
        if (id < nid) {
          u32 in;
          if (LDS_IDS) {
            in = info[id];
            atomicAdd(&hist[copy * nid + id], 1u);
          } else {
            in = A.op_info[id];
            atomicAdd(&A.id_hist[id], 1ull);
          }
          if ((in & 0xFFu) == KIND_BARRIER) bm |= 1u << j;
        } else {
          st.bad += 1;  // per lane; summed at the end
        }
      }
      u64 B = __ballot(bm != 0);
      const u64 lim = (cb + 8 * AIWC_WAVE < e1) ? cb + 8 * AIWC_WAVE : e1;
      // walk barrier and work-item-end markers of [cb, lim) in order
      while (true) {
        u64 nb = ~0ull;
        int bl = 0;
        u32 lm = 0;
        if (B) {
          bl = __builtin_ctzll(B);
          lm = (u32)__builtin_amdgcn_readlane((int)bm, bl);
          nb = cb + 8ull * bl + (u64)__builtin_ctz(lm);
        }
        if (cur_w < w_hi && cur_end <= lim && cur_end <= nb) {
          const u64 v = cur_end - seg_start, ipt = cur_end - cur_begin;
          record_value(v, itbh, A.itb_hist, A.itb_large, &A.acc->itb_large_n, A.large_cap, lane);
          record_value(ipt, ipth, A.ipt_hist, A.ipt_large, &A.acc->ipt_large_n, A.large_cap, lane);
          st.itb_min = v < st.itb_min ? v : st.itb_min;
          st.itb_max = v > st.itb_max ? v : st.itb_max;
          st.itb_cnt += 1; st.itb_sum += v;
          st.ipt_min = ipt < st.ipt_min ? ipt : st.ipt_min;
          st.ipt_max = ipt > st.ipt_max ? ipt : st.ipt_max;
          st.ipt_cnt += 1; st.ipt_sum += ipt;
          seg_start = cur_begin = cur_end;
          ++cur_w;
          cur_end = (cur_w < w_hi) ? A.wi_off[cur_w + 1] : ~0ull;
          continue;
        }
        if (B == 0) break;
        const u64 v = nb + 1 - seg_start;
        record_value(v, itbh, A.itb_hist, A.itb_large, &A.acc->itb_large_n, A.large_cap, lane);
        st.itb_min = v < st.itb_min ? v : st.itb_min;
        st.itb_max = v > st.itb_max ? v : st.itb_max;
        st.itb_cnt += 1; st.itb_sum += v;
        st.barriers += 1;
        seg_start = nb + 1;
        lm &= lm - 1;
        if (lane == bl) bm = lm;
        if (lm == 0) B &= B - 1;
      }
      }
    }
    // work-items left open at the end of the task (trailing empty ones)
    while (cur_w < w_hi) {
      const u64 v = cur_end - seg_start, ipt = cur_end - cur_begin;
      record_value(v, itbh, A.itb_hist, A.itb_large, &A.acc->itb_large_n, A.large_cap, lane);
      record_value(ipt, ipth, A.ipt_hist, A.ipt_large, &A.acc->ipt_large_n, A.large_cap, lane);
      st.itb_min = v < st.itb_min ? v : st.itb_min;
      st.itb_max = v > st.itb_max ? v : st.itb_max;
      st.itb_cnt += 1; st.itb_sum += v;
      st.ipt_min = ipt < st.ipt_min ? ipt : st.ipt_min;
      st.ipt_max = ipt > st.ipt_max ? ipt : st.ipt_max;
      st.ipt_cnt += 1; st.ipt_sum += ipt;
      seg_start = cur_begin = cur_end;
      ++cur_w;
      cur_end = (cur_w < w_hi) ? A.wi_off[cur_w + 1] : ~0ull;
    }
  }
  st.bad = wave_sum_u64(st.bad);
  if (lane == 0) ws[wave] = st;
  __syncthreads();

  if (LDS_IDS) {
    for (u32 id = tid; id < nid; id += OPS_BLOCK) {
      u64 s = 0;
      for (u32 c = 0; c < ncopies; ++c) s += hist[c * nid + id];
      if (s) atomicAdd(&A.id_hist[id], s);
    }
  }
  for (u32 v = tid; v < LDS_VALS; v += OPS_BLOCK) {
    if (itbh[v]) atomicAdd(&A.itb_hist[v], (u64)itbh[v]);
    if (ipth[v]) atomicAdd(&A.ipt_hist[v], (u64)ipth[v]);
  }
  if (tid == 0) {
    WaveStats r = ws[0];
    for (int w = 1; w < OPS_WAVES; ++w) {
      const WaveStats &o = ws[w];
      r.itb_min = o.itb_min < r.itb_min ? o.itb_min : r.itb_min;
      r.itb_max = o.itb_max > r.itb_max ? o.itb_max : r.itb_max;
      r.ipt_min = o.ipt_min < r.ipt_min ? o.ipt_min : r.ipt_min;
      r.ipt_max = o.ipt_max > r.ipt_max ? o.ipt_max : r.ipt_max;
      r.itb_cnt += o.itb_cnt; r.itb_sum += o.itb_sum;
      r.ipt_cnt += o.ipt_cnt; r.ipt_sum += o.ipt_sum;
      r.barriers += o.barriers; r.bad += o.bad;
    }
    DevAccum *acc = A.acc;
    if (r.itb_cnt) {
      atomicMax(&acc->itb_min_inv, ~r.itb_min);
      atomicMax(&acc->itb_max, r.itb_max);
      atomicAdd(&acc->itb_cnt, r.itb_cnt);
      atomicAdd(&acc->itb_sum, r.itb_sum);
    }
    if (r.ipt_cnt) {
      atomicMax(&acc->ipt_min_inv, ~r.ipt_min);
      atomicMax(&acc->ipt_max, r.ipt_max);
      atomicAdd(&acc->ipt_cnt, r.ipt_cnt);
      atomicAdd(&acc->ipt_sum, r.ipt_sum);
    }
    if (r.barriers) atomicAdd(&acc->barriers, r.barriers);
    if (r.bad) atomicAdd(&acc->bad_ids, r.bad);
  }
}

template <bool BATCH>
__global__ void k_zero(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  uint4 *p = (uint4 *)A.zero_base;
  const size_t n16 = A.zero_bytes / 16;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

}  // namespace

namespace aiwc_kernels {

hipError_t launch_zero(const TraceArgs &a, const BatchDims &d, hipStream_t s) {
  u64 n16 = d.max_zero16;
  if (n16 == 0) return hipSuccess;
  unsigned gx = (unsigned)((n16 + 255) / 256);
  if (gx > 2048) gx = 2048;
  if (d.batch) hipLaunchKernelGGL(k_zero<true>, dim3(gx, d.n), dim3(256), 0, s, a, d.batch);
  else hipLaunchKernelGGL(k_zero<false>, dim3(gx), dim3(256), 0, s, a, nullptr);
  return hipGetLastError();
}

size_t ops_lds_bytes(u32 n_ids) {
  const size_t tail = OPS_WAVES * sizeof(WaveStats) + 2 * LDS_VALS * 4;
  if (n_ids > 8192) return tail;
  return tail + 4 * ((size_t)ops_copies(n_ids) * n_ids + n_ids);
}

hipError_t launch_ops(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm) {
  if (d.max_ops_tasks == 0) return hipSuccess;
  if (d.batch || a.ops_wlo) {
    const dim3 gt((unsigned)((d.max_ops_tasks + 1 + 255) / 256), d.n);
    if (d.batch) hipLaunchKernelGGL(k_ops_bounds<true>, gt, dim3(256), 0, s, a, d.batch);
    else hipLaunchKernelGGL(k_ops_bounds<false>, gt, dim3(256), 0, s, a, nullptr);
  }
  u64 waves = d.max_ops_tasks < 4096 ? d.max_ops_tasks : 4096;
  unsigned gx = (unsigned)((waves + OPS_WAVES - 1) / OPS_WAVES);
  if (d.ops_max_blocks && gx > d.ops_max_blocks) gx = d.ops_max_blocks;
  size_t tail = OPS_WAVES * sizeof(WaveStats) + 2 * LDS_VALS * 4;
  const dim3 g(gx, d.n), blk(OPS_BLOCK);
  const TraceArgs *b = d.batch;
  const size_t lds = d.max_ids <= 8192 ? (d.ops_lds ? d.ops_lds : ops_lds_bytes(d.max_ids)) : tail;
#define OPS_LAUNCH(L, B, V) hipLaunchKernelGGL((k_ops<L, B, V>), g, blk, lds, s, a, b)
  if (d.max_ids <= 8192) {
    if (b) { if (d.ops_vec) OPS_LAUNCH(true, true, true); else OPS_LAUNCH(true, true, false); }
    else { if (d.ops_vec) OPS_LAUNCH(true, false, true); else OPS_LAUNCH(true, false, false); }
  } else {
    if (b) { if (d.ops_vec) OPS_LAUNCH(false, true, true); else OPS_LAUNCH(false, true, false); }
    else { if (d.ops_vec) OPS_LAUNCH(false, false, true); else OPS_LAUNCH(false, false, false); }
  }
#undef OPS_LAUNCH
  AIWC_MARK(pm, "k_ops", s);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
