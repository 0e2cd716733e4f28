// k_final.hip -- the kernelEnd statistics (Implementation section): turns
// the stage accumulators into the Table I metrics, on the device, in one
// block.  Exact integer work: class histogram, SIMD sums (128-bit), the
// coverage counts (90% rows of Table I), and the ITB / IPT medians (order
// statistics selected from the value histograms).  Floating point: one IEEE
// division per ratio, the square root of the exact SIMD variance numerator,
// and the conversion of the fixed-point entropy sums.
#include "common.h"

namespace {

constexpr int FB = 512;

constexpr u32 SPEC_LDS = 4096;   // spectrum pairs compacted into LDS

struct FinShared {
  u64 red[FB / AIWC_WAVE];
  u64 red2[FB / AIWC_WAVE];
  u64 bcast[4];
  u64 cf[SPEC_LDS], cm[SPEC_LDS];  // compacted (f, m_f) pairs of one space
  u32 nc;
};

__device__ u64 block_sum(u64 v, FinShared &S) {
  v = wave_sum_u64(v);
  __syncthreads();
  if (lane_id() == 0) S.red[threadIdx.x / AIWC_WAVE] = v;
  __syncthreads();
  u64 t = 0;
#pragma unroll
  for (int w = 0; w < FB / AIWC_WAVE; ++w) t += S.red[w];
  return t;
}

__device__ u64 block_max(u64 v, FinShared &S) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    u64 x = __shfl_xor(v, o, 64);
    v = x > v ? x : v;
  }
  __syncthreads();
  if (lane_id() == 0) S.red[threadIdx.x / AIWC_WAVE] = v;
  __syncthreads();
  u64 t = 0;
#pragma unroll
  for (int w = 0; w < FB / AIWC_WAVE; ++w) t = S.red[w] > t ? S.red[w] : t;
  return t;
}

// Items are (value f_i, multiplicity m_i).  Returns the fewest items that,
// taken largest value first, sum to at least 90% of total (10 cum >= 9 total):
// all items above the threshold value t*, plus the needed share of those at
// t*, where t* is the largest t with 10 * sum_{f >= t} m f >= 9 total.
template <typename Get>
__device__ u64 coverage90(u64 n_items, u64 total, Get get, FinShared &S) {
  if (total == 0) return 0;
  constexpr int R = 8;
  if (n_items <= (u64)R * FB) {
    // at most R items per thread: read once into registers, then the same
    // search over them
    u64 f[R], m[R], fmax = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const u64 i = threadIdx.x + (u64)r * FB;
      f[r] = 0;
      m[r] = 0;
      if (i < n_items) get(i, f[r], m[r]);
      if (!m[r]) f[r] = 0;
      fmax = f[r] > fmax ? f[r] : fmax;
    }
    fmax = block_max(fmax, S);
    u64 lo = 1, hi = fmax;
    while (lo < hi) {
      const u64 mid = lo + (hi - lo + 1) / 2;
      u64 mass = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) mass += f[r] >= mid ? m[r] * f[r] : 0ull;
      mass = block_sum(mass, S);
      if ((unsigned __int128)mass * 10 >= (unsigned __int128)total * 9) lo = mid; else hi = mid - 1;
    }
    const u64 t = lo;
    u64 above = 0, above_n = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (f[r] > t) { above += m[r] * f[r]; above_n += m[r]; }
    above = block_sum(above, S);
    above_n = block_sum(above_n, S);
    const unsigned __int128 need = (unsigned __int128)total * 9 - (unsigned __int128)above * 10;
    const unsigned __int128 per = (unsigned __int128)t * 10;
    return above_n + (u64)((need + per - 1) / per);
  }
  u64 fmax = 0;
  for (u64 i = threadIdx.x; i < n_items; i += FB) {
    u64 f, m;
    get(i, f, m);
    if (m && f > fmax) fmax = f;
  }
  fmax = block_max(fmax, S);
  u64 lo = 1, hi = fmax;
  while (lo < hi) {
    const u64 mid = lo + (hi - lo + 1) / 2;
    u64 mass = 0;
    for (u64 i = threadIdx.x; i < n_items; i += FB) {
      u64 f, m;
      get(i, f, m);
      if (f >= mid) mass += m * f;
    }
    mass = block_sum(mass, S);
    if ((unsigned __int128)mass * 10 >= (unsigned __int128)total * 9) lo = mid; else hi = mid - 1;
  }
  const u64 t = lo;
  u64 above = 0, above_n = 0;
  for (u64 i = threadIdx.x; i < n_items; i += FB) {
    u64 f, m;
    get(i, f, m);
    if (f > t) { above += m * f; above_n += m; }
  }
  above = block_sum(above, S);
  above_n = block_sum(above_n, S);
  const unsigned __int128 need = (unsigned __int128)total * 9 - (unsigned __int128)above * 10;
  const unsigned __int128 per = (unsigned __int128)t * 10;
  return above_n + (u64)((need + per - 1) / per);
}

// k-th smallest (0-based) value of the sample held as a dense histogram of
// values < VAL_DENSE plus a list of the larger values.
__device__ u64 select_kth(const u64 *hist, const u64 *large, u64 n_large, u64 k, FinShared &S) {
  constexpr int PER = VAL_DENSE / FB;  // 64 bins per thread
  u64 mine = 0;
  const u64 b0 = (u64)threadIdx.x * PER;
  for (int j = 0; j < PER; ++j) mine += hist[b0 + j];
  // exclusive prefix of 'mine' over threads
  u64 x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u64 y = __shfl_up(x, o, 64);
    if (lane_id() >= o) x += y;
  }
  __syncthreads();
  if (lane_id() == 63) S.red2[threadIdx.x / AIWC_WAVE] = x;
  if (threadIdx.x == 0) S.bcast[0] = ~0ull;
  __syncthreads();
  u64 before = 0, dense_total = 0;
  for (int w = 0; w < FB / AIWC_WAVE; ++w) {
    if (w < (int)(threadIdx.x / AIWC_WAVE)) before += S.red2[w];
    dense_total += S.red2[w];
  }
  before += x - mine;
  if (k < dense_total) {
    if (k >= before && k < before + mine) {
      u64 c = before;
      for (int j = 0; j < PER; ++j) {
        c += hist[b0 + j];
        if (k < c) { S.bcast[0] = b0 + j; break; }
      }
    }
    __syncthreads();
    return S.bcast[0];
  }
  __syncthreads();
  // among the large values: smallest v with #{x <= v} > k'
  const u64 kk = k - dense_total;
  u64 lo = VAL_DENSE, hi = 0;
  for (u64 i = threadIdx.x; i < n_large; i += FB) hi = large[i] > hi ? large[i] : hi;
  hi = block_max(hi, S);
  while (lo < hi) {
    const u64 mid = lo + (hi - lo) / 2;
    u64 c = 0;
    for (u64 i = threadIdx.x; i < n_large; i += FB) c += large[i] <= mid;
    c = block_sum(c, S);
    if (c > kk) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ double median_of(const u64 *hist, const u64 *large, u64 n_large, u64 count,
                            FinShared &S) {
  if (count == 0) return 0.0;
  if (count & 1) return (double)select_kth(hist, large, n_large, count / 2, S);
  const u64 a = select_kth(hist, large, n_large, count / 2 - 1, S);
  const u64 b = select_kth(hist, large, n_large, count / 2, S);
  return ((double)a + (double)b) * 0.5;
}

// The memory spaces' 90% footprints from their level-0 spectra (each
// compacted into LDS when it fits) and the spectra's export (block 2 of
// k_finalize).
__device__ void spectrum_part(const TraceArgs &A, FinShared &S, aiwc_metrics_host *o,
                              u64 *status) {
  const int tid = threadIdx.x;
  DevAccum *acc = A.acc;
  u64 fp90[2];
  for (int s = 0; s < 2; ++s) {
    const u64 *F = A.sp_f + (u64)s * A.sp_cap, *M = A.sp_m + (u64)s * A.sp_cap;
    const u64 N = acc->sp_reads[s] + acc->sp_writes[s];
    __syncthreads();
    if (tid == 0) S.nc = 0;
    __syncthreads();
    for (u64 i0 = tid; i0 < A.sp_cap; i0 += 8 * FB) {
      u64 f[8];   // eight loads in flight before any is tested
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = i0 + (u64)q * FB < A.sp_cap ? F[i0 + (u64)q * FB] : 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (!f[q]) continue;
        const u32 j = atomicAdd(&S.nc, 1u);
        if (j < SPEC_LDS) { S.cf[j] = f[q]; S.cm[j] = M[i0 + (u64)q * FB]; }
      }
    }
    __syncthreads();
    const u32 nc = S.nc;
    if (nc <= SPEC_LDS) {
      const u64 *cf = S.cf, *cm = S.cm;
      fp90[s] = coverage90((u64)nc, N, [cf, cm](u64 i, u64 &f, u64 &m) { f = cf[i]; m = cm[i]; }, S);
    } else {
      fp90[s] = coverage90((u64)A.sp_cap, N,
                           [F, M](u64 i, u64 &f, u64 &m) { f = F[i]; m = f ? M[i] : 0; }, S);
    }
  }

  if (tid == 0) { S.bcast[1] = 0; S.bcast[2] = 0; }
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    const u64 *F = A.sp_f + (u64)s * A.sp_cap, *M = A.sp_m + (u64)s * A.sp_cap;
    u64 *dst = A.out_spec + (u64)s * 2 * A.spec_export_cap;
    for (u64 i0 = tid; i0 < A.sp_cap; i0 += 8 * FB) {
      u64 f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = i0 + (u64)q * FB < A.sp_cap ? F[i0 + (u64)q * FB] : 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (!f[q]) continue;
        const u64 j = atomicAdd((u64 *)&S.bcast[1 + s], 1ull);
        if (j < A.spec_export_cap) { dst[2 * j] = f[q]; dst[2 * j + 1] = M[i0 + (u64)q * FB]; }
      }
    }
  }
  __syncthreads();

  if (tid == 0) {
    o->space[0].footprint_90 = fp90[0];
    o->space[1].footprint_90 = fp90[1];
    status[2] = S.bcast[1] | (S.bcast[2] << 32);
  }
}

template <bool BATCH>
__global__ void __launch_bounds__(FB) k_finalize(TraceArgs A0, const TraceArgs *batch) {
  __shared__ FinShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  const int tid = threadIdx.x;
  DevAccum *acc = A.acc;
  aiwc_metrics_host *o = A.out;
  u64 *status = reinterpret_cast<u64 *>(o + 1);
  // Three blocks per trace, each writing fields of its own: block 1 the IPT
  // median, block 2 the 90% footprints and the spectrum exports, block 0
  // everything else.
  const int part = blockIdx.x;
  if (part == 1) {
    const u64 nl_ipt = acc->ipt_large_n < A.large_cap ? acc->ipt_large_n : A.large_cap;
    const double ipt_med = median_of(A.ipt_hist, A.ipt_large, nl_ipt, acc->ipt_cnt, S);
    if (tid == 0) o->ipt_median = ipt_med;
    return;
  }
  if (part == 2) {
    spectrum_part(A, S, o, status);
    return;
  }

  // ---- compute: class histogram, SIMD sums, kind counts
  u64 s1 = 0, s2lo = 0, s2hi = 0, wmax = 0, nload = 0, nstore = 0, natom = 0, nbr = 0;
  for (u32 id = tid; id < A.n_ids; id += FB) {
    const u64 c = A.id_hist[id];
    if (!c) continue;
    const u32 in = A.op_info[id];
    const u64 w = (in >> 8) & 0xFFu;
    atomicAdd(&A.class_hist[in >> 16], c);
    s1 += c * w;
    const unsigned __int128 q = (unsigned __int128)c * (w * w);
    u64 nl = s2lo + (u64)q;
    s2hi += (u64)(q >> 64) + (nl < s2lo);
    s2lo = nl;
    wmax = w > wmax ? w : wmax;
    switch (in & 0xFFu) {
      case AIWC_KIND_LOAD: nload += c; break;
      case AIWC_KIND_STORE: nstore += c; break;
      case AIWC_KIND_ATOMIC_RMW: natom += c; break;
      case AIWC_KIND_BRANCH_COND: nbr += c; break;
      default: break;
    }
  }
  s1 = block_sum(s1, S);
  wmax = block_max(wmax, S);
  nload = block_sum(nload, S);
  nstore = block_sum(nstore, S);
  natom = block_sum(natom, S);
  nbr = block_sum(nbr, S);
  // 128-bit sum of S2: reduce lo with carries counted separately
  {
    u64 lo = s2lo, hi = s2hi;
    wave_sum_u128(lo, hi);
    __syncthreads();
    if (lane_id() == 0) { S.red[tid / AIWC_WAVE] = lo; S.red2[tid / AIWC_WAVE] = hi; }
    __syncthreads();
    lo = 0; hi = 0;
    for (int w = 0; w < FB / AIWC_WAVE; ++w) {
      u64 nl = lo + S.red[w];
      hi += S.red2[w] + (nl < lo);
      lo = nl;
    }
    s2lo = lo; s2hi = hi;
  }
  __threadfence();
  __syncthreads();
  u64 uniq = 0;
  for (u32 c = tid; c < A.n_classes; c += FB) uniq += A.class_hist[c] != 0;
  uniq = block_sum(uniq, S);
  const u64 *ch = A.class_hist;
  const u64 op90 = coverage90((u64)A.n_classes, A.n_events,
                              [ch](u64 i, u64 &f, u64 &m) { f = ch[i]; m = f ? 1 : 0; }, S);

  // ---- parallelism
  const u64 nl_itb = acc->itb_large_n < A.large_cap ? acc->itb_large_n : A.large_cap;
  const double itb_med = median_of(A.itb_hist, A.itb_large, nl_itb, acc->itb_cnt, S);

  // ---- branches
  const u32 *ss = A.seg_start, *se = A.seg_end;
  u64 usites = 0;
  for (u32 s = tid; s < A.n_sites; s += FB) usites += se[s] > ss[s];
  usites = block_sum(usites, S);
  const u64 br90 = (A.n_branch == 0) ? 0
      : coverage90((u64)A.n_sites, A.n_branch,
                   [ss, se](u64 i, u64 &f, u64 &m) { f = se[i] - ss[i]; m = f ? 1 : 0; }, S);

  // ---- export: class histogram
  for (u32 c = tid; c < A.n_classes; c += FB) A.out_class_hist[c] = A.class_hist[c];
  __syncthreads();

  if (tid != 0) return;
  o->struct_size = sizeof(aiwc_metrics_host);
  o->history_len = A.m;
  o->total_instructions = A.n_events;
  o->unique_opcodes = (uint32_t)uniq;
  o->opcodes_90 = (uint32_t)op90;
  o->simd_max = wmax;
  o->simd_sum = s1;
  o->simd_sumsq_lo = s2lo;
  o->simd_sumsq_hi = s2hi;
  if (A.n_events) {
    const double n = (double)A.n_events;
    o->simd_mean = (double)s1 / n;
    // U = N * S2 - S1^2, exact in 128 bits
    const unsigned __int128 S2 = ((unsigned __int128)s2hi << 64) | s2lo;
    const unsigned __int128 U = (unsigned __int128)A.n_events * S2 -
                                (unsigned __int128)s1 * (unsigned __int128)s1;
    const double ud = (double)(u64)(U >> 64) * 18446744073709551616.0 + (double)(u64)U;
    o->simd_sd = sqrt(ud) / n;
  } else {
    o->simd_mean = 0.0;
    o->simd_sd = 0.0;
  }
  o->work_items = A.n_wi;
  o->barriers_hit = acc->barriers;
  o->itb_count = acc->itb_cnt;
  o->itb_sum = acc->itb_sum;
  o->itb_min = acc->itb_cnt ? ~acc->itb_min_inv : 0;
  o->itb_max = acc->itb_max;
  o->itb_median = itb_med;
  o->ipt_min = acc->ipt_cnt ? ~acc->ipt_min_inv : 0;
  o->ipt_max = acc->ipt_max;
  for (int s = 0; s < 2; ++s) {
    aiwc_space_metrics &m = o->space[s];
    const u64 N = acc->sp_reads[s] + acc->sp_writes[s];
    m.total_accesses = N;
    m.total_reads = acc->sp_reads[s];
    m.total_writes = acc->sp_writes[s];
    m.unique_reads = acc->uniq_r[s];
    m.unique_writes = acc->uniq_w[s];
    m.footprint = acc->distinct[s][0];
    for (int k = 0; k < AIWC_NSKIP; ++k) {
      m.distinct[k] = acc->distinct[s][k];
      m.entropy[k] = N ? fx64_to_double(acc->ent_lo[s][k], acc->ent_hi[s][k]) / (double)N : 0.0;
    }
    m.unique_rw_ratio = (double)m.unique_reads / (double)m.unique_writes;
    m.reread_ratio = (double)m.unique_reads / (double)m.total_reads;
    m.rewrite_ratio = (double)m.unique_writes / (double)m.total_writes;
  }
  o->total_branches = A.n_branch;
  o->unique_branches = usites;
  o->branches_90 = br90;
  o->n_windows = acc->br_windows;
  o->albe_min_sum = acc->br_minsum;
  const double nw = (double)acc->br_windows;
  o->yokota_entropy = acc->br_windows ? fx64_to_double(acc->yok_lo, acc->yok_hi) / nw : 0.0;
  o->linear_branch_entropy = acc->br_windows ? (double)(2 * acc->br_minsum) / nw : 0.0;
  // pattern form of the branch history entropy, normalised by m; NaN when
  // the trace did not ask for it
  o->pattern_entropy = (A.br_flags & AIWC_BRANCH_PATTERN_ENTROPY)
                           ? (acc->br_windows
                                  ? fx64_to_double(acc->pat_lo, acc->pat_hi) / nw / (double)A.m
                                  : 0.0)
                           : __builtin_nan("");
  // derived parallelism metrics of the LU analysis: inverses of work-items,
  // mean ITB and mean SIMD width as single divisions of the exact integers
  // (x/0 = inf, 0/0 = NaN), and the spread of instructions per work-item
  o->granularity = 1.0 / (double)A.n_wi;
  o->barriers_per_instruction = (double)acc->itb_cnt / (double)acc->itb_sum;
  o->instructions_per_operand = (double)A.n_events / (double)s1;
  o->load_imbalance = o->ipt_max - o->ipt_min;
  o->overflow_redos = (uint32_t)acc->redos;
  o->partitions = A.n_mem ? (1u << A.pbits) : 0u;
  // status words: [0] invalid content, [1] inconsistent kinds, [2] spectrum
  // pairs, [3] on-chip tables whose split limit was reached
  status[0] = acc->bad_ids + acc->bad_mem;
  status[3] = acc->split_fail;
  status[1] = (nload + nstore + 2 * natom != A.n_mem || nbr != A.n_branch) ? 1ull : 0ull;
}

}  // namespace

namespace aiwc_kernels {

hipError_t launch_finalize(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm) {
  if (d.batch) hipLaunchKernelGGL(k_finalize<true>, dim3(3, d.n), dim3(FB), 0, s, a, d.batch);
  else hipLaunchKernelGGL(k_finalize<false>, dim3(3), dim3(FB), 0, s, a, nullptr);
  AIWC_MARK(pm, "k_finalize", s);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
