// k_mem.hip -- memory metrics (Table I, Memory rows; Metrics section).
//
// For each address space s and LSB skip k = 0..10 we need the exact
// multiset of bucket counts of (a >> k): the number of buckets (distinct_k),
// the plug-in Shannon entropy of their frequencies, and at k = 0 the count
// spectrum (90% footprint) and the distinct read / write addresses.
//
// The distinct sets of a full trace are far larger than on-chip memory, so
// the addresses are radix-partitioned once by a bijective hash of their
// 1 KiB page (a >> 10).  Every bucket a >> k with k <= 10 lies inside one
// page, hence inside one partition, and partitions are independent.
//   k_mem_hist    : per-block partition histogram of the address stream
//   k_mem_colscan : exclusive scan over blocks, per partition
//   k_mem_binscan : exclusive scan over partitions
//   k_mem_scatter : write one 64-bit record per access into its partition
//   k_mem_bucket  : per partition, an LDS open-addressing table of the
//                   distinct addresses (count + read/write flags), coarsened
//                   level by level (key >> 1) up to k = 10; each level adds
//                   its distinct count and its entropy terms
//                   c * log2(N / c) (exact 128-bit fixed point, so the sum is
//                   order independent), level 0 also its count spectrum.
//                   A partition whose distinct set overflows the table is
//                   split by further hash bits and redone (exact).
//
// Record layout (64 bits; P = 2^pbits partitions, h = mix54(a >> 10)):
//   [0]                  write flag
//   [1, 11)              a & 1023 (byte offset in the page)
//   [11, 65 - pbits)     h & (2^(54 - pbits) - 1)   (page id inside the partition)
//   [65 - pbits]         address space (1 = local)
// The partition index is h >> (54 - pbits); it is implied by the position.
#include "common.h"

namespace {

constexpr int MEM_BLOCK = 1024;
constexpr u32 TBL_C = 9216;       // LDS table slots
constexpr u32 TBL_CAP = 7680;     // live entries before a partition is split
constexpr u32 SPEC_SLOTS = 256;   // per-space LDS cache of the level-0 spectrum
constexpr u64 EMPTY = ~0ull;
constexpr int MAX_PER_THREAD = (TBL_CAP + MEM_BLOCK + MEM_BLOCK - 1) / MEM_BLOCK;  // 9

__device__ __forceinline__ u64 make_record(u64 a, uint8_t kind, u32 pbits, u32 &bin) {
  const u64 h = mix54(a >> 10);
  const u32 low_bits = PAGE_BITS - pbits;
  bin = (u32)(h >> low_bits);
  const u64 hl = h & ((1ull << low_bits) - 1ull);
  return ((u64)((kind >> 1) & 1u) << (65 - pbits)) | (hl << 11) | ((a & 1023ull) << 1) |
         (u64)(kind & 1u);
}

// -------------------------------------------------------------- histogram
constexpr u32 MAX_PARTS = 32768;

template <bool VEC, bool BATCH>
__global__ void __launch_bounds__(MEM_BLOCK) k_mem_hist(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u32 h[MAX_PARTS];
  __shared__ u64 sp_cnt[4];  // reads g, writes g, reads l, writes l
  const TraceArgs &A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || blockIdx.x >= A.n_hist_blocks) return;
  const u32 P = 1u << A.pbits;
  for (u32 i = threadIdx.x; i < P; i += MEM_BLOCK) h[i] = 0;
  if (threadIdx.x < 4) sp_cnt[threadIdx.x] = 0;
  __syncthreads();
  const u64 c0 = (u64)blockIdx.x * A.hist_chunk;
  const u64 c1 = (c0 + A.hist_chunk < A.n_mem) ? c0 + A.hist_chunk : A.n_mem;
  u32 cnt[4] = {0, 0, 0, 0};
  for (u64 i = c0 + 4ull * threadIdx.x; i < c1; i += 4ull * MEM_BLOCK) {
    u64 a[4];
    u32 kk;
    int n = 4;
    if (VEC && i + 4 <= c1) {
      const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(A.addr + i);
      ulonglong2 x = pa[0], y = pa[1];
      a[0] = x.x; a[1] = x.y; a[2] = y.x; a[3] = y.y;
      kk = *reinterpret_cast<const u32 *>(A.mem_kind + i);
    } else {
      n = (int)((c1 - i) < 4 ? (c1 - i) : 4);
      kk = 0;
      for (int j = 0; j < 4; ++j) {
        a[j] = j < n ? A.addr[i + j] : 0;
        kk |= (u32)(j < n ? A.mem_kind[i + j] : 0) << (8 * j);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < n) {
        const uint8_t k = (uint8_t)(kk >> (8 * j));
        u32 bin;
        make_record(a[j], k, A.pbits, bin);
        atomicAdd(&h[bin], 1u);
        cnt[((k >> 1) & 1u) * 2 + (k & 1u)] += 1;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    u64 v = wave_sum_u64(cnt[j]);
    if (lane_id() == 0 && v) atomicAdd(&sp_cnt[j], v);
  }
  __syncthreads();
  u32 *row = A.part_hist + (u64)blockIdx.x * P;
  for (u32 i = threadIdx.x; i < P; i += MEM_BLOCK) row[i] = h[i];
  if (threadIdx.x < 4 && sp_cnt[threadIdx.x]) {
    u64 *dst = (threadIdx.x & 1) ? &A.acc->sp_writes[threadIdx.x >> 1]
                                 : &A.acc->sp_reads[threadIdx.x >> 1];
    atomicAdd(dst, sp_cnt[threadIdx.x]);
  }
}

// Per partition: exclusive prefix over the histogram blocks (in place);
// the partition total goes to part_off[b].
template <bool BATCH>
__global__ void k_mem_colscan(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs &A = trace_args<BATCH>(A0, batch);
  const u32 P = 1u << A.pbits;
  const u32 b = blockIdx.x * blockDim.x + threadIdx.x;
  if (A.n_mem == 0 || b >= P) return;
  u32 s = 0;
  for (u32 w = 0; w < A.n_hist_blocks; ++w) {
    u32 *p = A.part_hist + (u64)w * P + b;
    u32 v = *p;
    *p = s;
    s += v;
  }
  A.part_off[b] = s;
}

// Exclusive scan of the partition totals (one block); part_off[P] = n_mem.
template <bool BATCH>
__global__ void __launch_bounds__(1024) k_mem_binscan(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u32 wsum[16];
  __shared__ u32 carry;
  const TraceArgs &A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0) return;
  const u32 P = 1u << A.pbits;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (u32 base = 0; base < P; base += 1024) {
    const u32 i = base + threadIdx.x;
    const u32 v = i < P ? A.part_off[i] : 0;
    // inclusive wave scan
    u32 x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      u32 y = __shfl_up(x, o, 64);
      if (lane_id() >= o) x += y;
    }
    if (lane_id() == 63) wsum[threadIdx.x / 64] = x;
    __syncthreads();
    u32 before = carry;
    for (u32 w = 0; w < threadIdx.x / 64; ++w) before += wsum[w];
    if (i < P) A.part_off[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) A.part_off[P] = carry;
}

// -------------------------------------------------------------- scatter
template <bool VEC, bool BATCH>
__global__ void __launch_bounds__(MEM_BLOCK) k_mem_scatter(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u32 cur[MAX_PARTS];
  const TraceArgs &A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || blockIdx.x >= A.n_hist_blocks) return;
  const u32 P = 1u << A.pbits;
  const u32 *row = A.part_hist + (u64)blockIdx.x * P;
  for (u32 i = threadIdx.x; i < P; i += MEM_BLOCK) cur[i] = A.part_off[i] + row[i];
  __syncthreads();
  const u64 c0 = (u64)blockIdx.x * A.hist_chunk;
  const u64 c1 = (c0 + A.hist_chunk < A.n_mem) ? c0 + A.hist_chunk : A.n_mem;
  for (u64 i = c0 + 4ull * threadIdx.x; i < c1; i += 4ull * MEM_BLOCK) {
    u64 a[4];
    u32 kk;
    int n = 4;
    if (VEC && i + 4 <= c1) {
      const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(A.addr + i);
      ulonglong2 x = pa[0], y = pa[1];
      a[0] = x.x; a[1] = x.y; a[2] = y.x; a[3] = y.y;
      kk = *reinterpret_cast<const u32 *>(A.mem_kind + i);
    } else {
      n = (int)((c1 - i) < 4 ? (c1 - i) : 4);
      kk = 0;
      for (int j = 0; j < 4; ++j) {
        a[j] = j < n ? A.addr[i + j] : 0;
        kk |= (u32)(j < n ? A.mem_kind[i + j] : 0) << (8 * j);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < n) {
        u32 bin;
        const u64 rec = make_record(a[j], (uint8_t)(kk >> (8 * j)), A.pbits, bin);
        const u32 pos = atomicAdd(&cur[bin], 1u);
        A.part_rec[pos] = rec;
      }
    }
  }
}

// ---------------------------------------------------------------- bucket
struct BucketShared {
  u64 key[TBL_C];            // (key << 2) | read/write flags, EMPTY if free
  u32 cnt[TBL_C];
  uint16_t live[TBL_C];
  u64 tlo[2][256], thi[2][256];   // entropy term table for c < 256, per space
  u64 spf[2][SPEC_SLOTS], spm[2][SPEC_SLOTS];  // level-0 spectrum cache
  u64 dist[2][AIWC_NSKIP], elo[2][AIWC_NSKIP], ehi[2][AIWC_NSKIP];
  u64 ur[2], uw[2];
  u64 redos;
  u32 live_n, overflow, work;
  u32 stack_m[64], stack_c[64];
  u32 sp_top;
};

// c * log2(N / c) as 2^-64 fixed point.
__device__ __forceinline__ void term_fx(u64 c, u64 N, u64 &lo, u64 &hi) {
  if (c == 0 || c >= N) { lo = hi = 0; return; }
  const double d = (double)c * (log1p((double)(N - c) / (double)c) * 1.4426950408889634074);
  to_fx64(d, lo, hi);
}

__device__ void global_spec_add(const TraceArgs &A, u32 s, u64 f, u64 m) {
  u64 *F = A.sp_f + (u64)s * A.sp_cap;
  u64 *M = A.sp_m + (u64)s * A.sp_cap;
  u32 slot = hash_slot(f, A.sp_cap);
  for (u32 probe = 0; probe < A.sp_cap; ++probe) {
    u64 old = atomicCAS(&F[slot], 0ull, f);
    if (old == 0ull || old == f) { atomicAdd(&M[slot], m); return; }
    slot = (slot + 1 == A.sp_cap) ? 0 : slot + 1;
  }
}

__device__ __forceinline__ void spec_cache_add(BucketShared &S, const TraceArgs &A, u32 s, u64 f,
                                               u64 m) {
  u32 slot = (u32)((f * 0x9E3779B97F4A7C15ull) >> 56);  // 0..255
  for (u32 probe = 0; probe < 16; ++probe) {
    u64 old = atomicCAS(&S.spf[s][slot], 0ull, f);
    if (old == 0ull || old == f) { atomicAdd(&S.spm[s][slot], m); return; }
    slot = (slot + 1) & (SPEC_SLOTS - 1);
  }
  global_spec_add(A, s, f, m);
}

// Level-0 inserts stop at TBL_CAP live entries (the partition is then split);
// coarser levels never hold more entries than level 0, so they skip the check
// and use the TBL_C - TBL_CAP spare slots only as probing slack.
__device__ __forceinline__ bool tbl_insert(BucketShared &S, u64 key, u64 flag, u32 c,
                                           bool capped) {
  u32 slot = hash_slot(key, TBL_C);
  const u64 word = (key << 2) | flag;
  while (true) {
    u64 w = S.key[slot];
    if (w == EMPTY) {
      if (capped && S.live_n >= TBL_CAP) { S.overflow = 1; return false; }
      u64 old = atomicCAS(&S.key[slot], EMPTY, word);
      if (old == EMPTY) {
        atomicAdd(&S.cnt[slot], c);
        u32 idx = atomicAdd(&S.live_n, 1u);
        if (idx < TBL_C) S.live[idx] = (uint16_t)slot;
        return true;
      }
      w = old;
    }
    if ((w >> 2) == key) {
      if (flag & ~w) atomicOr(&S.key[slot], flag);
      atomicAdd(&S.cnt[slot], c);
      return true;
    }
    slot = (slot + 1 == TBL_C) ? 0 : slot + 1;
  }
}

template <bool BATCH>
__global__ void __launch_bounds__(MEM_BLOCK) k_mem_bucket(TraceArgs A0, const TraceArgs *batch) {
  __shared__ BucketShared S;
  const TraceArgs &A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0) return;
  const int tid = threadIdx.x, lane = lane_id();
  const u32 P = 1u << A.pbits;
  const u64 N[2] = {A.acc->sp_reads[0] + A.acc->sp_writes[0],
                    A.acc->sp_reads[1] + A.acc->sp_writes[1]};
  for (u32 i = tid; i < TBL_C; i += MEM_BLOCK) { S.key[i] = EMPTY; S.cnt[i] = 0; }
  for (u32 i = tid; i < 2 * 256; i += MEM_BLOCK) {
    u64 lo, hi;
    term_fx(i & 255u, N[i >> 8], lo, hi);
    S.tlo[i >> 8][i & 255u] = lo;
    S.thi[i >> 8][i & 255u] = hi;
    S.spf[i >> 8][i & 255u] = 0;
    S.spm[i >> 8][i & 255u] = 0;
  }
  if (tid < 2 * AIWC_NSKIP) {
    (&S.dist[0][0])[tid] = 0; (&S.elo[0][0])[tid] = 0; (&S.ehi[0][0])[tid] = 0;
  }
  if (tid < 2) { S.ur[tid] = 0; S.uw[tid] = 0; }
  if (tid == 0) { S.redos = 0; S.live_n = 0; S.overflow = 0; }
  __syncthreads();

  while (true) {
    if (tid == 0) S.work = (u32)atomicAdd(&A.acc->mem_queue, 1ull);
    __syncthreads();
    const u32 p = S.work;
    if (p >= P) break;
    const u64 base = A.part_off[p];
    const u64 n = (u64)A.part_off[p + 1] - base;
    if (tid == 0) { S.sp_top = 1; S.stack_m[0] = 1; S.stack_c[0] = 0; }
    __syncthreads();
    while (S.sp_top > 0) {
      __syncthreads();
      const u32 M = S.stack_m[S.sp_top - 1], C = S.stack_c[S.sp_top - 1];
      __syncthreads();
      if (tid == 0) S.sp_top -= 1;
      // ---- level 0: insert this round's records
      for (u64 i = tid; i < n; i += MEM_BLOCK) {
        const u64 rec = A.part_rec[base + i];
        if ((((u32)(rec >> 11)) & (M - 1u)) != C) continue;
        if (!tbl_insert(S, rec >> 1, 1ull << (rec & 1ull), 1u, true)) break;
      }
      __syncthreads();
      if (S.overflow || S.live_n > TBL_CAP) {
        // clear, split this round in two by one more hash bit, retry later
        const u32 D = S.live_n < TBL_C ? S.live_n : TBL_C;
        for (u32 j = tid; j < D; j += MEM_BLOCK) { S.key[S.live[j]] = EMPTY; S.cnt[S.live[j]] = 0; }
        __syncthreads();
        if (tid == 0) {
          S.live_n = 0; S.overflow = 0; S.redos += 1;
          if (M >= (1u << 30) || S.sp_top + 2 > 64) {
            // hash bits exhausted (adversarial page ids): report, never spin
            atomicAdd(&A.acc->bad_mem, 1ull);
          } else {
            S.stack_m[S.sp_top] = 2 * M; S.stack_c[S.sp_top] = C;
            S.stack_m[S.sp_top + 1] = 2 * M; S.stack_c[S.sp_top + 1] = C + M;
            S.sp_top += 2;
          }
        }
        __syncthreads();
        continue;
      }
      // ---- levels 0..10
      for (int k = 0; k < AIWC_NSKIP; ++k) {
        const u32 D = S.live_n;
        const u32 sbit = 64u - A.pbits - (u32)k;   // space bit position in key_k
        u64 key[MAX_PER_THREAD];
        u32 c[MAX_PER_THREAD];
        u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
        u32 d1 = 0, ur0 = 0, uw0 = 0, ur1 = 0, uw1 = 0, dtot = 0;
#pragma unroll
        for (int q = 0; q < MAX_PER_THREAD; ++q) {
          const u32 j = tid + q * MEM_BLOCK;
          key[q] = EMPTY;
          c[q] = 0;
          if (j < D) {
            const u32 slot = S.live[j];
            const u64 w = S.key[slot];
            key[q] = w >> 2;
            c[q] = S.cnt[slot];
            const u32 s = (u32)(key[q] >> sbit) & 1u;
            u64 tl, th;
            if (c[q] < 256) { tl = S.tlo[s][c[q]]; th = S.thi[s][c[q]]; }
            else term_fx(c[q], N[s], tl, th);
            if (s) { u64 nl = lo1 + tl; hi1 += th + (nl < lo1); lo1 = nl; d1 += 1; }
            else   { u64 nl = lo0 + tl; hi0 += th + (nl < lo0); lo0 = nl; }
            dtot += 1;
            if (k == 0) {
              if (w & 1ull) { if (s) ur1 += 1; else ur0 += 1; }
              if (w & 2ull) { if (s) uw1 += 1; else uw0 += 1; }
            }
          }
        }
        // level statistics -> per-block accumulators
        wave_sum_u128(lo0, hi0);
        wave_sum_u128(lo1, hi1);
        const u64 sd1 = wave_sum_u64(d1), sdt = wave_sum_u64(dtot);
        if (lane == 0) {
          atomic_add_u128(&S.elo[0][k], &S.ehi[0][k], lo0, hi0);
          atomic_add_u128(&S.elo[1][k], &S.ehi[1][k], lo1, hi1);
          if (sd1) atomicAdd(&S.dist[1][k], sd1);
          if (sdt - sd1) atomicAdd(&S.dist[0][k], sdt - sd1);
        }
        if (k == 0) {
          const u64 a0 = wave_sum_u64(ur0), a1 = wave_sum_u64(uw0);
          const u64 a2 = wave_sum_u64(ur1), a3 = wave_sum_u64(uw1);
          if (lane == 0) {
            if (a0) atomicAdd(&S.ur[0], a0);
            if (a1) atomicAdd(&S.uw[0], a1);
            if (a2) atomicAdd(&S.ur[1], a2);
            if (a3) atomicAdd(&S.uw[1], a3);
          }
          // count spectrum: aggregate equal (space, count) pairs per wave
#pragma unroll
          for (int q = 0; q < MAX_PER_THREAD; ++q) {
            const u64 v = (key[q] == EMPTY) ? ~0ull
                                            : (((key[q] >> sbit) & 1ull) << 40) | (u64)c[q];
            u64 pend = __ballot(v != ~0ull);
            while (pend) {
              const int leader = __builtin_ctzll(pend);
              const u64 lv = __shfl(v, leader, 64);
              const u64 mask = __ballot(v == lv);
              if (lane == leader)
                spec_cache_add(S, A, (u32)(lv >> 40), lv & 0xFFFFFFFFFFull,
                               (u64)__builtin_popcountll(mask));
              pend &= ~mask;
            }
          }
        }
        __syncthreads();
        // free this level's slots
#pragma unroll
        for (int q = 0; q < MAX_PER_THREAD; ++q) {
          const u32 j = tid + q * MEM_BLOCK;
          if (j < D) { const u32 slot = S.live[j]; S.key[slot] = EMPTY; S.cnt[slot] = 0; }
        }
        __syncthreads();
        if (tid == 0) S.live_n = 0;
        __syncthreads();
        if (k + 1 < AIWC_NSKIP) {
#pragma unroll
          for (int q = 0; q < MAX_PER_THREAD; ++q)
            if (key[q] != EMPTY) tbl_insert(S, key[q] >> 1, 0ull, c[q], false);
          __syncthreads();
        }
      }
    }
    __syncthreads();
  }
  // ---- flush the block's accumulators
  __syncthreads();
  if (tid < 2 * AIWC_NSKIP) {
    const int s = tid / AIWC_NSKIP, k = tid % AIWC_NSKIP;
    if (S.dist[s][k]) atomicAdd(&A.acc->distinct[s][k], S.dist[s][k]);
    atomic_add_u128(&A.acc->ent_lo[s][k], &A.acc->ent_hi[s][k], S.elo[s][k], S.ehi[s][k]);
  }
  if (tid < 2) {
    if (S.ur[tid]) atomicAdd(&A.acc->uniq_r[tid], S.ur[tid]);
    if (S.uw[tid]) atomicAdd(&A.acc->uniq_w[tid], S.uw[tid]);
  }
  if (tid == 0 && S.redos) atomicAdd(&A.acc->redos, S.redos);
  for (u32 i = tid; i < 2 * SPEC_SLOTS; i += MEM_BLOCK) {
    const u32 s = i / SPEC_SLOTS, j = i % SPEC_SLOTS;
    if (S.spf[s][j]) global_spec_add(A, s, S.spf[s][j], S.spm[s][j]);
  }
}

}  // namespace

namespace aiwc_kernels {

size_t bucket_lds_bytes() { return sizeof(BucketShared); }

hipError_t launch_mem(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm) {
  if (!d.any_mem) return hipSuccess;
  const dim3 gh((unsigned)d.max_hist_blocks, d.n), gc((unsigned)((d.max_parts + 255) / 256), d.n);
  const dim3 g1(1, d.n), gb((unsigned)(d.max_parts < 256 ? d.max_parts : 256), d.n);
  const TraceArgs *b = d.batch;
  if (b) {
    if (d.vec) hipLaunchKernelGGL((k_mem_hist<true, true>), gh, dim3(MEM_BLOCK), 0, s, a, b);
    else hipLaunchKernelGGL((k_mem_hist<false, true>), gh, dim3(MEM_BLOCK), 0, s, a, b);
  } else {
    if (d.vec) hipLaunchKernelGGL((k_mem_hist<true, false>), gh, dim3(MEM_BLOCK), 0, s, a, b);
    else hipLaunchKernelGGL((k_mem_hist<false, false>), gh, dim3(MEM_BLOCK), 0, s, a, b);
  }
  AIWC_MARK(pm, "k_mem_hist", s);
  if (b) {
    hipLaunchKernelGGL(k_mem_colscan<true>, gc, dim3(256), 0, s, a, b);
    hipLaunchKernelGGL(k_mem_binscan<true>, g1, dim3(1024), 0, s, a, b);
  } else {
    hipLaunchKernelGGL(k_mem_colscan<false>, gc, dim3(256), 0, s, a, b);
    hipLaunchKernelGGL(k_mem_binscan<false>, g1, dim3(1024), 0, s, a, b);
  }
  AIWC_MARK(pm, "k_mem_scan", s);
  if (b) {
    if (d.vec) hipLaunchKernelGGL((k_mem_scatter<true, true>), gh, dim3(MEM_BLOCK), 0, s, a, b);
    else hipLaunchKernelGGL((k_mem_scatter<false, true>), gh, dim3(MEM_BLOCK), 0, s, a, b);
  } else {
    if (d.vec) hipLaunchKernelGGL((k_mem_scatter<true, false>), gh, dim3(MEM_BLOCK), 0, s, a, b);
    else hipLaunchKernelGGL((k_mem_scatter<false, false>), gh, dim3(MEM_BLOCK), 0, s, a, b);
  }
  AIWC_MARK(pm, "k_mem_scatter", s);
  if (b) hipLaunchKernelGGL(k_mem_bucket<true>, gb, dim3(MEM_BLOCK), 0, s, a, b);
  else hipLaunchKernelGGL(k_mem_bucket<false>, gb, dim3(MEM_BLOCK), 0, s, a, b);
  AIWC_MARK(pm, "k_mem_bucket", s);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
