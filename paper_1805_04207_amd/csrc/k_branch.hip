// k_branch.hip -- control metrics (Table I, Control rows).
//
// Reading of the paper's branch metrics (Implementation section: a
// per-site vector of outcomes; Metrics section: histories of 16 outcomes):
// every site keeps the history of its own previous m outcomes; an execution
// forms a window only once m earlier outcomes of its site exist.  For each
// key (site, history) with n0 / n1 following outcomes,
//   Yokota entropy  = sum [n0 log2(n/n0) + n1 log2(n/n1)] / N_w
//   linear entropy  = 2 sum min(n0, n1) / N_w.
//
// GPU plan:
//  1. k_br_pack     : (site, taken) -> u32 (site << 1 | taken), validated.
//  2. stable LSD radix sort by site, the site bits split evenly over passes
//     of at most 8 bits (4096 sites: 6 + 6): per-tile digit counts
//     (k_br_upsweep), one exclusive scan, and a stable scatter whose ranks
//     come from wavefront ballots (k_br_downsweep).  After it every site's
//     outcomes are contiguous and in stream order.
//  3. k_br_segments : start / end of every site segment.
//  4. k_br_windows  : work blocks of whole segments; each element's history
//     is m bits cut out of two 64-bit outcome ballots with funnel shifts;
//     (site, history) keys are counted in an LDS open-addressing table; the
//     table's entries give min(n0, n1) (exact integers) and the Yokota terms
//     (exact 128-bit fixed point sums, so the result is order independent).
//     A block whose distinct keys overflow the table is split by key hash
//     bits and redone.
//
// Variants (trace flags): zero-initialised histories mask the history bits
// that precede a site's first execution and keep every execution; the
// global history is cut from the stream-order outcomes in the pack kernel
// (k_br_pack_global) and travels with the site through the sort in 64-bit
// records (site << 33 | history << 1 | outcome, history bit 31 = "no full
// history yet"); the pattern entropy adds every key's window count to a
// 2^m-bin histogram of its history, reduced by k_br_pattern.
#include <type_traits>

#include "common.h"

namespace {

constexpr int BR_BLOCK = 256;
constexpr int BR_TILE = 4096;                 // elements per radix tile
constexpr int BR_ROUNDS = BR_TILE / BR_BLOCK; // 16
constexpr int WIN_BLOCK = 1024;
constexpr u64 WIN_T = 8192;                   // windows work-block size
constexpr u32 WT_C = 8192;                    // LDS table slots
constexpr u32 WT_CAP = 4096;
constexpr u64 EMPTY = ~0ull;

__device__ __forceinline__ bool global_history(const TraceArgs &A) {
  return (A.br_flags & AIWC_BRANCH_GLOBAL_HISTORY) != 0;
}

// site of a radix record: u32 records are site << 1 | outcome, u64 records
// site << 33 | history << 1 | outcome
template <typename R> __device__ __forceinline__ u32 rec_site(R v) {
  return (u32)(v >> (sizeof(R) == 8 ? 33 : 1));
}

// ------------------------------------------------------------------ pack
template <bool BATCH>
__global__ void k_br_pack(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (global_history(A)) return;
  u32 *out = A.br_a;
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u32 bad = 0;
  for (; i < A.n_branch; i += stride) {
    const u32 s = A.br_site[i];
    const u32 y = A.br_taken[i];
    if (s >= A.n_sites || y > 1u) { bad += 1; out[i] = 0; continue; }
    out[i] = (s << 1) | y;
  }
  u64 b = wave_sum_u64(bad);
  if (lane_id() == 0 && b) atomicAdd(&A.acc->bad_mem, b);
}

// Global history: one register over all branches in stream order.  A wave
// takes 64 consecutive executions; each lane's history is the m outcomes
// before it, cut from this chunk's and the previous chunk's outcome ballots
// (bits before the stream start are not-taken).
template <bool BATCH>
__global__ void k_br_pack_global(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!global_history(A)) return;
  u64 *out = reinterpret_cast<u64 *>(A.br_a);
  const int lane = lane_id();
  const u32 m = A.m;                                   // 1..31
  const u64 hmask = (1ull << m) - 1ull;
  const bool zero = (A.br_flags & AIWC_BRANCH_ZERO_HISTORY) != 0;
  const u64 wpb = blockDim.x / AIWC_WAVE;
  const u64 nwaves = (u64)gridDim.x * wpb;
  u32 bad = 0;
  for (u64 cb = ((u64)blockIdx.x * wpb + threadIdx.x / AIWC_WAVE) * AIWC_WAVE; cb < A.n_branch;
       cb += nwaves * AIWC_WAVE) {
    const u64 i = cb + lane;
    const bool valid = i < A.n_branch;
    const u32 s = valid ? A.br_site[i] : 0u;
    const u32 y = valid ? (u32)A.br_taken[i] : 0u;
    const u32 yp = (cb >= AIWC_WAVE) ? (u32)A.br_taken[i - AIWC_WAVE] : 0u;
    const u64 B = __ballot(valid && (y & 1u));
    const u64 Bp = __ballot((cb >= AIWC_WAVE) && (yp & 1u));
    const u32 sh = 64u + (u32)lane - m;                // in [33, 126]
    u64 E = (sh >= 64) ? (B >> (sh - 64)) : ((Bp >> sh) | (B << (64 - sh)));
    E &= hmask;
    if (!valid) continue;
    if (s >= A.n_sites || y > 1u) { bad += 1; out[i] = 0; continue; }
    const u32 hf = (u32)E | ((!zero && i < m) ? 0x80000000u : 0u);
    out[i] = ((u64)s << 33) | ((u64)hf << 1) | y;
  }
  u64 b = wave_sum_u64(bad);
  if (lane_id() == 0 && b) atomicAdd(&A.acc->bad_mem, b);
}

// -------------------------------------------------------------- radix sort
// R = u32 for per-site histories, u64 for the global history; a launch of
// either type skips the traces of the other (batches may mix them).
template <typename R> __device__ __forceinline__ bool rec_matches(const TraceArgs &A) {
  return (sizeof(R) == 8) == global_history(A);
}

// The site bits split evenly over the passes (at most 8 per pass): with 4096
// sites two passes of 6 bits, 64 digits each, rather than 8 + 4.
__device__ __forceinline__ u32 radix_bits(const TraceArgs &A) {
  u32 bits = 0;
  while (bits < 32 && (1u << bits) < A.n_sites) ++bits;
  return (bits + A.br_passes - 1) / A.br_passes;
}

template <bool BATCH, typename R>
__global__ void __launch_bounds__(BR_BLOCK) k_br_upsweep(TraceArgs A0, const TraceArgs *batch,
                                                        u32 pass) {
  __shared__ u32 h[256];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (pass >= A.br_passes || blockIdx.x >= A.br_tiles || !rec_matches<R>(A)) return;
  const R *in = reinterpret_cast<const R *>((pass & 1) ? A.br_b : A.br_a);
  const u64 n = A.n_branch, n_tiles = A.br_tiles;
  const u32 bpp = radix_bits(A);
  const u32 shift = (sizeof(R) == 8 ? 33u : 1u) + bpp * pass;
  const u32 dmask = (1u << bpp) - 1u;
  u32 *cnt = A.br_cnt;
  h[threadIdx.x] = 0;
  const u64 t = blockIdx.x;
  const u64 base = t * BR_TILE;
  R vals[BR_ROUNDS];
#pragma unroll
  for (int r = 0; r < BR_ROUNDS; ++r) {
    const u64 i = base + (u64)r * BR_BLOCK + threadIdx.x;
    vals[r] = i < n ? in[i] : ~(R)0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < BR_ROUNDS; ++r)
    if (vals[r] != ~(R)0) atomicAdd(&h[(u32)(vals[r] >> shift) & dmask], 1u);
  __syncthreads();
  cnt[(u64)threadIdx.x * n_tiles + t] = h[threadIdx.x];
}

// The stable scatter of one tile.  Each wavefront takes a contiguous quarter
// of the tile and ranks its records among its own records of the same digit
// (wavefront ballots, a running count per digit and wavefront in LDS: no
// block barrier per round); the quarters' counts then give each digit's
// start in the tile and each quarter's offset inside it, the tile is staged
// in LDS in digit order (stable: quarters, rounds and lanes in index order)
// and written out in runs, one run per digit.
template <bool BATCH, typename R>
__global__ void __launch_bounds__(BR_BLOCK) k_br_downsweep(TraceArgs A0, const TraceArgs *batch,
                                                          u32 pass) {
  constexpr int NW = BR_BLOCK / AIWC_WAVE;
  constexpr u32 SUB = BR_TILE / NW;            // records per wavefront
  constexpr int WR = (int)(SUB / AIWC_WAVE);   // rounds per wavefront
  __shared__ u32 gofs[256];
  __shared__ u32 start[256];
  __shared__ u32 wrun[NW][256];
  __shared__ u32 wsum[NW];
  __shared__ R staged[BR_TILE];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (pass >= A.br_passes || blockIdx.x >= A.br_tiles || !rec_matches<R>(A)) return;
  const R *in = reinterpret_cast<const R *>((pass & 1) ? A.br_b : A.br_a);
  R *out = reinterpret_cast<R *>((pass & 1) ? A.br_a : A.br_b);
  const u64 n = A.n_branch, n_tiles = A.br_tiles;
  const u32 bpp = radix_bits(A);
  const u32 shift = (sizeof(R) == 8 ? 33u : 1u) + bpp * pass;
  const u32 dmask = (1u << bpp) - 1u;
  const u32 *ofs = A.br_cnt;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / AIWC_WAVE;
  const u64 t = blockIdx.x;
  gofs[tid] = ofs[(u64)tid * n_tiles + t];
#pragma unroll
  for (int w = 0; w < NW; ++w) wrun[w][tid] = 0;
  const u64 base = t * BR_TILE;
  const u32 nt = (u32)((n - base) < (u64)BR_TILE ? (n - base) : (u64)BR_TILE);
  const u64 lt = (1ull << lane) - 1ull;
  const u32 k0 = (u32)wave * SUB + (u32)lane;
  R vals[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const u32 k = k0 + (u32)r * AIWC_WAVE;
    vals[r] = k < nt ? in[base + k] : (R)0;
  }
  __syncthreads();
  // digit << 16 | rank among this wavefront's records of that digit
  u32 slot[WR];
  u32 *run = wrun[wave];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const bool valid = k0 + (u32)r * AIWC_WAVE < nt;
    const u32 d = (u32)(vals[r] >> shift) & dmask;
    u64 peers = __ballot(valid);
    for (u32 b = 0; b < bpp; ++b) {
      const u64 m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const u32 rank = (u32)__builtin_popcountll(peers & lt);
    // every lane reads its digit's count before the group's first lane
    // adds the group (LDS operations of a wavefront complete in order)
    const u32 before = run[d];
    slot[r] = (d << 16) | (before + rank);
    if (valid && rank == 0) run[d] = before + (u32)__builtin_popcountll(peers);
  }
  __syncthreads();
  // per digit (one per thread): the quarters' exclusive prefix, in place,
  // and the tile's count; then the digits' starts in the tile
  {
    u32 x = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const u32 c = wrun[w][tid];
      wrun[w][tid] = x;
      x += c;
    }
    u32 incl = x;
#pragma unroll
    for (int o = 1; o < AIWC_WAVE; o <<= 1) {
      const u32 y = __shfl_up(incl, o, AIWC_WAVE);
      if (lane >= o) incl += y;
    }
    if (lane == AIWC_WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    u32 off = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) off += w < wave ? wsum[w] : 0u;
    start[tid] = off + incl - x;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    if (k0 + (u32)r * AIWC_WAVE >= nt) continue;
    const u32 d = slot[r] >> 16;
    staged[start[d] + run[d] + (slot[r] & 0xFFFFu)] = vals[r];
  }
  __syncthreads();
  for (u32 i = (u32)tid; i < nt; i += BR_BLOCK) {
    const R v = staged[i];
    const u32 d = (u32)(v >> shift) & dmask;
    out[gofs[d] + (i - start[d])] = v;
  }
}

// Generic exclusive scan of u32 values (totals < 2^32): block sums, a scan of
// the sums in one block, then per-block scans with the carried offset.
constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_PER = 8;
constexpr u64 SCAN_TILE = (u64)SCAN_BLOCK * SCAN_PER;

__device__ u32 block_exclusive_scan(u32 v, u32 *wsum, u32 &total) {
  u32 x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u32 y = __shfl_up(x, o, 64);
    if (lane_id() >= o) x += y;
  }
  if (lane_id() == 63) wsum[threadIdx.x / 64] = x;
  __syncthreads();
  u32 before = 0, tot = 0;
  for (u32 w = 0; w < blockDim.x / 64; ++w) {
    if (w < threadIdx.x / 64) before += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  total = tot;
  return before + x - v;
}

template <bool BATCH>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(TraceArgs A0, const TraceArgs *batch,
                                                           u32 pass) {
  __shared__ u32 wsum[16];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  const u64 n = 256ull * A.br_tiles;
  if (pass >= A.br_passes || blockIdx.x >= (n + SCAN_TILE - 1) / SCAN_TILE) return;
  const u32 *in = A.br_cnt;
  u32 *sums = A.scan_tmp;
  const u64 base = (u64)blockIdx.x * SCAN_TILE;
  u32 s = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    const u64 i = base + (u64)j * SCAN_BLOCK + threadIdx.x;
    if (i < n) s += in[i];
  }
  u32 tot;
  block_exclusive_scan(s, wsum, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <bool BATCH>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_sums(TraceArgs A0, const TraceArgs *batch,
                                                         u32 pass) {
  __shared__ u32 wsum[16];
  __shared__ u32 carry;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (pass >= A.br_passes) return;
  u32 *sums = A.scan_tmp;
  const u64 nb = (256ull * A.br_tiles + SCAN_TILE - 1) / SCAN_TILE;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (u64 b = 0; b < nb; b += SCAN_BLOCK) {
    const u64 i = b + threadIdx.x;
    const u32 v = i < nb ? sums[i] : 0u;
    u32 tot;
    const u32 ex = block_exclusive_scan(v, wsum, tot);
    const u32 c = carry;
    if (i < nb) sums[i] = c + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
}

template <bool BATCH>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(TraceArgs A0, const TraceArgs *batch,
                                                          u32 pass) {
  __shared__ u32 wsum[16];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  const u64 n = 256ull * A.br_tiles;
  if (pass >= A.br_passes || blockIdx.x >= (n + SCAN_TILE - 1) / SCAN_TILE) return;
  u32 *data = A.br_cnt;
  const u32 *sums = A.scan_tmp;
  const u64 base = (u64)blockIdx.x * SCAN_TILE;
  // each thread owns SCAN_PER consecutive elements
  u32 v[SCAN_PER];
  u32 s = 0;
  const u64 mine = base + (u64)threadIdx.x * SCAN_PER;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    v[j] = (mine + j < n) ? data[mine + j] : 0u;
    s += v[j];
  }
  u32 tot;
  u32 ex = block_exclusive_scan(s, wsum, tot) + sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (mine + j < n) data[mine + j] = ex;
    ex += v[j];
  }
}

// ------------------------------------------------------------- segments
template <bool BATCH, typename R>
__global__ void k_br_segments(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!rec_matches<R>(A)) return;
  const R *sorted = reinterpret_cast<const R *>(A.br_sorted);
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 n = A.n_branch;
  for (; i < n; i += stride) {
    const u32 s = rec_site(sorted[i]);
    if (i == 0 || rec_site(sorted[i - 1]) != s) A.seg_start[s] = (u32)i;
    if (i + 1 == n || rec_site(sorted[i + 1]) != s) A.seg_end[s] = (u32)(i + 1);
  }
}

// --------------------------------------------------------------- windows
struct WinShared {
  u64 key[WT_C];
  u32 n0[WT_C], n1[WT_C];
  uint16_t live[WT_C];
  u64 tlo[256], thi[256];     // Yokota terms for n0, n1 < 16
  u64 minsum, windows, ylo, yhi;
  u32 live_n, overflow, next;
  u32 stack_m[64], stack_c[64];
  u32 sp_top;
};

// n0 log2(n / n0) + n1 log2(n / n1), 2^-64 fixed point
__device__ __forceinline__ void yterm(u32 a, u32 b, u64 &lo, u64 &hi) {
  if (a == 0 || b == 0) { lo = hi = 0; return; }
  const double da = (double)a, db = (double)b;
  const double d = (da * log1p(db / da) + db * log1p(da / db)) * 1.4426950408889634074;
  to_fx64(d, lo, hi);
}

template <typename R>
__device__ __forceinline__ u64 range_begin(const TraceArgs &A, const R *sorted, u64 b) {
  const u64 x = b * WIN_T;
  if (x == 0) return 0;
  if (x >= A.n_branch) return A.n_branch;
  const u32 s = rec_site(sorted[x]);
  if (rec_site(sorted[x - 1]) != s) return x;
  return A.seg_end[s];
}

// Adds (a, b) to the counts of key.  Returns the slot, with fresh set when
// the key was new, or WT_C when the table is over its cap.  The live count
// lags by at most one block step of insertions (< WT_C - WT_CAP), so the table
// never fills.
__device__ __forceinline__ u32 win_insert(WinShared &S, u64 key, u32 a, u32 b, bool &fresh) {
  u32 slot = hash_slot(key, WT_C);
  fresh = false;
  while (true) {
    u64 w = S.key[slot];
    if (w == EMPTY) {
      if (S.live_n >= WT_CAP) { S.overflow = 1; return WT_C; }
      u64 old = atomicCAS(&S.key[slot], EMPTY, key);
      if (old == EMPTY) { fresh = true; w = key; }
      else w = old;
    }
    if (w == key) {
      if (a) atomicAdd(&S.n0[slot], a);
      if (b) atomicAdd(&S.n1[slot], b);
      return slot;
    }
    slot = (slot + 1 == WT_C) ? 0 : slot + 1;
  }
}

// LISTED: the ranges the sorting kernel left in the list (br_cnt, br_big_n
// (start, end) pairs), taken from a second queue.
template <bool BATCH, bool GLOBAL, bool LISTED>
__global__ void __launch_bounds__(WIN_BLOCK) k_br_windows(TraceArgs A0, const TraceArgs *batch) {
  using R = typename std::conditional<GLOBAL, u64, u32>::type;
  __shared__ WinShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_branch == 0 || global_history(A) != GLOBAL) return;
  const u64 nblk = LISTED ? A.acc->br_big_n : A.br_blocks;
  if (nblk == 0) return;
  unsigned long long *const queue =
      (unsigned long long *)(LISTED ? &A.acc->br_queue2 : &A.acc->br_queue);
  const R *sorted = reinterpret_cast<const R *>(A.br_sorted);
  const bool zero = (A.br_flags & AIWC_BRANCH_ZERO_HISTORY) != 0;
  u32 *const pat = A.pat_hist;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / AIWC_WAVE;
  const u32 m = A.m;
  const u64 hmask = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
  const u64 below = (1ull << lane) - 1ull;
  for (u32 i = tid; i < WT_C; i += WIN_BLOCK) { S.key[i] = EMPTY; S.n0[i] = 0; S.n1[i] = 0; }
  if (tid < 256) yterm(tid >> 4, tid & 15, S.tlo[tid], S.thi[tid]);
  if (tid == 0) {
    S.minsum = S.windows = S.ylo = S.yhi = 0; S.live_n = 0; S.overflow = 0;
    S.next = (u32)atomicAdd(queue, 1ull);
  }
  // per-thread sums over all work blocks, reduced once at the end
  u64 mins = 0, wins = 0, lo = 0, hi = 0;
  __syncthreads();
  while (true) {
    const u64 q = S.next;
    if (q >= nblk) break;
    __syncthreads();
    // the next work block is fetched while this one is processed
    if (tid == 0) S.next = (u32)atomicAdd(queue, 1ull);
    const u64 r0 = LISTED ? (u64)A.br_cnt[2 * q] : range_begin(A, sorted, q);
    const u64 r1 = LISTED ? (u64)A.br_cnt[2 * q + 1] : range_begin(A, sorted, q + 1);
    if (r1 <= r0) { __syncthreads(); continue; }
    // a block holds at most r1 - r0 keys: split by key-hash bits up front so
    // that each pass stays within the table's cap (a pass that still
    // overflows is split further)
    if (tid == 0) {
      u32 M0 = 1;
      while (M0 < 16 && (u64)M0 * WT_CAP < r1 - r0) M0 <<= 1;
      for (u32 c = 0; c < M0; ++c) { S.stack_m[c] = M0; S.stack_c[c] = c; }
      S.sp_top = M0;
    }
    __syncthreads();
    while (S.sp_top > 0) {
      __syncthreads();
      const u32 M = S.stack_m[S.sp_top - 1], C = S.stack_c[S.sp_top - 1];
      __syncthreads();
      if (tid == 0) S.sp_top -= 1;
      bool stop = false;
      for (u64 cb0 = r0 + (u64)wave * AIWC_WAVE; cb0 < r1; cb0 += 4ull * WIN_BLOCK) {
        // four chunks' loads in flight before any is used
        R pv[4];
        u32 pp[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const u64 cb = cb0 + (u64)q * WIN_BLOCK, i = cb + lane;
          pv[q] = (i < r1) ? sorted[i] : (R)0;
          if constexpr (!GLOBAL)
            pp[q] = (cb >= AIWC_WAVE && cb < r1) ? sorted[i - AIWC_WAVE] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const u64 cb = cb0 + (u64)q * WIN_BLOCK;
          if (cb >= r1) break;
          const u64 i = cb + lane;
          const bool valid = i < r1;
          const R v = pv[q];
          u64 key;
          bool windowed;
          if constexpr (GLOBAL) {
            // the history came with the record; bit 31 marks "no full
            // history yet" (the first m executions of the stream)
            const u32 hf = (u32)(v >> 1);
            key = ((u64)rec_site(v) << m) | (hf & hmask);
            windowed = valid && !(hf >> 31);
          } else {
            const u32 vp = pp[q];
            const u64 B = __ballot(valid && (v & 1u));
            const u64 Bp = __ballot((cb >= AIWC_WAVE) && (vp & 1u));
            const u32 s = v >> 1;
            const u32 sh = 64u + (u32)lane - m;         // in [32, 127]
            u64 E;
            if (sh >= 64) E = B >> (sh - 64);
            else E = (Bp >> sh) | (B << (64 - sh));
            E &= hmask;
            // d earlier executions of this site: bit j of E is the outcome
            // m - j executions back, so bits j < m - d precede the site's
            // first execution (not-taken when histories start at zero)
            const u64 d = i - A.seg_start[s];
            if (zero && d < m) E &= ~((1ull << (m - d)) - 1ull);
            key = ((u64)s << m) | E;
            windowed = valid && (zero || d >= m);
          }
          const bool use = windowed &&
                           (M == 1 || (((u32)((key * 0x9E3779B97F4A7C15ull) >> 40)) & (M - 1u)) == C);
          // runs of one key among neighbouring lanes (biased sites repeat
          // their history) are added once, by their first lane
          const u64 ends = run_ends(use ? key : EMPTY);
          const u64 Y = __ballot(use && (v & 1u));
          const bool head = use && (lane == 0 || ((ends >> (lane - 1)) & 1ull) != 0);
          bool fresh = false;
          u32 slot = WT_C;
          if (head && !stop) {
            const u32 e = (u32)__builtin_ctzll(ends & ~below);
            const u64 run = (e == 63 ? ~0ull : ((1ull << (e + 1)) - 1ull)) & ~below;
            const u32 ones = (u32)__builtin_popcountll(Y & run), len = e - (u32)lane + 1u;
            slot = win_insert(S, key, len - ones, ones, fresh);
            if (slot == WT_C) stop = true;
          }
          // new keys join the live list: one counter update per wavefront
          const u64 F = __ballot(fresh);
          if (F) {
            u32 base = 0;
            if (lane == 0) base = atomicAdd(&S.live_n, (u32)__builtin_popcountll(F));
            base = (u32)__builtin_amdgcn_readfirstlane((int)base);
            const u32 idx = base + (u32)__builtin_popcountll(F & below);
            if (fresh && idx < WT_C) S.live[idx] = (uint16_t)slot;
          }
        }
      }
      __syncthreads();
      const u32 D = S.live_n < WT_C ? S.live_n : WT_C;
      if (S.overflow || S.live_n > WT_CAP) {
        for (u32 j = tid; j < D; j += WIN_BLOCK) {
          const u32 slot = S.live[j];
          S.key[slot] = EMPTY; S.n0[slot] = 0; S.n1[slot] = 0;
        }
        __syncthreads();
        if (tid == 0) {
          S.live_n = 0; S.overflow = 0;
          if (M >= (1u << 23) || S.sp_top + 2 > 64) {
            atomicAdd(&A.acc->split_fail, 1ull);   // hash bits exhausted: report
          } else {
            S.stack_m[S.sp_top] = 2 * M; S.stack_c[S.sp_top] = C;
            S.stack_m[S.sp_top + 1] = 2 * M; S.stack_c[S.sp_top + 1] = C + M;
            S.sp_top += 2;
          }
        }
        __syncthreads();
        continue;
      }
      for (u32 j = tid; j < D; j += WIN_BLOCK) {
        const u32 slot = S.live[j];
        const u32 a = S.n0[slot], c = S.n1[slot];
        mins += a < c ? a : c;
        wins += (u64)a + c;
        u64 tl, th;
        if (a < 16 && c < 16) { tl = S.tlo[a * 16 + c]; th = S.thi[a * 16 + c]; }
        else yterm(a, c, tl, th);
        u64 nl = lo + tl; hi += th + (nl < lo); lo = nl;
        if (pat) atomicAdd(&pat[S.key[slot] & hmask], a + c);
        S.key[slot] = EMPTY; S.n0[slot] = 0; S.n1[slot] = 0;
      }
      __syncthreads();
      if (tid == 0) S.live_n = 0;
      __syncthreads();
    }
    __syncthreads();
  }
  mins = wave_sum_u64(mins);
  wins = wave_sum_u64(wins);
  wave_sum_u128(lo, hi);
  if (lane == 0) {
    if (mins) atomicAdd(&S.minsum, mins);
    if (wins) atomicAdd(&S.windows, wins);
    atomic_add_u128(&S.ylo, &S.yhi, lo, hi);
  }
  __syncthreads();
  if (tid == 0) {
    if (S.minsum) atomicAdd(&A.acc->br_minsum, S.minsum);
    if (S.windows) atomicAdd(&A.acc->br_windows, S.windows);
    atomic_add_u128(&A.acc->yok_lo, &A.acc->yok_hi, S.ylo, S.yhi);
  }
}

// ------------------------------------------------ windows by LDS sort
// A work block whose windows fit on chip is counted here rather than in a
// hash table.  Each windowed execution becomes the word
// (site - range's first site) << (m + 1) | history << 1 | outcome.
//  - Few keys (key bits <= DENSE_BITS): a direct LDS table of counters, n0
//    in the low and n1 in the high half of a key's word, in passes of
//    DENSE_WORDS keys; each wave lists the keys it touched first, and only
//    listed words are read back (and cleared).
//  - More keys: an LSD radix sort of the words in LDS (digits of at most 9
//    bits; each element's digit rank from wavefront ballots, kept in
//    registers from the counting step to the scatter step); between the
//    boundaries of equal words, a key's run with outcome 0 is n0 and the
//    run with outcome 1 is n1.
// A block larger than a sort block is its leading whole segments (fewer
// than WIN_T records) and its last segment; a last segment of at least
// AIWC_HOT_MIN records with m <= 16 is a hot segment: it gets a table of 2^m
// 64-bit counters (n0 | n1 << 32) in scratch, k_br_windows_hot counts its
// pieces in parallel into that table and k_br_hot_terms reads it.  Ranges that fit
// none of these are listed (br_cnt, br_big_n) for the hash-table kernel,
// which runs last on the same stream.
constexpr u32 SORT_CAP = AIWC_SORT_CAP;
constexpr u32 SORT_WAVES = WIN_BLOCK / AIWC_WAVE;   // 16
constexpr u32 SORT_CH = SORT_CAP / WIN_BLOCK;       // chunks of 64 per wave and pass
constexpr u32 DIG_MAX = 9;
constexpr u32 NBIN = 1u << DIG_MAX;
constexpr u32 DENSE_BITS = 16;                      // key bits counted in a direct table
constexpr u32 DENSE_WORDS = 2 * SORT_CAP;           // table words per pass

struct SortShared {
  u32 keys[2 * SORT_CAP];           // two key buffers, or one direct count table
  uint16_t off[SORT_WAVES][NBIN];   // per wave digit counts / offsets, or key lists
  u64 tlo[256], thi[256];
  u32 wsum[NBIN / AIWC_WAVE];
  u64 minsum, windows, ylo, yhi;
  u32 n, next, dirty, over, hidx, total;
};

// Smallest set bit at position >= p (a set bit at or after p must exist).
__device__ __forceinline__ u32 next_set(const u32 *bm, u32 p) {
  u32 w = p >> 5;
  u32 x = bm[w] & (~0u << (p & 31));
  while (x == 0) x = bm[++w];
  return (w << 5) + (u32)__builtin_ctz(x);
}

// The records [r0, r1) of the site-sorted stream, s0 the site of r0.
struct WordRange {
  const u32 *sorted;
  u64 r0, r1;
  u32 s0, m;
  u64 hmask;
  bool zero;
};

// The range's windowed executions as words (~0 where the execution forms no
// window), handed chunk by chunk to emit(t, word) with the whole wavefront
// present.  Each wave takes a run of consecutive 64-record chunks, all of
// whose loads are in flight at once; the chunk before its first supplies
// the carried ballots (it may lie before r0: the previous records of the
// same site give the history).  History: m outcome bits cut from the
// ballots of two chunks (bit j = the execution m - j back).  Records are
// sorted by site, so an execution has m earlier ones of its site exactly
// when no site boundary lies among the last m positions; the zero-history
// variant clears the history bits before the latest boundary.
template <class Emit>
__device__ __forceinline__ void range_words(const WordRange &R, u32 wave, int lane, Emit &&emit) {
  const u32 m = R.m;
  const u64 nch = (R.r1 - R.r0 + AIWC_WAVE - 1) / AIWC_WAVE;
  const u64 cpw = (nch + SORT_WAVES - 1) / SORT_WAVES;     // <= 16
  const u64 c0 = (u64)wave * cpw;
  const u64 p0 = R.r0 + c0 * AIWC_WAVE;                    // first record of the wave
  u32 pv[SORT_CH];
#pragma unroll
  for (u32 t = 0; t < SORT_CH; ++t) {
    const u64 i = p0 + (u64)t * AIWC_WAVE + lane;
    pv[t] = (t < cpw && i < R.r1) ? R.sorted[i] : 0u;
  }
  const bool have_prev = p0 >= AIWC_WAVE && c0 < nch;
  const u32 vprev = have_prev ? R.sorted[p0 - AIWC_WAVE + lane] : 0u;
  u64 Bo = __ballot(have_prev && (vprev & 1u));
  const u32 sp = (u32)__shfl((int)(vprev >> 1), (int)(lane == 0 ? 0 : lane - 1), AIWC_WAVE);
  u64 Bs = have_prev ? __ballot((vprev >> 1) != sp) : ~0ull;
  u32 last_site = (u32)__builtin_amdgcn_readlane((int)(vprev >> 1), 63);
  if (!have_prev) last_site = 0xFFFFFFFFu;
#pragma unroll
  for (u32 t = 0; t < SORT_CH; ++t) {
    if (t >= cpw || c0 + t >= nch) { emit(t, ~0u); continue; }
    const u64 i = p0 + (u64)t * AIWC_WAVE + lane;
    const bool valid = i < R.r1;
    const u32 v = pv[t], st = v >> 1;
    const u32 left = (u32)__shfl((int)st, (int)(lane == 0 ? 0 : lane - 1), AIWC_WAVE);
    const u32 before = lane == 0 ? last_site : left;
    const u64 B = __ballot(valid && (v & 1u));
    const u64 Bb = __ballot(!valid || st != before);
    const u32 sh = 64u + (u32)lane - m;                 // in [34, 126]
    u64 E = (sh >= 64) ? (B >> (sh - 64)) : ((Bo >> sh) | (B << (64 - sh)));
    E &= R.hmask;
    const u32 sb = sh + 1;                              // boundaries at the last m positions
    u64 F = (sb >= 64) ? (Bb >> (sb - 64)) : ((Bs >> sb) | (Bb << (64 - sb)));
    F &= R.hmask;
    bool windowed;
    if (R.zero) {
      // a boundary at window bit j starts the segment at history bit j: the
      // bits below it precede the site's first execution
      if (F) {
        const u32 q = 63u - (u32)__builtin_clzll(F);
        E &= ~((2ull << q) - 1ull);
      }
      windowed = valid;
    } else {
      windowed = valid && F == 0;
    }
    emit(t, windowed ? (u32)((((u64)(st - R.s0)) << (m + 1)) | (E << 1) | (v & 1u)) : ~0u);
    Bo = B;
    Bs = Bb;
    last_site = (u32)__builtin_amdgcn_readlane((int)st, 63);
  }
}

// Direct-table count of the range's words (keys below 2^kb); take(key, n0,
// n1) for every key present.  The table is left cleared.
template <class Take>
__device__ __forceinline__ void dense_count(SortShared &S, const WordRange &R, u32 kb, int tid,
                                            u32 wave, int lane, u64 below, Take &&take) {
  u32 *T = S.keys;
  if (S.dirty) {
    for (u32 j = tid; j < DENSE_WORDS; j += WIN_BLOCK) T[j] = 0;
    __syncthreads();
  }
  const u32 nkeys = 1u << kb;
  const u32 pk = nkeys < DENSE_WORDS ? nkeys : DENSE_WORDS;
  uint16_t *const list = &S.off[wave][0];
  for (u32 pass = 0; pass * pk < nkeys; ++pass) {
    u32 nl = 0;   // wave-uniform list length
    range_words(R, wave, lane, [&](u32, u32 w) {
      const bool mine = w != ~0u && (w >> 1) / pk == pass;
      u32 old = 1;
      if (mine) old = atomicAdd(&T[(w >> 1) % pk], (w & 1u) ? 0x10000u : 1u);
      const u64 F = __ballot(mine && old == 0);
      const u32 at = nl + (u32)__builtin_popcountll(F & below);
      if (mine && old == 0 && at < NBIN) list[at] = (uint16_t)((w >> 1) % pk);
      nl += (u32)__builtin_popcountll(F);
    });
    if (lane == 0 && nl > NBIN) S.over = 1;   // a list overflowed: read every word
    __syncthreads();
    auto one = [&](u32 j) {
      const u32 x = T[j];
      if (!x) return;
      T[j] = 0;
      take(pass * pk + j, x & 0xFFFFu, x >> 16);
    };
    if (S.over) {
      for (u32 j = tid; j < pk; j += WIN_BLOCK) one(j);
    } else {
      for (u32 q = (u32)lane; q < nl; q += AIWC_WAVE) one((u32)list[q]);
    }
    __syncthreads();
    if (tid == 0) S.over = 0;
    __syncthreads();
  }
  if (tid == 0) S.dirty = 0;
}

// Sorted count of the range's words (kbits <= 31 bits with the outcome, at
// most SORT_CAP records); take(key, n0, n1) for every key present.
template <class Take>
__device__ __forceinline__ void sort_count(SortShared &S, const WordRange &R, u32 kbits, int tid,
                                           u32 wave, int lane, u64 below, Take &&take) {
  {
    u32 kw[SORT_CH];
    range_words(R, wave, lane, [&](u32 t, u32 w) { kw[t] = w; });
    u32 cnt = 0;
#pragma unroll
    for (u32 t = 0; t < SORT_CH; ++t) cnt += (u32)__builtin_popcountll(__ballot(kw[t] != ~0u));
    u32 base = 0;
    if (lane == 0 && cnt) base = atomicAdd(&S.n, cnt);
    base = (u32)__builtin_amdgcn_readfirstlane((int)base);
#pragma unroll
    for (u32 t = 0; t < SORT_CH; ++t) {
      const u64 W = __ballot(kw[t] != ~0u);
      if (kw[t] != ~0u) S.keys[base + (u32)__builtin_popcountll(W & below)] = kw[t];
      base += (u32)__builtin_popcountll(W);
    }
  }
  if (tid == 0) S.dirty = 1;
  __syncthreads();
  const u32 N = S.n;
  // LSD radix passes over bits [0, kbits)
  u32 *src = S.keys, *dst = S.keys + SORT_CAP;
  const u32 per = ((N + SORT_WAVES - 1) / SORT_WAVES + 63u) & ~63u;   // <= 1024
  const u32 w0 = wave * per;
  const u32 passes = (kbits + DIG_MAX - 1) / DIG_MAX;
  u32 shift = 0;
  for (u32 p = 0; p < passes; ++p) {
    const u32 db = (kbits - shift + (passes - p) - 1) / (passes - p);
    const u32 nbin = 1u << db, dmask = nbin - 1u;
    for (u32 j = (u32)lane; j < nbin; j += AIWC_WAVE) S.off[wave][j] = 0;
    // per element: the key, and its in-chunk rank | group leader << 6 |
    // group size << 12 (the size on the leader only); ranks from ballots ...
    u32 key[SORT_CH], rk[SORT_CH];
#pragma unroll
    for (u32 c = 0; c < SORT_CH; ++c) {
      const u32 e = w0 + c * AIWC_WAVE + (u32)lane;
      const bool ok = c * AIWC_WAVE < per && e < N;
      const u32 kv = ok ? src[e] : 0u;
      key[c] = kv;
      rk[c] = (u32)lane << 6;
      const u64 any = __ballot(ok);
      if (any == 0) continue;
      const u32 dg = (kv >> shift) & dmask;
      u64 peers = any;
      for (u32 bb = 0; bb < db; ++bb) {
        const bool bit = (dg >> bb) & 1u;
        const u64 bm = __ballot(bit);
        peers &= bit ? bm : ~bm;
      }
      if (ok) {
        const u32 ld = (u32)__builtin_ctzll(peers);
        rk[c] = (u32)__builtin_popcountll(peers & below) | (ld << 6);
        if ((u32)lane == ld) rk[c] |= (u32)__builtin_popcountll(peers) << 12;
      }
    }
    // ... every chunk's group counts added in chunk order (LDS atomics of one
    // wave complete in issue order), two u16 counters per word ...
    u32 pos[SORT_CH];
#pragma unroll
    for (u32 c = 0; c < SORT_CH; ++c) {
      pos[c] = 0;
      const u32 g = rk[c] >> 12;
      if (g) {
        const u32 dg = (key[c] >> shift) & dmask, hs = (dg & 1u) * 16u;
        u32 *w = reinterpret_cast<u32 *>(&S.off[wave][dg & ~1u]);
        pos[c] = (atomicAdd(w, g << hs) >> hs) & 0xFFFFu;
      }
    }
    // ... and the groups' bases handed to their lanes: pos = rank in wave
#pragma unroll
    for (u32 c = 0; c < SORT_CH; ++c)
      pos[c] = (u32)__shfl((int)pos[c], (int)((rk[c] >> 6) & 63u), AIWC_WAVE) + (rk[c] & 63u);
    __syncthreads();
    // offsets in (digit, wave) order
    u32 excl = 0;
    if ((u32)tid < nbin) {
      u32 run = 0;
#pragma unroll
      for (u32 w = 0; w < SORT_WAVES; ++w) run += S.off[w][tid];
      u32 x = run;
      for (int o = 1; o < AIWC_WAVE; o <<= 1) {
        const u32 y = (u32)__shfl_up((int)x, o, AIWC_WAVE);
        if (lane >= o) x += y;
      }
      const u32 last = nbin < AIWC_WAVE ? nbin - 1u : (u32)AIWC_WAVE - 1u;
      if ((u32)lane == last) S.wsum[wave] = x;
      excl = x - run;
    }
    __syncthreads();
    if ((u32)tid < nbin) {
      u32 base = excl;
      for (u32 w = 0; w < wave; ++w) base += S.wsum[w];
#pragma unroll
      for (u32 w = 0; w < SORT_WAVES; ++w) {
        const u32 c = S.off[w][tid];
        S.off[w][tid] = (uint16_t)base;
        base += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (u32 c = 0; c < SORT_CH; ++c) {
      const u32 e = w0 + c * AIWC_WAVE + (u32)lane;
      if (c * AIWC_WAVE < per && e < N) {
        const u32 dg = (key[c] >> shift) & dmask;
        dst[S.off[wave][dg] + pos[c]] = key[c];
      }
    }
    __syncthreads();
    u32 *t = src; src = dst; dst = t;
    shift += db;
  }
  // boundaries of equal words as a bitmap (bit N: a sentinel), for the runs
  // that leave their chunk
  u32 *bm = dst;
  for (u32 cb = wave * AIWC_WAVE; cb < N; cb += WIN_BLOCK) {
    const u32 e = cb + (u32)lane;
    const bool ok = e < N;
    const u32 v = ok ? src[e] : 0u;
    const u32 vq = (ok && e > 0) ? src[e - 1] : 0u;
    const u64 Bd = __ballot(ok && (e == 0 || v != vq));
    if (lane == 0) bm[cb >> 5] = (u32)Bd;
    if (lane == 1) bm[(cb >> 5) + 1] = (u32)(Bd >> 32);
  }
  __syncthreads();
  if (tid == 0) {
    if ((N & 63) == 0) { bm[N >> 5] = 0; bm[(N >> 5) + 1] = 0; }
    bm[N >> 5] |= 1u << (N & 31);
  }
  __syncthreads();
  // every key's (n0, n1) from its runs: a run's end is the next boundary,
  // found in the chunk's boundary ballot unless the run leaves the chunk
  for (u32 cb = wave * AIWC_WAVE; cb < N; cb += WIN_BLOCK) {
    const u32 e = cb + (u32)lane;
    const bool ok = e < N;
    const u32 v = ok ? src[e] : 0u;
    const u32 vq = (ok && e > 0) ? src[e - 1] : 0u;
    u64 Bd = __ballot(ok && (e == 0 || v != vq));
    if (N - cb < 64) Bd |= 1ull << (N - cb);            // the sentinel
    const bool head = ok && ((Bd >> lane) & 1ull);
    const u64 above = (lane == 63) ? 0ull : (Bd & ~((2ull << lane) - 1ull));
    const u32 e1 = above ? cb + (u32)__builtin_ctzll(above) : 0u;
    const u32 j1 = above ? (u32)__builtin_ctzll(above) : 0u;
    const u32 v1s = (u32)__shfl((int)v, (int)(j1 & 63u), AIWC_WAVE);
    if (!head) continue;
    if ((v & 1u) && e > 0 && (vq >> 1) == (v >> 1)) continue;   // its key's second run
    const u32 end1 = above ? e1 : next_set(bm, cb + AIWC_WAVE);
    u32 a, c;
    if (v & 1u) { a = 0; c = end1 - e; }
    else {
      a = end1 - e;
      c = 0;
      if (end1 < N) {
        const bool inside = end1 < cb + AIWC_WAVE;
        const u32 v1 = inside ? v1s : src[end1];
        if (v1 == (v | 1u)) {
          u64 above2 = 0;
          if (inside) {
            const u32 j = end1 - cb;
            above2 = (j == 63) ? 0ull : (Bd & ~((2ull << j) - 1ull));
          }
          const u32 end2 = above2 ? cb + (u32)__builtin_ctzll(above2)
                                  : next_set(bm, inside ? cb + AIWC_WAVE : end1 + 1);
          c = end2 - end1;
        }
      }
    }
    take(v >> 1, a, c);
  }
}

// Window statistics of keys with counts (n0, n1): exact integer sums and
// 2^-64 fixed-point Yokota terms (order independent).
struct Terms {
  u64 mins = 0, wins = 0, lo = 0, hi = 0;
  __device__ __forceinline__ void add(u32 a, u32 c, const u64 *tlo, const u64 *thi) {
    mins += a < c ? a : c;
    wins += (u64)a + c;
    u64 tl, th;
    if (a < 16 && c < 16) { tl = tlo[a * 16 + c]; th = thi[a * 16 + c]; }
    else yterm(a, c, tl, th);
    const u64 nl = lo + tl;
    hi += th + (nl < lo);
    lo = nl;
  }
  // block reduction into the trace's accumulators (all threads call it)
  __device__ __forceinline__ void flush(const TraceArgs &A, u64 *sm) {
    mins = wave_sum_u64(mins);
    wins = wave_sum_u64(wins);
    wave_sum_u128(lo, hi);
    if (threadIdx.x == 0) sm[0] = sm[1] = sm[2] = sm[3] = 0;
    __syncthreads();
    if (lane_id() == 0) {
      if (mins) atomicAdd(&sm[0], mins);
      if (wins) atomicAdd(&sm[1], wins);
      atomic_add_u128(&sm[2], &sm[3], lo, hi);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (sm[0]) atomicAdd(&A.acc->br_minsum, sm[0]);
      if (sm[1]) atomicAdd(&A.acc->br_windows, sm[1]);
      atomic_add_u128(&A.acc->yok_lo, &A.acc->yok_hi, sm[2], sm[3]);
    }
  }
};

__device__ __forceinline__ void list_range(const TraceArgs &A, u64 r0, u64 r1) {
  const u64 k = atomicAdd(&A.acc->br_big_n, 1ull);
  A.br_cnt[2 * k] = (u32)r0;
  A.br_cnt[2 * k + 1] = (u32)r1;
}

template <bool BATCH>
__global__ void __launch_bounds__(WIN_BLOCK) k_br_windows_sort(TraceArgs A0, const TraceArgs *batch) {
  __shared__ SortShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_branch == 0 || global_history(A)) return;
  const u32 *sorted = A.br_sorted;
  const bool zero = (A.br_flags & AIWC_BRANCH_ZERO_HISTORY) != 0;
  u32 *const pat = A.pat_hist;
  const int tid = threadIdx.x, lane = lane_id();
  const u32 wave = (u32)__builtin_amdgcn_readfirstlane(tid / AIWC_WAVE);
  const u32 m = A.m;
  const u64 hmask = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
  const u64 below = (1ull << lane) - 1ull;
  if (tid < 256) yterm(tid >> 4, tid & 15, S.tlo[tid], S.thi[tid]);
  if (tid == 0) {
    S.dirty = 1;
    S.over = 0;
    S.next = (u32)atomicAdd(&A.acc->br_queue, 1ull);
  }
  Terms acc;
  auto take = [&](u32 key, u32 a, u32 c) {
    acc.add(a, c, S.tlo, S.thi);
    if (pat) atomicAdd(&pat[key & hmask], a + c);
  };
  // a range of whole segments of at most SORT_CAP records: counted here, or
  // listed for the hash-table kernel when its keys exceed 31 bits
  auto count_range = [&](u64 ra, u64 rb) {
    const u32 s0 = sorted[ra] >> 1, sl = sorted[rb - 1] >> 1;
    const u32 sbits = (sl == s0) ? 0u : 32u - (u32)__builtin_clz(sl - s0);
    if (sbits + m + 1 > 31) {
      if (tid == 0) list_range(A, ra, rb);
      return;
    }
    if (tid == 0) S.n = 0;
    __syncthreads();
    const WordRange R{sorted, ra, rb, s0, m, hmask, zero};
    if (sbits + m <= DENSE_BITS) dense_count(S, R, sbits + m, tid, wave, lane, below, take);
    else sort_count(S, R, sbits + m + 1, tid, wave, lane, below, take);
    __syncthreads();
  };
  // the next work block, fetched at a block's start and published at its
  // end (the queue's latency hides behind the block's work)
  u32 pending = 0;
  __syncthreads();
  while (true) {
    const u64 b = S.next;
    if (b >= A.br_blocks) break;
    __syncthreads();
    if (tid == 0) pending = (u32)atomicAdd(&A.acc->br_queue, 1ull);
    const u64 r0 = range_begin(A, sorted, b), r1 = range_begin(A, sorted, b + 1);
    if (r1 > r0 && r1 - r0 <= SORT_CAP) {
      count_range(r0, r1);
    } else if (r1 > r0) {
      // leading whole segments (within one WIN_T stride) and the last segment
      const u64 ls = A.seg_start[sorted[r1 - 1] >> 1];
      if (ls > r0) count_range(r0, ls);
      if (r1 - ls <= SORT_CAP) {
        count_range(ls, r1);
      } else if (A.br_hot_cap && m <= 16 && r1 - ls >= AIWC_HOT_MIN) {
        if (tid == 0) {
          const u32 k = (u32)atomicAdd(&A.acc->br_hot_n, 1ull);
          S.hidx = k;
          if (k < A.br_hot_cap) { A.br_hot_list[2 * k] = (u32)ls; A.br_hot_list[2 * k + 1] = (u32)r1; }
          else list_range(A, ls, r1);
        }
        __syncthreads();
        const u32 k = S.hidx;
        if (k < A.br_hot_cap)   // its table starts at zero
          for (u32 j = tid; j < (1u << m); j += WIN_BLOCK) A.br_hot_tab[((u64)k << m) + j] = 0;
      } else if (tid == 0) {
        list_range(A, ls, r1);
      }
    }
    if (tid == 0) S.next = pending;
    __syncthreads();
  }
  acc.flush(A, &S.minsum);
}

// Pieces of SORT_CAP records of the hot segments, counted in LDS and added
// to their segment's table with 64-bit atomics.
template <bool BATCH>
__global__ void __launch_bounds__(WIN_BLOCK) k_br_windows_hot(TraceArgs A0, const TraceArgs *batch) {
  __shared__ SortShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_branch == 0 || global_history(A) || A.br_hot_cap == 0) return;
  const u32 nh = (u32)(A.acc->br_hot_n < A.br_hot_cap ? A.acc->br_hot_n : A.br_hot_cap);
  if (nh == 0) return;
  const u32 *sorted = A.br_sorted;
  const int tid = threadIdx.x, lane = lane_id();
  const u32 wave = (u32)__builtin_amdgcn_readfirstlane(tid / AIWC_WAVE);
  const u32 m = A.m;
  const u64 hmask = (1ull << m) - 1ull;
  const u64 below = (1ull << lane) - 1ull;
  const bool zero = (A.br_flags & AIWC_BRANCH_ZERO_HISTORY) != 0;
  if (tid == 0) {
    u32 total = 0;
    for (u32 e = 0; e < nh; ++e)
      total += (A.br_hot_list[2 * e + 1] - A.br_hot_list[2 * e] + SORT_CAP - 1) / SORT_CAP;
    S.total = total;
    S.dirty = 1;
    S.over = 0;
    S.next = (u32)atomicAdd(&A.acc->br_piece_q, 1ull);
  }
  u32 pending = 0;
  __syncthreads();
  while (true) {
    u32 p = S.next;
    if (p >= S.total) break;
    __syncthreads();
    if (tid == 0) pending = (u32)atomicAdd(&A.acc->br_piece_q, 1ull);
    u32 e = 0, st = 0, en = 0;
    for (; e < nh; ++e) {
      st = A.br_hot_list[2 * e];
      en = A.br_hot_list[2 * e + 1];
      const u32 np = (en - st + SORT_CAP - 1) / SORT_CAP;
      if (p < np) break;
      p -= np;
    }
    const u64 x0 = (u64)st + (u64)p * SORT_CAP;
    const u64 x1 = (u64)en < x0 + SORT_CAP ? (u64)en : x0 + SORT_CAP;
    const WordRange R{sorted, x0, x1, sorted[st] >> 1, m, hmask, zero};
    unsigned long long *tab = A.br_hot_tab + ((u64)e << m);
    dense_count(S, R, m, tid, wave, lane, below, [&](u32 key, u32 a, u32 c) {
      atomicAdd(&tab[key], (unsigned long long)a | ((unsigned long long)c << 32));
    });
    if (tid == 0) S.next = pending;
    __syncthreads();
  }
}

// The hot segments' tables: every history's (n0, n1) to the window sums.
template <bool BATCH>
__global__ void __launch_bounds__(256) k_br_hot_terms(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u64 tlo[256], thi[256], sm[4];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_branch == 0 || global_history(A) || A.br_hot_cap == 0) return;
  const u64 nh = A.acc->br_hot_n < A.br_hot_cap ? A.acc->br_hot_n : A.br_hot_cap;
  if (nh == 0) return;
  yterm(threadIdx.x >> 4, threadIdx.x & 15, tlo[threadIdx.x], thi[threadIdx.x]);
  __syncthreads();
  const u32 m = A.m;
  const u64 hmask = (1ull << m) - 1ull;
  Terms acc;
  const u64 n = nh << m;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256) {
    const unsigned long long x = A.br_hot_tab[i];
    if (!x) continue;
    const u32 a = (u32)x, c = (u32)(x >> 32);
    acc.add(a, c, tlo, thi);
    if (A.pat_hist) atomicAdd(&A.pat_hist[i & hmask], a + c);
  }
  acc.flush(A, sm);
}

// Pattern entropy: sum over the 2^m history patterns of c log2(N_w / c),
// each term converted to 2^-64 fixed point, so the sum is exact and order
// independent; N_w is the window count k_br_windows accumulated.
template <bool BATCH>
__global__ void __launch_bounds__(256) k_br_pattern(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!A.pat_hist || A.n_branch == 0) return;
  const u64 nbins = 1ull << A.m;
  const double N = (double)A.acc->br_windows;
  u64 lo = 0, hi = 0;
  for (u64 b = (u64)blockIdx.x * blockDim.x + threadIdx.x; b < nbins;
       b += (u64)gridDim.x * blockDim.x) {
    const u32 c = A.pat_hist[b];
    if (c == 0) continue;
    u64 tl, th;
    to_fx64((double)c * log2(N / (double)c), tl, th);
    const u64 nl = lo + tl;
    hi += th + (nl < lo);
    lo = nl;
  }
  wave_sum_u128(lo, hi);
  if (lane_id() == 0) atomic_add_u128(&A.acc->pat_lo, &A.acc->pat_hi, lo, hi);
}

}  // namespace

namespace aiwc_kernels {

u64 scan_tmp_elems(u64 n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }
u64 br_tiles_for(u64 n) { return (n + BR_TILE - 1) / BR_TILE; }
u64 br_blocks_for(u64 n) { return (n + WIN_T - 1) / WIN_T; }

u64 scan_blocks_for(u64 n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

// Launches of the per-site (u32 records) and global-history (u64 records)
// variants; each kernel skips the traces of the other variant.
template <bool B>
static void branch_launches(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                            StageMarks *pm) {
  const TraceArgs *b = d.batch;
  u64 gx = (d.max_tiles * BR_TILE + 255) / 256;
  if (gx > 8192) gx = 8192;
  if (gx == 0) gx = 1;
  const dim3 gp((unsigned)gx, d.n);
  if (d.any_local) hipLaunchKernelGGL(k_br_pack<B>, gp, dim3(256), 0, s, a, b);
  if (d.any_global) hipLaunchKernelGGL(k_br_pack_global<B>, gp, dim3(256), 0, s, a, b);
  AIWC_MARK(pm, "k_br_pack", s);
  const dim3 gt((unsigned)d.max_tiles, d.n), gs((unsigned)d.max_scan_blocks, d.n), g1(1, d.n);
  for (u32 p = 0; p < d.max_passes; ++p) {
    if (d.any_local) hipLaunchKernelGGL((k_br_upsweep<B, u32>), gt, dim3(BR_BLOCK), 0, s, a, b, p);
    if (d.any_global) hipLaunchKernelGGL((k_br_upsweep<B, u64>), gt, dim3(BR_BLOCK), 0, s, a, b, p);
    hipLaunchKernelGGL(k_scan_reduce<B>, gs, dim3(SCAN_BLOCK), 0, s, a, b, p);
    hipLaunchKernelGGL(k_scan_sums<B>, g1, dim3(SCAN_BLOCK), 0, s, a, b, p);
    hipLaunchKernelGGL(k_scan_apply<B>, gs, dim3(SCAN_BLOCK), 0, s, a, b, p);
    if (d.any_local) hipLaunchKernelGGL((k_br_downsweep<B, u32>), gt, dim3(BR_BLOCK), 0, s, a, b, p);
    if (d.any_global) hipLaunchKernelGGL((k_br_downsweep<B, u64>), gt, dim3(BR_BLOCK), 0, s, a, b, p);
  }
  AIWC_MARK(pm, "k_br_sort", s);
  if (d.any_local) hipLaunchKernelGGL((k_br_segments<B, u32>), gp, dim3(256), 0, s, a, b);
  if (d.any_global) hipLaunchKernelGGL((k_br_segments<B, u64>), gp, dim3(256), 0, s, a, b);
  AIWC_MARK(pm, "k_br_segments", s);
  u64 nb = d.max_br_blocks < 256 ? d.max_br_blocks : 256;
  const dim3 gw((unsigned)nb, d.n);
  if (d.any_local) {
    hipLaunchKernelGGL((k_br_windows_sort<B>), gw, dim3(WIN_BLOCK), 0, s, a, b);
    if (d.any_hot) {
      hipLaunchKernelGGL((k_br_windows_hot<B>), dim3(256, d.n), dim3(WIN_BLOCK), 0, s, a, b);
      hipLaunchKernelGGL((k_br_hot_terms<B>), dim3(256, d.n), dim3(256), 0, s, a, b);
    }
    hipLaunchKernelGGL((k_br_windows<B, false, true>), gw, dim3(WIN_BLOCK), 0, s, a, b);
  }
  if (d.any_global)
    hipLaunchKernelGGL((k_br_windows<B, true, false>), gw, dim3(WIN_BLOCK), 0, s, a, b);
  AIWC_MARK(pm, "k_br_windows", s);
  if (d.any_pattern) {
    u64 pb = (d.max_pattern_bins + 255) / 256;
    if (pb > 1024) pb = 1024;
    hipLaunchKernelGGL(k_br_pattern<B>, dim3((unsigned)pb, d.n), dim3(256), 0, s, a, b);
    AIWC_MARK(pm, "k_br_pattern", s);
  }
}

hipError_t launch_branch(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm) {
  if (!d.any_branch) return hipSuccess;
  if (d.batch) branch_launches<true>(a, d, s, pm);
  else branch_launches<false>(a, d, s, pm);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
