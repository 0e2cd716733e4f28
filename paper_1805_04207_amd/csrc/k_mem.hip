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
//   k_mem_hist      : per-block partition histogram of the address stream
//                     (and the reads / writes of each space)
//   k_mem_colscan   : exclusive scan over blocks, per partition
//   k_mem_binscan   : exclusive scan over partitions; the bucket kernel's
//                     queue (longest partitions first), the hot partitions,
//                     and the cursors of the two-level scatter
//   k_mem_scatter   : one 64-bit record per access into its partition
//                     (below 2^12 partitions), or
//   k_mem_scatter_a : tiles sorted in LDS by coarse bucket (256 partitions)
//   k_mem_scatter_b : and within each bucket by partition, written in runs
//   k_mem_hot_pick  : candidate pages of each hot partition (2^18 records
//                     and more) from a sample of its records
//   k_mem_hot_count : the candidates' offsets counted in parallel pieces into
//                     per-page tables, the other records compacted
//   k_mem_bucket    : per partition (persistent blocks, a queue): an LDS table
//                     of its pages, the records regrouped page by page in
//                     LDS, and every level's nodes (the records of a page
//                     whose offsets agree on bits k..9) from wavefront
//                     ballots (small pages) or 1024 LDS offset counters
//                     (larger pages); each node adds 1 to distinct_k and
//                     c * log2(N / c) to level k (fixed point, integer sums,
//                     so the result is order independent), level 0 also its
//                     count spectrum.  A partition whose pages overflow the
//                     table is split by further hash bits and redone (exact).
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
// two-level scatter: coarse buckets of 256 partitions, then the partitions
constexpr u32 FINE_BITS = 8;
constexpr int SC_BLOCK = 1024;
constexpr u32 SC_T = 8192;                 // records per tile (8 per thread)
static_assert(SC_T <= (1u << 24), "a rank travels above an 8-bit digit in 32 bits");
constexpr u32 SPEC_SLOTS = 64;    // per-space LDS cache of the level-0 spectrum
constexpr u64 EMPTY = ~0ull;

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
  extern __shared__ u32 h[];   // [P]
  __shared__ u64 sp_cnt[4];  // reads g, writes g, reads l, writes l
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || blockIdx.x >= A.n_hist_blocks) return;
  const u32 P = 1u << A.pbits;
  for (u32 i = threadIdx.x; i < P; i += MEM_BLOCK) h[i] = 0;
  if (threadIdx.x < 4) sp_cnt[threadIdx.x] = 0;
  __syncthreads();
  const u64 c0 = (u64)blockIdx.x * A.hist_chunk;
  const u64 c1 = (c0 + A.hist_chunk < A.n_mem) ? c0 + A.hist_chunk : A.n_mem;
  u32 cnt[4] = {0, 0, 0, 0};
  for (u64 i = c0 + 8ull * threadIdx.x; i < c1; i += 8ull * MEM_BLOCK) {
    u64 a[8];
    uint2 kk2;
    int n = 8;
    if (VEC && i + 8 <= c1) {
      const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(A.addr + i);
#pragma unroll
      for (int q = 0; q < 4; ++q) { const ulonglong2 x = pa[q]; a[2 * q] = x.x; a[2 * q + 1] = x.y; }
      kk2 = *reinterpret_cast<const uint2 *>(A.mem_kind + i);
    } else {
      n = (int)((c1 - i) < 8 ? (c1 - i) : 8);
      kk2 = make_uint2(0, 0);
      for (int j = 0; j < 8; ++j) {
        a[j] = j < n ? A.addr[i + j] : 0;
        const u32 kb = j < n ? A.mem_kind[i + j] : 0;
        if (j < 4) kk2.x |= kb << (8 * j); else kk2.y |= kb << (8 * (j - 4));
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < n) {
        const uint8_t k = (uint8_t)((j < 4 ? kk2.x : kk2.y) >> (8 * (j & 3)));
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

// ------------------------------------------------------------- hot pages
// A partition of AIWC_HOT_PART records or more usually holds pages that take
// most of them (a work-group's local tile, a histogram's bins), and one
// bucket block would stream it alone.  Such a partition (up to
// AIWC_HOT_PMAX of them) gets up to AIWC_HOT_CAND candidate pages: the pages
// with HOT_CAND_MIN or more of its first HOT_SAMPLE records.  Every record
// of a candidate page is counted, by many blocks in parallel, into the
// page's table (1024 byte-offset counters, then 32 read- and 32
// write-bitmap words); the partition's other records are compacted into
// part_cmp and reduced by k_mem_bucket as usual, which then evaluates each
// candidate from its table exactly as a heavy page.  Which pages are
// candidates only decides how the work is split: every page takes one path
// whole.
//   state (u32 words): [0] hot partitions, [1] pieces, [2] piece queue,
//   then HotPart[AIWC_HOT_PMAX], the candidates' page keys (u64), and from
//   word 2048 the tables.
constexpr u32 HOT_SAMPLE = 16384, HOT_CAND_MIN = 1024, HOT_PIECE = 65536;
constexpr u32 HOT_TAB = 1024 + 64;
constexpr u32 HOT_SLOTS = 4096;                   // page table of the sample
struct HotPart { u32 p, first_piece, kept, ncand, pad[4]; };
static_assert(4 + 8 * AIWC_HOT_PMAX + 2 * AIWC_HOT_PMAX * AIWC_HOT_CAND <= 2048,
              "hot-partition headers fit below the tables");
static_assert(AIWC_HOT_PMAX <= AIWC_WAVE, "a wavefront looks up the hot partitions, one per lane");
__device__ __forceinline__ HotPart *hot_parts(u32 *h) { return reinterpret_cast<HotPart *>(h + 4); }
__device__ __forceinline__ u64 *hot_keys(u32 *h) {
  return reinterpret_cast<u64 *>(h + 4 + 8 * AIWC_HOT_PMAX);
}
__device__ __forceinline__ u32 *hot_tab(u32 *h, u32 hp, u32 c) {
  return h + 2048 + (hp * AIWC_HOT_CAND + c) * HOT_TAB;
}
__device__ __forceinline__ u32 hot_pieces(u32 n) { return (n + HOT_PIECE - 1) / HOT_PIECE; }

// Per partition: exclusive prefix over the histogram blocks (in place);
// the partition total goes to part_off[b].
template <bool BATCH>
__global__ void k_mem_colscan(TraceArgs A0, const TraceArgs *batch) {
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  const u32 P = 1u << A.pbits;
  const u32 b = blockIdx.x * blockDim.x + threadIdx.x;
  if (A.n_mem == 0 || b >= P) return;
  // sixteen loads in flight, then their prefix written back
  u32 s = 0;
  const u32 nb = A.n_hist_blocks;
  for (u32 w0 = 0; w0 < nb; w0 += 16) {
    u32 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = w0 + j < nb ? A.part_hist[(u64)(w0 + j) * P + b] : 0u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (w0 + j >= nb) break;
      A.part_hist[(u64)(w0 + j) * P + b] = s;
      s += v[j];
    }
  }
  A.part_off[b] = s;
}

// Exclusive scan of the partition totals (one block); part_off[P] = n_mem.
template <bool BATCH>
__global__ void __launch_bounds__(1024) k_mem_binscan(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u32 wsum[16];
  __shared__ u32 carry;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
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
  // the bucket kernel's queue order: partitions of more than STAGE records
  // (several rounds, or heavy pages whose records are read once per page)
  // first, so that the longest ones do not start last; the order of the
  // rest is free (results do not depend on it)
  // The hot partitions (AIWC_HOT_PART records or more, the first
  // AIWC_HOT_PMAX found) and where their pieces start in the piece queue.
  __shared__ u32 nbig, nsmall, nhot, hot[AIWC_HOT_PMAX];
  if (threadIdx.x == 0) { nbig = 0; nsmall = 0; nhot = 0; }
  __syncthreads();
  // list appends: one LDS atomic per wavefront and list, ranks from ballots
  const int lane = lane_id();
  const u64 lt = (1ull << lane) - 1ull;
  auto append = [&](u32 &count, bool mine) {
    const u64 B = __ballot(mine);
    u32 base = 0;
    if (lane == 0 && B) base = atomicAdd(&count, (u32)__builtin_popcountll(B));
    return (u32)__builtin_amdgcn_readfirstlane((int)base) + (u32)__builtin_popcountll(B & lt);
  };
  for (u32 i0 = 0; i0 < P; i0 += 1024) {
    const u32 i = i0 + threadIdx.x;
    const u32 sz = i < P ? A.part_off[i + 1] - A.part_off[i] : 0u;
    const bool big = i < P && sz > AIWC_STAGE_CAP;
    const u32 kb = append(nbig, big);
    if (big) A.part_order[kb] = i;
    const bool isHot = i < P && A.mem_hot && sz >= AIWC_HOT_PART;
    const u32 kh = append(nhot, isHot);
    if (isHot && kh < AIWC_HOT_PMAX) hot[kh] = i;
  }
  __syncthreads();
  if (A.mem_hot && threadIdx.x == 0) {
    u32 *H = A.mem_hot;
    const u32 nh = nhot < AIWC_HOT_PMAX ? nhot : AIWC_HOT_PMAX;
    u32 pieces = 0;
    for (u32 h = 0; h < nh; ++h) {
      HotPart &hp = hot_parts(H)[h];
      hp.p = hot[h];
      hp.first_piece = pieces;
      hp.kept = 0;
      hp.ncand = 0;
      pieces += hot_pieces(A.part_off[hot[h] + 1] - A.part_off[hot[h]]);
    }
    H[0] = nh;
    H[1] = pieces;
    H[2] = 0;
  }
  const u32 nb = nbig;
  for (u32 i0 = 0; i0 < P; i0 += 1024) {
    const u32 i = i0 + threadIdx.x;
    const bool small = i < P && A.part_off[i + 1] - A.part_off[i] <= AIWC_STAGE_CAP;
    const u32 ks = append(nsmall, small);
    if (small) A.part_order[nb + ks] = i;
  }
  if (!A.part_tmp) return;
  // two-level scatter: fine cursors (one per partition), coarse cursors
  // (one per 256 partitions), and where each coarse bucket's tiles start
  const u32 NC = P >> FINE_BITS;
  u32 *fcur = A.part_cur, *ccur = A.part_cur + P, *tst = A.part_cur + P + NC;
  for (u32 i = threadIdx.x; i < P; i += 1024) fcur[i] = A.part_off[i];
  for (u32 c = threadIdx.x; c < NC; c += 1024) ccur[c] = A.part_off[c << FINE_BITS];
  if (threadIdx.x == 0) {
    u32 t = 0;
    for (u32 c = 0; c < NC; ++c) {
      tst[c] = t;
      const u32 sz = A.part_off[(c + 1) << FINE_BITS] - A.part_off[c << FINE_BITS];
      t += (sz + SC_T - 1) / SC_T;
    }
    tst[NC] = t;
  }
}

// ------------------------------------------------------ two-level scatter
// With 2^15 partitions one pass cannot write coalesced runs: a block's
// records of one partition are a few 8-byte stores among 32768 open
// destinations.  From 2^12 partitions on the records go through two
// passes instead.  Each pass takes tiles of SC_T records, counts them per
// digit in LDS, reserves every digit's range of the destination with one
// atomic on its cursor, sorts the tile by digit in LDS and writes it out in
// runs: pass A to 2^(pbits-8) coarse buckets (the record carries its fine
// digit in bits 56..63), pass B within each coarse bucket to its 256
// partitions.  Record order inside a partition is free.
struct TileShared {
  u64 stage[SC_T];
  uint8_t dig[SC_T];
  u32 cnt[256], start[256], gbase[256];
  u32 tst[257];
};

// Exclusive prefix of cnt[0..256) into start[] (one wavefront, 4 per lane).
__device__ __forceinline__ void tile_scan(TileShared &S) {
  const int l = lane_id();
  const u32 a = S.cnt[4 * l], b = S.cnt[4 * l + 1], c = S.cnt[4 * l + 2], d = S.cnt[4 * l + 3];
  u32 x = a + b + c + d;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u32 y = __shfl_up(x, o, 64);
    if (l >= o) x += y;
  }
  const u32 e = x - (a + b + c + d);
  S.start[4 * l] = e;
  S.start[4 * l + 1] = e + a;
  S.start[4 * l + 2] = e + a + b;
  S.start[4 * l + 3] = e + a + b + c;
}

// Stage the tile's records by digit and write them out in runs: dst[gbase[d]
// + rank among the tile's records of digit d].  Every thread calls it with
// its own records (nv of them), dk = digit | rank << 8.  RANKED: the rank is
// the value the record's counting atomic returned, so no second atomic is
// needed; otherwise dk holds the digit alone and the ranks come from atomics
// after the scan.  TOP: the digit is the record's top byte, cleared on the
// way out (no digit array in LDS).
template <int R, bool TOP, bool RANKED>
__device__ __forceinline__ void tile_write(TileShared &S, const u64 (&rec)[R], const u32 (&dk)[R],
                                           int nv, u32 n, u64 *dst, u32 ndig, u32 *cursor) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) tile_scan(S);
  __syncthreads();
  if (tid < (int)ndig) {
    const u32 c = S.cnt[tid];
    if (c) S.gbase[tid] = atomicAdd(&cursor[tid], c);
    if (!RANKED) S.cnt[tid] = S.start[tid];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j < nv) {
      const u32 d = dk[j] & 255u;
      const u32 r = RANKED ? S.start[d] + (dk[j] >> 8) : atomicAdd(&S.cnt[d], 1u);
      S.stage[r] = rec[j];
      if (!TOP) S.dig[r] = (uint8_t)d;
    }
  }
  __syncthreads();
  for (u32 i = tid; i < n; i += SC_BLOCK) {
    const u64 v = S.stage[i];
    const u32 d = TOP ? (u32)(v >> 56) : S.dig[i];
    dst[S.gbase[d] + (i - S.start[d])] = TOP ? v & ((1ull << 56) - 1ull) : v;
  }
  __syncthreads();
}

template <bool VEC, bool BATCH>
__global__ void __launch_bounds__(SC_BLOCK, 8) k_mem_scatter_a(TraceArgs A0, const TraceArgs *batch) {
  __shared__ TileShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || !A.part_tmp) return;
  const int tid = threadIdx.x;
  const u32 P = 1u << A.pbits, NC = P >> FINE_BITS;
  u32 *ccur = A.part_cur + P;
  const u64 ntiles = (A.n_mem + SC_T - 1) / SC_T;
  // the blocks of one XCD take one contiguous eighth of the tiles (as in
  // pass B)
  const u32 X = (gridDim.x % 8u == 0) ? 8u : 1u;
  const u32 xcd = blockIdx.x % X, per = gridDim.x / X;
  const u64 t_lo = ntiles * xcd / X, t_hi = ntiles * (xcd + 1) / X;
  for (u64 t = t_lo + blockIdx.x / X; t < t_hi; t += per) {
    const u64 t0 = t * SC_T;
    const u32 n = (u32)((A.n_mem - t0) < SC_T ? (A.n_mem - t0) : SC_T);
    if (tid < 256) S.cnt[tid] = 0;
    __syncthreads();
    const u64 i = t0 + 8ull * tid;
    u64 a[8];
    uint2 kk2 = make_uint2(0, 0);
    int nv = 0;
    if (i < A.n_mem) {
      if (VEC && i + 8 <= A.n_mem) {
        const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(A.addr + i);
#pragma unroll
        for (int q = 0; q < 4; ++q) { const ulonglong2 x = pa[q]; a[2 * q] = x.x; a[2 * q + 1] = x.y; }
        kk2 = *reinterpret_cast<const uint2 *>(A.mem_kind + i);
        nv = 8;
      } else {
        nv = (int)((A.n_mem - i) < 8 ? (A.n_mem - i) : 8);
        for (int j = 0; j < 8; ++j) {
          a[j] = j < nv ? A.addr[i + j] : 0;
          const u32 kb = j < nv ? A.mem_kind[i + j] : 0;
          if (j < 4) kk2.x |= kb << (8 * j); else kk2.y |= kb << (8 * (j - 4));
        }
      }
    }
    u64 rec[8];
    u32 dk[8];   // the coarse digit (ranked after the scan: the ranks'
                 // registers would spill here, and ranking early gained nothing)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      rec[j] = 0;
      dk[j] = 0;
      if (j < nv) {
        u32 bin;
        const uint8_t k = (uint8_t)((j < 4 ? kk2.x : kk2.y) >> (8 * (j & 3)));
        rec[j] = make_record(a[j], k, A.pbits, bin) | ((u64)(bin & 255u) << 56);
        dk[j] = bin >> FINE_BITS;
        atomicAdd(&S.cnt[dk[j]], 1u);
      }
    }
    tile_write<8, false, false>(S, rec, dk, nv, n, A.part_tmp, NC, ccur);
  }
}

template <bool BATCH>
__global__ void __launch_bounds__(SC_BLOCK, 8) k_mem_scatter_b(TraceArgs A0, const TraceArgs *batch) {
  __shared__ TileShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || !A.part_tmp) return;
  const int tid = threadIdx.x;
  const u32 P = 1u << A.pbits, NC = P >> FINE_BITS;
  const u32 *tst_g = A.part_cur + P + NC;
  for (u32 c = tid; c <= NC; c += SC_BLOCK) S.tst[c] = tst_g[c];
  __syncthreads();
  const u32 ntiles = S.tst[NC];
  // blocks are dealt to the 8 XCDs in turn; the blocks of one XCD take one
  // contiguous eighth of the tiles, so that a coarse bucket's cursors and
  // its partitions' write runs stay with one XCD's L2
  const u32 X = (gridDim.x % 8u == 0) ? 8u : 1u;
  const u32 xcd = blockIdx.x % X, per = gridDim.x / X;
  const u32 t_lo = (u32)((u64)ntiles * xcd / X), t_hi = (u32)((u64)ntiles * (xcd + 1) / X);
  for (u32 t = t_lo + blockIdx.x / X; t < t_hi; t += per) {
    // the coarse bucket of tile t: the last c with tst[c] <= t
    u32 lo = 0, hi = NC;
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (S.tst[mid] <= t) lo = mid; else hi = mid;
    }
    const u32 c = lo;
    const u64 b0 = A.part_off[c << FINE_BITS], b1 = A.part_off[(c + 1) << FINE_BITS];
    const u64 t0 = b0 + (u64)(t - S.tst[c]) * SC_T;
    const u32 n = (u32)((b1 - t0) < SC_T ? (b1 - t0) : SC_T);
    if (tid < 256) S.cnt[tid] = 0;
    __syncthreads();
    u64 rec[8];
    u32 dk[8];   // fine digit | rank << 8
    int nv = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      // record j of this thread: t0 + j * SC_BLOCK + tid (coalesced)
      const u32 k = (u32)j * SC_BLOCK + (u32)tid;
      rec[j] = 0;
      dk[j] = 0;
      if (k < n) {
        const u64 r = A.part_tmp[t0 + k];
        const u32 d = (u32)(r >> 56);
        rec[j] = r;   // the fine digit stays in the top byte until written out
        dk[j] = d | (atomicAdd(&S.cnt[d], 1u) << 8);
        nv = j + 1;
      }
    }
    tile_write<8, true, true>(S, rec, dk, nv, n, A.part_rec, 256u, A.part_cur + (c << FINE_BITS));
  }
}

// -------------------------------------------------------------- scatter
template <bool VEC, bool BATCH>
__global__ void __launch_bounds__(MEM_BLOCK) k_mem_scatter(TraceArgs A0, const TraceArgs *batch) {
  extern __shared__ u32 cur[];   // [P]
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0 || blockIdx.x >= A.n_hist_blocks || A.part_tmp) return;
  const u32 P = 1u << A.pbits;
  const u32 *row = A.part_hist + (u64)blockIdx.x * P;
  for (u32 i = threadIdx.x; i < P; i += MEM_BLOCK) cur[i] = A.part_off[i] + row[i];
  __syncthreads();
  const u64 c0 = (u64)blockIdx.x * A.hist_chunk;
  const u64 c1 = (c0 + A.hist_chunk < A.n_mem) ? c0 + A.hist_chunk : A.n_mem;
  for (u64 i = c0 + 8ull * threadIdx.x; i < c1; i += 8ull * MEM_BLOCK) {
    u64 a[8];
    uint2 kk2;
    int n = 8;
    if (VEC && i + 8 <= c1) {
      const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(A.addr + i);
#pragma unroll
      for (int q = 0; q < 4; ++q) { const ulonglong2 x = pa[q]; a[2 * q] = x.x; a[2 * q + 1] = x.y; }
      kk2 = *reinterpret_cast<const uint2 *>(A.mem_kind + i);
    } else {
      n = (int)((c1 - i) < 8 ? (c1 - i) : 8);
      kk2 = make_uint2(0, 0);
      for (int j = 0; j < 8; ++j) {
        a[j] = j < n ? A.addr[i + j] : 0;
        const u32 kb = j < n ? A.mem_kind[i + j] : 0;
        if (j < 4) kk2.x |= kb << (8 * j); else kk2.y |= kb << (8 * (j - 4));
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < n) {
        u32 bin;
        const u64 rec = make_record(a[j], (uint8_t)((j < 4 ? kk2.x : kk2.y) >> (8 * (j & 3))),
                                    A.pbits, bin);
        const u32 pos = atomicAdd(&cur[bin], 1u);
        A.part_rec[pos] = rec;
      }
    }
  }
}

// ------------------------------------------------- partition groups (streams)
// A stream whose memory events exceed the device budget is reduced one
// group of partitions at a time (partitions hold disjoint pages, so the
// groups' sums are the whole's).  k_mem_count: per-partition record counts
// and the per-space read / write totals of one chunk of the memory stream,
// added to the stream's totals.  k_mem_scatter_range: the records of one
// chunk whose partition lies in [p0, p1) go to their partition's range of
// the group's record array (cursor[p], advanced by one reservation per
// block and partition).
constexpr int GRP_BLOCK = 1024;

__global__ void __launch_bounds__(GRP_BLOCK) k_mem_count(TraceArgs A, u32 *count) {
  extern __shared__ u32 h[];   // [P]
  __shared__ u64 sp_cnt[4];
  const u32 P = 1u << A.pbits;
  for (u32 i = threadIdx.x; i < P; i += GRP_BLOCK) h[i] = 0;
  if (threadIdx.x < 4) sp_cnt[threadIdx.x] = 0;
  __syncthreads();
  u32 cnt[4] = {0, 0, 0, 0};
  for (u64 i = (u64)blockIdx.x * GRP_BLOCK + threadIdx.x; i < A.n_mem;
       i += (u64)gridDim.x * GRP_BLOCK) {
    const uint8_t k = A.mem_kind[i];
    u32 bin;
    make_record(A.addr[i], k, A.pbits, bin);
    atomicAdd(&h[bin], 1u);
    cnt[((k >> 1) & 1u) * 2 + (k & 1u)] += 1;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const u64 v = wave_sum_u64(cnt[j]);
    if (lane_id() == 0 && v) atomicAdd(&sp_cnt[j], v);
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < P; i += GRP_BLOCK)
    if (h[i]) atomicAdd(&count[i], h[i]);
  if (threadIdx.x < 4 && sp_cnt[threadIdx.x]) {
    u64 *dst = (threadIdx.x & 1) ? &A.acc->sp_writes[threadIdx.x >> 1]
                                 : &A.acc->sp_reads[threadIdx.x >> 1];
    atomicAdd(dst, sp_cnt[threadIdx.x]);
  }
}

__global__ void __launch_bounds__(GRP_BLOCK) k_mem_scatter_range(TraceArgs A, u32 p0, u32 p1,
                                                                 u32 *cursor, u64 *rec) {
  extern __shared__ u32 h[];   // [p1 - p0]: counts, then this block's cursors
  const u32 np = p1 - p0;
  for (u32 i = threadIdx.x; i < np; i += GRP_BLOCK) h[i] = 0;
  __syncthreads();
  // the block's slice of the chunk
  const u64 per = (A.n_mem + gridDim.x - 1) / gridDim.x;
  const u64 c0 = (u64)blockIdx.x * per;
  const u64 c1 = c0 + per < A.n_mem ? c0 + per : A.n_mem;
  for (u64 i = c0 + threadIdx.x; i < c1; i += GRP_BLOCK) {
    u32 bin;
    make_record(A.addr[i], A.mem_kind[i], A.pbits, bin);
    if (bin >= p0 && bin < p1) atomicAdd(&h[bin - p0], 1u);
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < np; i += GRP_BLOCK)
    if (h[i]) h[i] = atomicAdd(&cursor[p0 + i], h[i]);
  __syncthreads();
  for (u64 i = c0 + threadIdx.x; i < c1; i += GRP_BLOCK) {
    u32 bin;
    const u64 r = make_record(A.addr[i], A.mem_kind[i], A.pbits, bin);
    if (bin >= p0 && bin < p1) rec[atomicAdd(&h[bin - p0], 1u)] = r;
  }
}

// Candidate pages of one hot partition (one block each) from the pages of
// its first HOT_SAMPLE records; their tables start at zero.
template <bool BATCH>
__global__ void __launch_bounds__(1024) k_mem_hot_pick(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u64 key[HOT_SLOTS];
  __shared__ u32 cnt[HOT_SLOTS];
  __shared__ u32 nc;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!A.mem_hot || A.n_mem == 0) return;
  u32 *H = A.mem_hot;
  const u32 h = blockIdx.x;
  if (h >= H[0]) return;
  HotPart &hp = hot_parts(H)[h];
  const u64 base = A.part_off[hp.p];
  const u32 size = A.part_off[hp.p + 1] - (u32)base;
  for (u32 i = threadIdx.x; i < HOT_SLOTS; i += 1024) { key[i] = EMPTY; cnt[i] = 0; }
  if (threadIdx.x == 0) nc = 0;
  __syncthreads();
  const u32 ns = size < HOT_SAMPLE ? size : HOT_SAMPLE;
  const int lane = lane_id();
  for (u32 i0 = threadIdx.x - lane; i0 < ns; i0 += 1024) {
    const u32 i = i0 + (u32)lane;
    const bool valid = i < ns;
    const u64 pk = valid ? A.part_rec[base + i] >> 11 : EMPTY;
    // the lanes on lane 0's page add once (a hot page takes most lanes)
    const u64 pk0 = ((u64)__builtin_amdgcn_readfirstlane((int)(u32)(pk >> 32)) << 32) |
                    (u32)__builtin_amdgcn_readfirstlane((int)(u32)pk);
    const u64 B = __ballot(valid && pk == pk0);
    u32 add = 0;
    if (valid && pk == pk0) add = lane == 0 ? (u32)__builtin_popcountll(B) : 0u;
    else if (valid) add = 1;
    if (add) {
      u32 slot = hash_slot(pk, HOT_SLOTS);
      for (u32 probe = 0; probe < HOT_SLOTS; ++probe) {   // a full table: the page is skipped
        u64 w = key[slot];
        if (w == EMPTY) {
          const u64 old = atomicCAS(&key[slot], EMPTY, pk);
          w = old == EMPTY ? pk : old;
        }
        if (w == pk) { atomicAdd(&cnt[slot], add); break; }
        slot = slot + 1 == HOT_SLOTS ? 0 : slot + 1;
      }
    }
  }
  __syncthreads();
  u64 *keys = hot_keys(H) + (u64)h * AIWC_HOT_CAND;
  for (u32 i = threadIdx.x; i < HOT_SLOTS; i += 1024) {
    if (cnt[i] >= HOT_CAND_MIN) {
      const u32 k = atomicAdd(&nc, 1u);
      if (k < AIWC_HOT_CAND) keys[k] = key[i];
    }
  }
  __syncthreads();
  const u32 ncand = nc < AIWC_HOT_CAND ? nc : AIWC_HOT_CAND;
  if (threadIdx.x == 0) hp.ncand = ncand;
  for (u32 c = 0; c < ncand; ++c) {
    u32 *t = hot_tab(H, h, c);
    for (u32 j = threadIdx.x; j < HOT_TAB; j += 1024) t[j] = 0;
  }
}

// Pieces of the hot partitions: candidate records into LDS tables (added to
// the candidates' tables), the others compacted to part_cmp.  The others are
// staged in LDS and written once per piece; a piece with more of them than
// the staging array holds reads its records a second time to write them.
// The counters sit at hot_slot(offset), which spreads 4-byte-aligned
// offsets over all banks.
constexpr u32 HOT_REST_CAP = 4096;
__device__ __forceinline__ u32 hot_slot(u32 off) { return ((off & 3u) << 8) | (off >> 2); }
template <bool BATCH>
__global__ void __launch_bounds__(1024) k_mem_hot_count(TraceArgs A0, const TraceArgs *batch) {
  __shared__ u32 tc[AIWC_HOT_CAND][1024];
  __shared__ u32 tb[AIWC_HOT_CAND][64];
  __shared__ u64 stage[HOT_REST_CAP];
  __shared__ u32 piece, nstage, wrest[17];
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (!A.mem_hot || A.n_mem == 0) return;
  u32 *H = A.mem_hot;
  const u32 nh = H[0], total = H[1];
  if (nh == 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / AIWC_WAVE;
  const u64 below = (1ull << lane) - 1ull;
  while (true) {
    if (tid == 0) { piece = atomicAdd(&H[2], 1u); nstage = 0; }
    __syncthreads();
    const u32 pc = piece;
    if (pc >= total) break;
    u32 h = 0;
    while (h + 1 < nh && pc >= hot_parts(H)[h + 1].first_piece) ++h;
    HotPart &hp = hot_parts(H)[h];
    const u64 base = A.part_off[hp.p];
    const u32 size = A.part_off[hp.p + 1] - (u32)base;
    const u32 r0 = (pc - hp.first_piece) * HOT_PIECE;
    const u32 r1 = size - r0 < HOT_PIECE ? size : r0 + HOT_PIECE;
    const u32 ncand = hp.ncand;
    u64 ck[AIWC_HOT_CAND];
#pragma unroll
    for (u32 c = 0; c < AIWC_HOT_CAND; ++c) ck[c] = c < ncand ? hot_keys(H)[h * AIWC_HOT_CAND + c] : EMPTY;
    for (u32 i = tid; i < AIWC_HOT_CAND * 1024; i += 1024) (&tc[0][0])[i] = 0;
    for (u32 i = tid; i < AIWC_HOT_CAND * 64; i += 1024) (&tb[0][0])[i] = 0;
    __syncthreads();
    // a wave takes a contiguous run of the piece: candidates counted, the
    // other records counted per wave and staged
    const u32 per = ((r1 - r0 + 1023u) / 1024u) * AIWC_WAVE;
    const u32 w0 = r0 + (u32)wave * per, w1 = w0 + per < r1 ? w0 + per : r1;
    auto cand = [&](u64 rec) {
      const u64 pk = rec >> 11;
      u32 c = AIWC_HOT_CAND;
#pragma unroll
      for (u32 q = 0; q < AIWC_HOT_CAND; ++q)
        if (pk == ck[q]) c = q;
      return c;
    };
    u32 nrest = 0;
    for (u32 i0 = w0; i0 < w1; i0 += AIWC_WAVE) {
      const u32 i = i0 + (u32)lane;
      const bool valid = i < w1;
      const u64 rec = valid ? A.part_rec[base + i] : EMPTY;
      const u32 c = valid ? cand(rec) : 0u;
      if (valid && c < AIWC_HOT_CAND) {
        const u32 off = (u32)(rec >> 1) & 1023u;
        atomicAdd(&tc[c][hot_slot(off)], 1u);
        u32 *w = &tb[c][((u32)rec & 1u) * 32u + (off >> 5)];
        const u32 bit = 1u << (off & 31u);
        if (!(*w & bit)) atomicOr(w, bit);   // a set bit stays set
      }
      const bool rest = valid && c == AIWC_HOT_CAND;
      const u64 W = __ballot(rest);
      if (W) {
        const u32 k = (u32)__builtin_popcountll(W);
        u32 at = 0;
        if (lane == 0) at = atomicAdd(&nstage, k);
        at = (u32)__shfl((int)at, 0, AIWC_WAVE) + (u32)__builtin_popcountll(W & below);
        if (rest && at < HOT_REST_CAP) stage[at] = rec;
        nrest += k;
      }
    }
    if (lane == 0) wrest[wave] = nrest;
    __syncthreads();
    const u32 ns = nstage;
    if (tid == 0) {
      u32 run = 0;
      for (int w = 0; w < 16; ++w) { const u32 x = wrest[w]; wrest[w] = run; run += x; }
      wrest[16] = run ? atomicAdd(&hp.kept, run) : 0u;
    }
    __syncthreads();
    if (ns <= HOT_REST_CAP) {
      u64 *dst = A.part_cmp + base + wrest[16];
      for (u32 j = tid; j < ns; j += 1024) dst[j] = stage[j];
    } else {
      // ... too many to stage: one more read, each wave writing its own
      u32 at = wrest[16] + wrest[wave];
      for (u32 i0 = w0; i0 < w1; i0 += AIWC_WAVE) {
        const u32 i = i0 + (u32)lane;
        const bool valid = i < w1;
        const u64 rec = valid ? A.part_rec[base + i] : EMPTY;
        const bool rest = valid && cand(rec) == AIWC_HOT_CAND;
        const u64 W = __ballot(rest);
        if (rest) A.part_cmp[base + at + (u32)__builtin_popcountll(W & below)] = rec;
        at += (u32)__builtin_popcountll(W);
      }
    }
    for (u32 c = 0; c < ncand; ++c) {
      u32 *t = hot_tab(H, h, c);
      for (u32 j = tid; j < 1024; j += 1024) {
        const u32 v = tc[c][hot_slot(j)];
        if (v) atomicAdd(&t[j], v);
      }
      if (tid < 64 && tb[c][tid]) atomicOr(&t[1024 + tid], tb[c][tid]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- bucket
// One block per partition at a time (persistent, partitions from a queue).
//  1. page pass   : an LDS table of the partition's pages (record >> 11, which
//                   includes the space bit) counts the records of each page.
//                   More than PT_CAP pages: the partition is split into rounds
//                   by page-hash bits (never by record, so every a >> k bucket
//                   stays whole) and redone.
//  2. regroup     : records are regrouped page by page into an LDS staging
//                   array (u32: compact page index, byte offset, write flag),
//                   small pages (<= SMALL records) of space 0, then of space 1,
//                   then every other page up to HEAVY records.  A round whose
//                   staged records exceed STAGE_CAP is split like a page
//                   overflow.
//  3. levels      : the node of level k holding a record is the set of records
//                   of its page whose byte offsets agree on bits k..9.
//       pages <= MEDIUM records, one record per lane: that set is the page's
//                   lane mask AND-ed with one ballot per offset bit; its lowest
//                   lane owns the node and adds its count.  Small pages are
//                   packed: a wavefront takes the pages that start in a window
//                   of SMALL staging positions (they end within 2 * SMALL).
//       larger pages: the wavefront counts the page's byte offsets in 1024
//                   dense LDS counters, then reduces them level by level.
//       pages > HEAVY records are not staged: the whole block counts them
//                   straight from the partition's records.
//     Each node adds 1 to distinct_k and its entropy term c*log2(N/c) (fixed
//     point, truncated to 2^-40, integer sums) to level k; nodes with c = 1
//     are only counted and multiplied by log2(N) when the accumulators are
//     flushed.  Level-0 counts below SPEC_LDS go to an LDS spectrum histogram;
//     dense-tree nodes with c >= 256 are listed and added by the block after
//     the round.
constexpr u32 PT_SLOTS = 2048;
constexpr u32 PT_CAP = 1536;
constexpr int BK_BLOCK = 512;                    // 8 waves: 256 VGPRs per lane
constexpr int BK_WAVES = BK_BLOCK / AIWC_WAVE;    // 8
constexpr u32 HEAVY = 8192;
constexpr u32 SMALL = 32;
constexpr u32 MEDIUM = 64;
constexpr int UNROLL = 8;                         // records in flight per thread
constexpr u32 SPEC_LDS = 256;
constexpr u32 STAGE_CAP = AIWC_STAGE_CAP;         // staged records per round
constexpr u32 TAG_POS = (1u << 21) - 1u;          // position field of a record tag
constexpr u32 HEAVY_TAG = 1u << 31;               // big-list entry of an unstaged page
// Dense-tree nodes of count >= 256 found by the wavefronts in one round, kept
// for the block: at most 11 levels * STAGE_CAP / 256 of them.
constexpr u32 BLIST_CAP = AIWC_NSKIP * STAGE_CAP / 256;
static_assert(STAGE_CAP < 0xFFFFu, "staging positions travel in 16 bits");
static_assert(PT_SLOTS <= 2048, "a slot travels in the 11 high bits of a tag and of a staged record");
static_assert(STAGE_CAP <= (1u << 15) && HEAVY < (1u << 15),
              "start | size << 15 (table word) and start | size << 16 (big list) fit 32 bits");

struct BucketShared {
  u64 pkey[PT_SLOTS];              // page key, EMPTY if free
  u32 pcnt[PT_SLOTS];              // records of the page
  uint16_t pslot[PT_CAP];          // slot of compact index
  uint16_t psz[PT_CAP];            // records of compact index (saturated at 65535)
  u32 pend[PT_CAP];                // staging cursor, then end, of compact index
  u32 dense[BK_WAVES][1024];       // per-wave byte-offset counters
  u32 rbits[32], wbits[32];        // read / write bitmaps of a heavy page
  u32 hotp[AIWC_HOT_PMAX];         // the hot partitions' indices
  u64 term[2][256];                // c*log2(N_s/c) for c < 256, 2^-40 units
  u32 spec[2][SPEC_LDS];           // level-0 nodes of count c, 2 <= c < SPEC_LDS
  u64 spf[2][SPEC_SLOTS], spm[2][SPEC_SLOTS];
  u64 dist[2][AIWC_NSKIP];
  u64 el[2][AIWC_NSKIP][3];        // entropy, 2^-40 units: el0 + el1 * 2^32 + el2 * 2^64
  u64 ur[2], uw[2];
  u64 redos;
  // pages > SMALL, space 0 from the front, 1 from the back: compact index
  // (class phase), then start | size << 16 (staged) or HEAVY_TAG | index
  u32 big[PT_CAP];
  u32 ctot[3], ccur[3];
  u32 npages, overflow, work, nbig0, nbig1, nheavy, next_item, sp_top;
  u32 stack_m[32], stack_c[32];
  u32 stage[STAGE_CAP];            // the round's records, page by page
  u32 blist[BLIST_CAP];            // space << 31 | level << 24 | count
  u32 nblist;
};

// c * log2(N / c) in units of 2^-40, truncated (lo, hi words).  Every term
// of every path is rounded this one way, so the sums do not depend on how the
// work was split; with N < 2^32 the sum of a level's terms is at least
// (nodes - 1), so the truncation costs at most 2^-39 relative.
__device__ __forceinline__ void term_fx(u64 c, u64 N, u64 &lo, u64 &hi) {
  if (c == 0 || c >= N) { lo = hi = 0; return; }
  const double d = (double)c * (log1p((double)(N - c) / (double)c) * 1.4426950408889634074);
  u64 l64, h64;
  to_fx64(d, l64, h64);
  lo = (l64 >> 24) | (h64 << 40);
  hi = h64 >> 24;
}

// The sparse level-0 spectrum of one space in global memory: f -> m_f.
struct SpecRef {
  u64 *f, *m;
  u32 cap;
};

__device__ void global_spec_add(SpecRef G, u32 s, u64 f, u64 m) {
  u64 *F = G.f + (u64)s * G.cap;
  u64 *M = G.m + (u64)s * G.cap;
  u32 slot = hash_slot(f, G.cap);
  for (u32 probe = 0; probe < G.cap; ++probe) {
    u64 old = atomicCAS(&F[slot], 0ull, f);
    if (old == 0ull || old == f) { atomicAdd(&M[slot], m); return; }
    slot = (slot + 1 == G.cap) ? 0 : slot + 1;
  }
}

__device__ __noinline__ void spec_cache_add(BucketShared &S, SpecRef G, u32 s, u64 f, u64 m) {
  u32 slot = (u32)((f * 0x9E3779B97F4A7C15ull) >> 56) & (SPEC_SLOTS - 1);
  for (u32 probe = 0; probe < 16; ++probe) {
    u64 old = atomicCAS(&S.spf[s][slot], 0ull, f);
    if (old == 0ull || old == f) { atomicAdd(&S.spm[s][slot], m); return; }
    slot = (slot + 1) & (SPEC_SLOTS - 1);
  }
  global_spec_add(G, s, f, m);
}

// Per-lane accumulators of one address space within one round (flushed when
// the space changes and at the end of the round) for nodes of count < 256.
// A round stages at most STAGE_CAP records, so per level its terms sum below
// STAGE_CAP * 32 < 2^20 (2^60 units) and its nodes number below 2^16 (dn:
// nodes | nodes of count 1 << 16); a heavy page has at most 1024 nodes per
// level, whose small terms sum below 1024 * 256 * 32 = 2^23.  Level-0 nodes
// of count 2..5 (the common small counts) are tallied in two packed words
// (count 2 | count 3 << 16, count 4 | count 5 << 16: at most STAGE_CAP nodes
// per lane and round) instead of LDS atomics on a few hot spectrum bins.
struct LaneAcc {
  u64 lo[AIWC_NSKIP];              // 2^-40 units
  u32 dn[AIWC_NSKIP];
  u32 ur, uw;
  u32 sp23, sp45;
  int space;
};

__device__ __forceinline__ void lacc_clear(LaneAcc &L, int space) {
#pragma unroll
  for (int k = 0; k < AIWC_NSKIP; ++k) { L.lo[k] = 0; L.dn[k] = 0; }
  L.ur = L.uw = 0;
  L.sp23 = L.sp45 = 0;
  L.space = space;
}

__device__ __forceinline__ void add128(u64 &lo, u64 &hi, u64 tl, u64 th) {
  const u64 nl = lo + tl;
  hi += th + (nl < lo ? 1ull : 0ull);
  lo = nl;
}


// Sum over each row of 16 lanes by DPP butterflies (lane ^ 1, lane ^ 2, half
// row mirror, row mirror); every lane of the wavefront must be active.
__device__ __forceinline__ u32 dpp_row_sum(u32 v) {
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
  return v;
}

// Wavefront sum of values below 2^26, as a wave-uniform value.
__device__ __forceinline__ u32 wave_total(u32 v) {
  v = dpp_row_sum(v);
  return (u32)__builtin_amdgcn_readlane((int)v, 0) + (u32)__builtin_amdgcn_readlane((int)v, 16) +
         (u32)__builtin_amdgcn_readlane((int)v, 32) + (u32)__builtin_amdgcn_readlane((int)v, 48);
}

// Inclusive prefix sum over the wavefront by DPP: row shifts by 1, 2, 4, 8
// (sums inside rows of 16), then each row adds the totals of the rows before
// it (row broadcasts of lanes 15 and 31).  Every lane must be active.
__device__ __forceinline__ u32 wave_scan(u32 v) {
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
  v += (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
  return v;
}

// Adds a 2^-40-unit value, given as 32-bit-aligned pieces, to a level's limbs.
__device__ __forceinline__ void limbs_add(u64 *el, u64 l0, u64 l1, u64 l2) {
  if (l0) atomicAdd(&el[0], l0);
  if (l1) atomicAdd(&el[1], l1);
  if (l2) atomicAdd(&el[2], l2);
}

// Called by the whole wavefront (no lane masked off).  Lane sums are below
// 2^63 (terms) and 2^16 (counts); they are cut into 24-bit pieces so that
// every wavefront sum fits 32 bits.
__device__ __forceinline__ void lacc_flush(LaneAcc &L, BucketShared &S) {
  const int s = L.space;
  const int lane = lane_id();
  const u64 t1 = S.term[s][1];
#pragma unroll
  for (int k = 0; k < AIWC_NSKIP; ++k) {
    const u64 lo = L.lo[k];
    const u64 a0 = wave_total((u32)lo & 0xFFFFFFu);
    const u64 a1 = wave_total((u32)(lo >> 24) & 0xFFFFFFu);
    const u64 a2 = wave_total((u32)(lo >> 48));
    const u64 d = wave_total(L.dn[k] & 0xFFFFu), n1 = wave_total(L.dn[k] >> 16);
    // a0 + a1 * 2^24 + a2 * 2^48 + n1 * log2(N)
    const u64 plo = t1 * n1, phi = __umul64hi(t1, n1);
    if (lane == 0) {
      limbs_add(S.el[s][k], a0 + ((a1 & 0xFFull) << 24) + (plo & 0xFFFFFFFFull),
                (a1 >> 8) + (a2 << 16) + (plo >> 32), phi);
      if (d) atomicAdd(&S.dist[s][k], d);
      if (k == 0 && n1) atomicAdd(&S.spec[s][1], (u32)n1);
    }
  }
  const u64 r = wave_total(L.ur), w = wave_total(L.uw);
  const u32 f2 = wave_total(L.sp23 & 0xFFFFu), f3 = wave_total(L.sp23 >> 16);
  const u32 f4 = wave_total(L.sp45 & 0xFFFFu), f5 = wave_total(L.sp45 >> 16);
  if (lane == 0) {
    if (r) atomicAdd(&S.ur[s], r);
    if (w) atomicAdd(&S.uw[s], w);
    if (f2) atomicAdd(&S.spec[s][2], f2);
    if (f3) atomicAdd(&S.spec[s][3], f3);
    if (f4) atomicAdd(&S.spec[s][4], f4);
    if (f5) atomicAdd(&S.spec[s][5], f5);
  }
  lacc_clear(L, s);
}

// A node of level k with count c < 256 (c = 0: no node).  Count-1 nodes are
// only counted; the others add their tabulated term.  Branch free, so that a
// wavefront issues its table loads back to back.
__device__ __forceinline__ void add_small_node(LaneAcc &L, const BucketShared &S, int k, u32 c) {
  L.lo[k] += S.term[L.space][c >= 2 ? c : 0u];   // term[0] = 0
  L.dn[k] += (c != 0 ? 1u : 0u) + (c == 1 ? 0x10000u : 0u);
}

// The level-0 spectrum entry of a node of count c < SPEC_LDS (c < 2: none).
__device__ __forceinline__ void spec_node(LaneAcc &L, BucketShared &S, u32 c) {
  L.sp23 += (c == 2 ? 1u : 0u) + (c == 3 ? 0x10000u : 0u);
  L.sp45 += (c == 4 ? 1u : 0u) + (c == 5 ? 0x10000u : 0u);
  if (c >= 6) atomicAdd(&S.spec[L.space][c], 1u);
}

// A node of count >= 256 (rare): its term goes straight to the block's
// accumulators.
__device__ __forceinline__ void big_node(BucketShared &S, SpecRef G, int s, int k, u32 v,
                                         u64 N) {
  u64 lo, hi;
  term_fx(v, N, lo, hi);
  limbs_add(S.el[s][k], lo & 0xFFFFFFFFull, lo >> 32, hi);
  atomicAdd(&S.dist[s][k], 1ull);
  if (k == 0) spec_cache_add(S, G, (u32)s, v, 1ull);
}

// Dense byte-offset counters are stored swizzled: offset o of group
// g = o >> 4 sits at word o ^ cswz(g), still inside its group of 16.  Bits
// 2..3 of the swizzle, (g >> 1) & 3, make the 16-byte reads of eight
// neighbouring lanes (lane l reads group l) cover all 32 LDS banks; bits 0..1,
// (g >> 3) & 3, spread the counting atomics of 4-byte aligned and 16-byte
// strided offsets over all 32 banks (without them such offsets share 8).
__device__ __forceinline__ u32 cswz(u32 g) { return (((g >> 1) & 3u) << 2) | ((g >> 3) & 3u); }
__device__ __forceinline__ u32 cslot(u32 off) { return off ^ cswz(off >> 4); }

// A dense counter's access count.  Counters of staged pages (at most HEAVY
// records) hold reads | writes << 16 (RW); heavy pages count plainly.
template <bool RW>
__device__ __forceinline__ u32 cval(u32 x) { return RW ? (x & 0xFFFFu) + (x >> 16) : x; }

// The nodes of count >= 256 of the dense tree over cnt[1024] (see
// page_levels).  Few pages have any: plain loops, so that the logarithm is
// emitted twice rather than once per node (and no call spills registers).
template <bool RW>
__device__ __forceinline__ void big_pass(BucketShared &S, SpecRef G, const u32 *cnt, int s,
                                         u64 N) {
  const int lane = lane_id();
  const u32 *my = cnt + 16 * lane;
  const u32 sw = cswz((u32)lane);
#pragma unroll 1
  for (int k = 0; k <= 4; ++k) {
#pragma unroll 1
    for (int j = 0; j < (16 >> k); ++j) {
      u32 v = 0;
#pragma unroll 1
      for (int q = 0; q < (1 << k); ++q) v += cval<RW>(my[((j << k) + q) ^ sw]);
      if (v >= 256) big_node(S, G, s, k, v, N);
    }
  }
  u32 t = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) t += cval<RW>(my[q]);
  u32 tk[AIWC_NSKIP - 5];
#pragma unroll
  for (int k = 5; k < AIWC_NSKIP; ++k) {
    t += __shfl_xor(t, 1 << (k - 5), 64);
    tk[k - 5] = ((lane & ((1 << (k - 4)) - 1)) == 0) ? t : 0u;
  }
#pragma unroll 1
  for (int k = 5; k < AIWC_NSKIP; ++k) {
    u32 v = tk[0];
#pragma unroll
    for (int q = 1; q < AIWC_NSKIP - 5; ++q) v = (k == 5 + q) ? tk[q] : v;
    if (v >= 256) big_node(S, G, s, k, v, N);
  }
}

// As big_pass, but the nodes are appended to the block's list (their counts
// stay below 2^24: a staged page has at most HEAVY records).
template <bool RW>
__device__ __forceinline__ void big_collect(BucketShared &S, const u32 *cnt, int s) {
  const int lane = lane_id();
  const u32 *my = cnt + 16 * lane;
  const u32 sw = cswz((u32)lane);
  const u32 tag = (u32)s << 31;
#pragma unroll 1
  for (int k = 0; k <= 4; ++k) {
#pragma unroll 1
    for (int j = 0; j < (16 >> k); ++j) {
      u32 v = 0;
#pragma unroll 1
      for (int q = 0; q < (1 << k); ++q) v += cval<RW>(my[((j << k) + q) ^ sw]);
      if (v >= 256) {
        const u32 bi = atomicAdd(&S.nblist, 1u);
        if (bi < BLIST_CAP) S.blist[bi] = tag | ((u32)k << 24) | v;
      }
    }
  }
  u32 t = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) t += cval<RW>(my[q]);
#pragma unroll
  for (int k = 5; k < AIWC_NSKIP; ++k) {
    t += __shfl_xor(t, 1 << (k - 5), 64);
    if ((lane & ((1 << (k - 4)) - 1)) == 0 && t >= 256) {
      const u32 bi = atomicAdd(&S.nblist, 1u);
      if (bi < BLIST_CAP) S.blist[bi] = tag | ((u32)k << 24) | t;
    }
  }
}

// All levels of one page whose byte-offset counts sit in cnt[1024] (LDS,
// owned by this wavefront): with RW each counter holds reads | writes << 16,
// otherwise plain counts with read / write bitmaps in rb[32], wb[32].
// Lane l loads counters 16l..16l+15 (swizzled, see cslot): levels 0..4 are
// sums inside the lane, levels 5..10 sums across 2, 4, .., 64 lanes (the
// lowest lane owns the node).  Counts below 256 are accumulated in one pass
// (branch free, so that the table loads of a level issue back to back); if
// any node reaches 256, a second pass walks the tree again for those nodes
// only.
template <bool DEFER, bool RW>
__device__ __forceinline__ void page_levels(LaneAcc &L, BucketShared &S, SpecRef G,
                                            const u32 *cnt, const u32 *rb, const u32 *wb,
                                            u64 N) {
  const int lane = lane_id();
  const int s = L.space;
  const uint4 *src = reinterpret_cast<const uint4 *>(cnt + 16 * lane);
  const u32 sw = cswz((u32)lane);
  const u32 sh = sw >> 2;                  // which 16-byte chunk
  const bool s0 = (sw & 1u) != 0, s1 = (sw & 2u) != 0;   // order inside it
  u32 c[16];
  // the four loads are issued together (the scheduler would otherwise wait
  // for each before the next)
  uint4 xs[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) xs[q] = src[q ^ sh];
  __builtin_amdgcn_sched_group_barrier(0x0100, 4, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 x = xs[q];
    // element e of the chunk holds position e ^ (sw & 3)
    u32 a0 = s0 ? x.y : x.x, a1 = s0 ? x.x : x.y, a2 = s0 ? x.w : x.z, a3 = s0 ? x.z : x.w;
    c[4 * q] = s1 ? a2 : a0; c[4 * q + 1] = s1 ? a3 : a1;
    c[4 * q + 2] = s1 ? a0 : a2; c[4 * q + 3] = s1 ? a1 : a3;
  }
  // positions and nodes that are empty in every lane (most of them on
  // strided pages) are skipped by the whole wavefront
  if constexpr (RW) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (c[j] == 0) continue;
      L.ur += (c[j] & 0xFFFFu) != 0 ? 1u : 0u;
      L.uw += (c[j] >> 16) != 0 ? 1u : 0u;
      c[j] = (c[j] & 0xFFFFu) + (c[j] >> 16);
    }
  } else if (lane < 32) {
    L.ur += __builtin_popcount(rb[lane]);
    L.uw += __builtin_popcount(wb[lane]);
  }
  bool anybig = false;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (__ballot(c[j] != 0) == 0) continue;
    const u32 v = c[j] < 256 ? c[j] : 0u;
    add_small_node(L, S, 0, v);
    spec_node(L, S, v);
    anybig |= c[j] >= 256;
  }
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
#pragma unroll
    for (int j = 0; j < (16 >> k); ++j) {
      c[j] = c[2 * j] + c[2 * j + 1];
      if (c[j] == 0) continue;
      add_small_node(L, S, k, c[j] < 256 ? c[j] : 0u);
      anybig |= c[j] >= 256;
    }
  }
  // levels 5..8: sums over 2, 4, 8, 16 lanes by DPP (lane ^ 1, lane ^ 2,
  // half-row and row mirrors); 9 and 10 across rows
  u32 t = c[0];
#pragma unroll
  for (int k = 5; k < AIWC_NSKIP; ++k) {
    if (k == 5) t += (u32)__builtin_amdgcn_update_dpp(0, (int)t, 0xB1, 0xF, 0xF, false);
    else if (k == 6) t += (u32)__builtin_amdgcn_update_dpp(0, (int)t, 0x4E, 0xF, 0xF, false);
    else if (k == 7) t += (u32)__builtin_amdgcn_update_dpp(0, (int)t, 0x141, 0xF, 0xF, false);
    else if (k == 8) t += (u32)__builtin_amdgcn_update_dpp(0, (int)t, 0x140, 0xF, 0xF, false);
    else t += __shfl_xor(t, 1 << (k - 5), 64);
    const bool own = (lane & ((1 << (k - 4)) - 1)) == 0;
    add_small_node(L, S, k, (own && t < 256) ? t : 0u);
    anybig |= own && t >= 256;
  }
  if (__ballot(anybig) != 0) {
    if constexpr (DEFER) big_collect<RW>(S, cnt, s);
    else big_pass<RW>(S, G, cnt, s, N);
  }
}

// Up to 64 records of one address space, one per lane.  pm: the lanes that
// hold records of this lane's page (0 for an idle lane).  The level-k node of
// a lane's record is pm AND the lanes whose byte offsets agree with it on
// bits k..9; its lowest lane owns it.  Counts are at most 64.
__device__ __forceinline__ void match_levels(LaneAcc &L, BucketShared &S, u32 off, u32 w,
                                             u64 pm) {
  const int lane = lane_id();
  const u64 below = (1ull << lane) - 1ull;
  // counts of the owned nodes at every level first (ballots only), then all
  // table terms in one batch of loads
  u32 c[AIWC_NSKIP];
  u64 P = pm;
#pragma unroll
  for (int k = AIWC_NSKIP - 1; k >= 0; --k) {
    if (k < AIWC_NSKIP - 1) {
      const bool b = ((off >> k) & 1u) != 0;
      const u64 B = __ballot(b);
      P &= b ? B : ~B;
    }
    const bool own = P != 0 && (P & below) == 0;
    c[k] = own ? (u32)__builtin_popcountll(P) : 0u;
  }
  u64 t[AIWC_NSKIP];
#pragma unroll
  for (int k = 0; k < AIWC_NSKIP; ++k) t[k] = S.term[L.space][c[k] >= 2 ? c[k] : 0u];
#pragma unroll
  for (int k = 0; k < AIWC_NSKIP; ++k) {
    L.lo[k] += t[k];
    L.dn[k] += (c[k] != 0 ? 1u : 0u) + (c[k] == 1 ? 0x10000u : 0u);
  }
  spec_node(L, S, c[0]);
  // distinct read / written addresses: the lowest read (write) of each level-0 node
  const u64 Bw = __ballot(w != 0);
  const u64 Q = P & (w ? Bw : ~Bw);
  if (P != 0 && (Q & below) == 0) {
    if (w) L.uw += 1;
    else L.ur += 1;
  }
}

// Home slot of a page key in the page table (Fibonacci hashing: the high
// bits of the product depend on every key bit, including those above the
// ones a split fixes).
__device__ __forceinline__ u32 pt_slot(u64 pk) {
  return (u32)((pk * 0x9E3779B97F4A7C15ull) >> (64 - 11));
}

__device__ __forceinline__ u64 low_mask(u32 n) { return n >= 64 ? ~0ull : (1ull << n) - 1ull; }

template <bool BATCH>
__global__ void __launch_bounds__(BK_BLOCK) k_mem_bucket(TraceArgs A0, const TraceArgs *batch) {
  __shared__ BucketShared S;
  const TraceArgs A = trace_args<BATCH>(A0, batch);
  if (A.n_mem == 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / AIWC_WAVE;
  const u32 P = 1u << A.pbits;
  const u32 sbit = PAGE_BITS - A.pbits;            // space bit position in a page key
  const u64 N0 = A.acc->sp_reads[0] + A.acc->sp_writes[0];
  const u64 N1 = A.acc->sp_reads[1] + A.acc->sp_writes[1];
  const SpecRef G = {A.sp_f, A.sp_m, A.sp_cap};
  for (u32 i = tid; i < PT_SLOTS; i += BK_BLOCK) { S.pkey[i] = EMPTY; S.pcnt[i] = 0; }
  for (u32 i = tid; i < 2 * 256; i += BK_BLOCK) {
    u64 lo, hi;
    term_fx(i & 255u, (i >> 8) ? N1 : N0, lo, hi);
    S.term[i >> 8][i & 255u] = lo;   // below 2^54: hi is 0
    (&S.spec[0][0])[i] = 0;
  }
  for (u32 i = tid; i < 2 * SPEC_SLOTS; i += BK_BLOCK) {
    (&S.spf[0][0])[i] = 0;
    (&S.spm[0][0])[i] = 0;
  }
  if (tid < 2 * AIWC_NSKIP) {
    (&S.dist[0][0])[tid] = 0;
    S.el[tid / AIWC_NSKIP][tid % AIWC_NSKIP][0] = 0;
    S.el[tid / AIWC_NSKIP][tid % AIWC_NSKIP][1] = 0;
    S.el[tid / AIWC_NSKIP][tid % AIWC_NSKIP][2] = 0;
  }
  if (tid < 2) { S.ur[tid] = 0; S.uw[tid] = 0; }
  if (tid == 0) { S.redos = 0; S.npages = 0; S.overflow = 0; S.nblist = 0; }
  // the hot partitions (set before this kernel), read once
  const u32 nhot = A.mem_hot ? A.mem_hot[0] : 0u;
  if ((u32)tid < nhot) S.hotp[tid] = hot_parts(A.mem_hot)[tid].p;
  __syncthreads();

  const u32 Q = A.part_queue ? A.part_queue : P;   // entries of part_order to take
  while (true) {
    if (tid == 0) S.work = (u32)atomicAdd(&A.acc->mem_queue, 1ull);
    __syncthreads();
    if (S.work >= Q) break;
    const u32 p = A.part_order[S.work];
    const u64 base = A.part_off[p];
    u32 n = A.part_off[p + 1] - (u32)base;
    // a hot partition: its records off the candidate pages (compacted), the
    // candidates afterwards from their tables
    const u64 *prec = A.part_rec;
    int hidx = -1;
    if (nhot) {   // one entry per lane (nhot <= 64)
      const u64 hb = __ballot((u32)lane < nhot && S.hotp[lane < (int)nhot ? lane : 0] == p);
      if (hb) {
        hidx = __builtin_ctzll(hb);
        prec = A.part_cmp;
        n = hot_parts(A.mem_hot)[hidx].kept;
      }
    }
    if (tid == 0) { S.sp_top = 1; S.stack_m[0] = 1; S.stack_c[0] = 0; }
    __syncthreads();
    while (S.sp_top > 0) {
      const u32 M = S.stack_m[S.sp_top - 1], C = S.stack_c[S.sp_top - 1];
      __syncthreads();
      if (tid == 0) S.sp_top -= 1;
      // ---- 1. page pass (UNROLL records in flight per thread; the first
      // lane of each run of one page's records counts the whole run).  The
      // count before the run's addition is the run's first position inside
      // its page: every record leaves its tag (slot << 21 | position,
      // saturated) in part_tag, so that the regroup needs no table lookup.
      const u64 below = (1ull << lane) - 1ull;
      // software pipelined: the next batch's loads are in flight while this
      // batch is counted
      u64 nx[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const u32 i = (u32)tid + (u32)u * BK_BLOCK;
        nx[u] = i < n ? prec[base + i] : EMPTY;
      }
      for (u32 w0 = (u32)(tid - lane); w0 < n; w0 += BK_BLOCK * UNROLL) {
        u64 rv[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          rv[u] = nx[u];
          const u32 i = w0 + (u32)(BK_BLOCK * UNROLL) + (u32)u * BK_BLOCK + (u32)lane;
          nx[u] = i < n ? prec[base + i] : EMPTY;
        }
        // run heads and their first probe slots for all records at once
        u32 hs[UNROLL], run[UNROLL];
        u64 hw[UNROLL], HB[UNROLL];
        u32 vbits = 0;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const u64 pk = rv[u] >> 11;
          const bool valid = rv[u] != EMPTY && ((u32)pk & (M - 1u)) == C;
          const u64 ends = run_ends(valid ? pk : EMPTY);
          const bool head = valid && (lane == 0 || ((ends >> (lane - 1)) & 1ull) != 0);
          run[u] = head ? (u32)__builtin_ctzll(ends & ~below) - (u32)lane + 1u : 0u;
          hs[u] = pt_slot(pk);
          HB[u] = __ballot(head);
          vbits |= (valid ? 1u : 0u) << u;
        }
        // first probes: the page is usually in its home slot already, so the
        // table loads and the count atomics of all records are in flight
        // together; the rest take the probing loop
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) hw[u] = run[u] ? S.pkey[hs[u]] : EMPTY;
        u32 hv[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const u64 pk = rv[u] >> 11;
          hv[u] = 0;
          if (run[u] && hw[u] == pk) {
            const u32 at = atomicAdd(&S.pcnt[hs[u]], run[u]);
            hv[u] = (hs[u] << 21) | (at < TAG_POS ? at : TAG_POS);
            run[u] = 0;
          }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          if (!run[u]) continue;
          const u64 pk = rv[u] >> 11;
          u32 slot = hs[u];
          while (true) {
            u64 w = S.pkey[slot];
            if (w == EMPTY) {
              if (S.npages >= PT_CAP) { S.overflow = 1; break; }
              u64 old = atomicCAS(&S.pkey[slot], EMPTY, pk);
              if (old == EMPTY) {
                const u32 ci = atomicAdd(&S.npages, 1u);
                if (ci < PT_CAP) S.pslot[ci] = (uint16_t)slot;
                else S.overflow = 1;
                w = pk;
              } else {
                w = old;
              }
            }
            if (w == pk) {
              const u32 at = atomicAdd(&S.pcnt[slot], run[u]);
              hv[u] = (slot << 21) | (at < TAG_POS ? at : TAG_POS);
              break;
            }
            slot = (slot + 1 == PT_SLOTS) ? 0 : slot + 1;
          }
        }
        // each lane of a run takes its head's slot and the next position
        u32 *tagp = A.part_tag + base + w0 + (u32)lane;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const bool valid = ((vbits >> u) & 1u) != 0;
          const u64 H = HB[u] & (below | (1ull << lane));
          const int hl = H ? 63 - __builtin_clzll(H) : lane;
          const u32 h0 = __shfl(hv[u], hl, 64);
          const u32 pos = (h0 & TAG_POS) + (u32)(lane - hl);
          if (valid) tagp[u * BK_BLOCK] = (h0 & ~TAG_POS) | (pos < TAG_POS ? pos : TAG_POS);
        }
      }
      __syncthreads();
      const u32 np = S.npages < PT_CAP ? S.npages : PT_CAP;
      // ---- 2. page classes (small space 0 / small space 1 / other) and
      // staging offsets; order inside a class is free
      if (tid < 3) S.ctot[tid] = 0;
      if (tid == 0) { S.nbig0 = 0; S.nbig1 = 0; S.nheavy = 0; S.next_item = 0; }
      __syncthreads();
      for (u32 j0 = 0; j0 < np; j0 += BK_BLOCK) {
        const u32 j = j0 + tid;
        u32 c = 0, cl = 3, sp = 0;
        if (j < np) {
          const u32 slot = S.pslot[j];
          c = S.pcnt[slot];
          sp = (u32)((S.pkey[slot] >> sbit) & 1ull);
          cl = c <= SMALL ? sp : (c <= HEAVY ? 2u : 3u);
          S.psz[j] = (uint16_t)(c < 65535u ? c : 65535u);
        }
        // pages > SMALL join the space's list: one counter update per wavefront
        const bool l0 = j < np && c > SMALL && sp == 0, l1 = j < np && c > SMALL && sp == 1;
        const u64 B0 = __ballot(l0), B1 = __ballot(l1), BH = __ballot(j < np && c > HEAVY);
        u32 b0 = 0, b1 = 0;
        if (lane == 0) {
          if (B0) b0 = atomicAdd(&S.nbig0, (u32)__builtin_popcountll(B0));
          if (B1) b1 = atomicAdd(&S.nbig1, (u32)__builtin_popcountll(B1));
          if (BH) atomicAdd(&S.nheavy, (u32)__builtin_popcountll(BH));
        }
        b0 = (u32)__builtin_amdgcn_readfirstlane((int)b0);
        b1 = (u32)__builtin_amdgcn_readfirstlane((int)b1);
        // pend[j] holds the page's slot in the list until its start is known
        if (l0) {
          const u32 bi = b0 + (u32)__builtin_popcountll(B0 & below);
          S.big[bi] = j;
          S.pend[j] = bi;
        }
        if (l1) {
          const u32 bi = PT_CAP - 1 - (b1 + (u32)__builtin_popcountll(B1 & below));
          S.big[bi] = j;
          S.pend[j] = bi;
        }
        // class totals (classes 0 and 1 share a word: their counts are <= SMALL)
        const u32 t01 = wave_total((cl == 0 ? c : 0u) | ((cl == 1 ? c : 0u) << 16));
        const u32 t2 = wave_total(cl == 2 ? c : 0u);
        if (lane == 0) {
          if (t01 & 0xFFFFu) atomicAdd(&S.ctot[0], t01 & 0xFFFFu);
          if (t01 >> 16) atomicAdd(&S.ctot[1], t01 >> 16);
          if (t2) atomicAdd(&S.ctot[2], t2);
        }
      }
      __syncthreads();
      if (S.overflow || S.ctot[0] + S.ctot[1] + S.ctot[2] > STAGE_CAP) {
        // too many pages or records for one round: clear and split by one
        // more hash bit
        for (u32 i = tid; i < PT_SLOTS; i += BK_BLOCK) { S.pkey[i] = EMPTY; S.pcnt[i] = 0; }
        __syncthreads();
        if (tid == 0) {
          S.npages = 0; S.overflow = 0; S.redos += 1;
          if (M >= (1u << 30) || S.sp_top + 2 > 32) {
            atomicAdd(&A.acc->split_fail, 1ull);   // hash bits exhausted: report, never spin
          } else {
            S.stack_m[S.sp_top] = 2 * M; S.stack_c[S.sp_top] = C;
            S.stack_m[S.sp_top + 1] = 2 * M; S.stack_c[S.sp_top + 1] = C + M;
            S.sp_top += 2;
          }
        }
        __syncthreads();
        continue;
      }
      if (tid == 0) { S.ccur[0] = 0; S.ccur[1] = S.ctot[0]; S.ccur[2] = S.ctot[0] + S.ctot[1]; }
      __syncthreads();
      for (u32 j0 = 0; j0 < np; j0 += BK_BLOCK) {
        const u32 j = j0 + tid;
        u32 c = 0, cl = 3;
        if (j < np) {
          c = S.psz[j];
          cl = c <= SMALL ? (u32)((S.pkey[S.pslot[j]] >> sbit) & 1ull) : (c <= HEAVY ? 2u : 3u);
        }
        // per-class inclusive prefixes (a round stages <= STAGE_CAP < 2^16
        // records, so classes 0 and 1 share a word)
        const u32 v01 = (cl == 0 ? c : 0u) | ((cl == 1 ? c : 0u) << 16);
        const u32 v2 = cl == 2 ? c : 0u;
        const u32 x01 = wave_scan(v01), x2 = wave_scan(v2);
        const u32 w01 = (u32)__builtin_amdgcn_readlane((int)x01, 63);
        const u32 w2 = (u32)__builtin_amdgcn_readlane((int)x2, 63);
        u32 c0 = 0, c1 = 0, c2 = 0;
        if (lane == 0) {
          if (w01 & 0xFFFFu) c0 = atomicAdd(&S.ccur[0], w01 & 0xFFFFu);
          if (w01 >> 16) c1 = atomicAdd(&S.ccur[1], w01 >> 16);
          if (w2) c2 = atomicAdd(&S.ccur[2], w2);
        }
        c0 = (u32)__builtin_amdgcn_readfirstlane((int)c0);
        c1 = (u32)__builtin_amdgcn_readfirstlane((int)c1);
        c2 = (u32)__builtin_amdgcn_readfirstlane((int)c2);
        // pend: the page's end in the staging array; the page's table word
        // becomes its start | size << 15 (~0: not staged)
        u32 end = 0;
        if (cl == 0) end = c0 + (x01 & 0xFFFFu);
        else if (cl == 1) end = c1 + (x01 >> 16);
        else if (cl == 2) end = c2 + x2;
        if (j < np) {
          // a larger page's list entry becomes its start and size (one load
          // per item), a heavy page's keeps its index
          if (c > SMALL) S.big[S.pend[j]] = cl == 2 ? (end - c) | (c << 16) : HEAVY_TAG | j;
          S.pend[j] = end;
          S.pcnt[S.pslot[j]] = cl < 3 ? (end - c) | (c << 15) : ~0u;
        }
      }
      __syncthreads();
      // regroup: every staged record goes to its page's start plus the
      // position the page pass gave it
      u64 nr[UNROLL];
      u32 nt[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const u32 i = (u32)tid + (u32)u * BK_BLOCK;
        nr[u] = i < n ? prec[base + i] : EMPTY;
        nt[u] = i < n ? A.part_tag[base + i] : 0u;
      }
      for (u32 w0 = (u32)tid; w0 < n; w0 += BK_BLOCK * UNROLL) {
        u64 rv[UNROLL];
        u32 tg[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          rv[u] = nr[u];
          tg[u] = nt[u];
          const u32 i = w0 + (u32)(BK_BLOCK * UNROLL) + (u32)u * BK_BLOCK;
          nr[u] = i < n ? prec[base + i] : EMPTY;
          nt[u] = i < n ? A.part_tag[base + i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          if (rv[u] == EMPTY || ((u32)(rv[u] >> 11) & (M - 1u)) != C) continue;
          const u32 slot = tg[u] >> 21;
          const u32 pc = S.pcnt[slot];
          if (pc == ~0u) continue;
          const u32 p0 = (pc & 0x7FFFu) + (tg[u] & TAG_POS);
          if (p0 < STAGE_CAP) S.stage[p0] = (slot << 11) | (u32)(rv[u] & 2047ull);
        }
      }
      __syncthreads();
      const u32 nb0 = S.nbig0, nb1 = S.nbig1;
      // ---- 3a. heavy pages: counted by the whole block into dense[0]
      if (S.nheavy) {
        for (u32 bi = 0; bi < nb0 + nb1; ++bi) {
          const u32 be = S.big[bi < nb0 ? bi : PT_CAP - 1 - (bi - nb0)];
          if (!(be & HEAVY_TAG)) continue;
          const u32 ci = be & 0xFFFFu;
          const u64 hk = S.pkey[S.pslot[ci]];
          for (u32 i = tid; i < 1024; i += BK_BLOCK) S.dense[0][i] = 0;
          if (tid < 32) { S.rbits[tid] = 0; S.wbits[tid] = 0; }
          __syncthreads();
          for (u32 i0 = tid; i0 < n; i0 += BK_BLOCK * UNROLL) {
            u64 rv[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
              const u32 i = i0 + (u32)u * BK_BLOCK;
              rv[u] = i < n ? prec[base + i] : EMPTY;
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
              if (rv[u] == EMPTY || (rv[u] >> 11) != hk) continue;
              const u32 off = (u32)(rv[u] >> 1) & 1023u;
              atomicAdd(&S.dense[0][cslot(off)], 1u);
              atomicOr((rv[u] & 1u) ? &S.wbits[off >> 5] : &S.rbits[off >> 5],
                       1u << (off & 31u));
            }
          }
          __syncthreads();
          if (wave == 0) {
            const int sp = bi < nb0 ? 0 : 1;
            LaneAcc H;
            lacc_clear(H, sp);
            page_levels<false, false>(H, S, G, S.dense[0], S.rbits, S.wbits, sp ? N1 : N0);
            lacc_flush(H, S);
          }
          __syncthreads();
        }
      }
      // ---- 3b. per-wavefront items, space 0 first: small-page windows,
      // then larger pages; then the same for space 1
      {
        const u32 R0 = S.ctot[0], R1 = S.ctot[1];
        const u32 W0 = (R0 + SMALL - 1) / SMALL, W1 = (R1 + SMALL - 1) / SMALL;
        const u32 e0 = W0, e1 = e0 + nb0, e2 = e1 + W1, e3 = e2 + nb1;
        u32 *dn = S.dense[wave];
        LaneAcc L;
        lacc_clear(L, 0);
        // the next item's index is fetched while this one is processed
        u32 nxt = 0;
        if (lane == 0) nxt = atomicAdd(&S.next_item, 1u);
        while (true) {
          const u32 it = (u32)__builtin_amdgcn_readfirstlane((int)nxt);
          if (it >= e3) break;
          if (lane == 0) nxt = atomicAdd(&S.next_item, 1u);
          const int sp = (it < e1) ? 0 : 1;
          const u64 N = sp ? N1 : N0;
          if (sp != L.space) { lacc_flush(L, S); L.space = sp; }
          if (it < e0 || (it >= e1 && it < e2)) {
            // window of SMALL start positions inside the small pages of space sp
            const u32 lo = (it < e0) ? it * SMALL : R0 + (it - e1) * SMALL;
            const u32 rend = (it < e0) ? R0 : R0 + R1;
            const u32 i = lo + (u32)lane;
            u32 v = 0;
            u64 pm = 0;
            if (i < rend) {
              v = S.stage[i];
              const u32 pc = S.pcnt[v >> 11];
              const u32 sz = pc >> 15, st = pc & 0x7FFFu;
              if (st >= lo && st < lo + SMALL) pm = low_mask(sz) << (st - lo);
            }
            match_levels(L, S, (v >> 1) & 1023u, v & 1u, pm);
            continue;
          }
          const u32 be = S.big[(it < e1) ? it - e0 : PT_CAP - 1 - (it - e2)];
          if (be & HEAVY_TAG) continue;
          const u32 sz = be >> 16, o0 = be & 0xFFFFu, o1 = o0 + sz;
          if (sz <= MEDIUM) {
            const u32 v = (u32)lane < sz ? S.stage[o0 + lane] : 0u;
            match_levels(L, S, (v >> 1) & 1023u, v & 1u, (u32)lane < sz ? low_mask(sz) : 0ull);
            continue;
          }
          uint4 *z = reinterpret_cast<uint4 *>(dn + 16 * lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) z[q] = make_uint4(0, 0, 0, 0);
          __builtin_amdgcn_wave_barrier();
          for (u32 i0 = o0 + lane; i0 < o1; i0 += AIWC_WAVE * 4) {
            // four loads in flight together (an index past the page reads
            // the page's first record, which is then not counted)
            u32 vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const u32 i = i0 + (u32)u * AIWC_WAVE;
              vv[u] = S.stage[i < o1 ? i : o0];
            }
            __builtin_amdgcn_sched_group_barrier(0x0100, 4, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (i0 + (u32)u * AIWC_WAVE >= o1) continue;
              const u32 off = (vv[u] >> 1) & 1023u;
              atomicAdd(&dn[cslot(off)], (vv[u] & 1u) ? 0x10000u : 1u);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          page_levels<true, true>(L, S, G, dn, nullptr, nullptr, N);
          __builtin_amdgcn_wave_barrier();
        }
        lacc_flush(L, S);
      }
      __syncthreads();
      // ---- the round's dense-tree nodes of count >= 256
      const u32 nbl = S.nblist < BLIST_CAP ? S.nblist : BLIST_CAP;
      for (u32 i = tid; i < nbl; i += BK_BLOCK) {
        const u32 e = S.blist[i];
        const int sp = (int)(e >> 31);
        big_node(S, G, sp, (int)((e >> 24) & 127u), e & 0xFFFFFFu, sp ? N1 : N0);
      }
      __syncthreads();
      if (tid == 0) S.nblist = 0;
      // ---- release the page table for the next round / partition
      for (u32 j = tid; j < np; j += BK_BLOCK) {
        const u32 slot = S.pslot[j];
        S.pkey[slot] = EMPTY;
        S.pcnt[slot] = 0;
      }
      __syncthreads();
      if (tid == 0) S.npages = 0;
      __syncthreads();
    }
    // ---- a hot partition's candidate pages, each from its table (counts by
    // byte offset, read and write bitmaps), evaluated as a heavy page
    if (hidx >= 0) {
      const u32 nc = hot_parts(A.mem_hot)[hidx].ncand;
      for (u32 c = 0; c < nc; ++c) {
        const u32 *t = hot_tab(A.mem_hot, (u32)hidx, c);
        const u64 hk = hot_keys(A.mem_hot)[(u32)hidx * AIWC_HOT_CAND + c];
        for (u32 i = tid; i < 1024; i += BK_BLOCK) S.dense[0][cslot(i)] = t[i];
        if (tid < 32) { S.rbits[tid] = t[1024 + tid]; S.wbits[tid] = t[1056 + tid]; }
        __syncthreads();
        if (wave == 0) {
          const int sp = (int)((hk >> sbit) & 1ull);
          LaneAcc HL;
          lacc_clear(HL, sp);
          page_levels<false, false>(HL, S, G, S.dense[0], S.rbits, S.wbits, sp ? N1 : N0);
          lacc_flush(HL, S);
        }
        __syncthreads();
      }
    }
  }
  // ---- flush the block's accumulators
  __syncthreads();
  if (tid < 2 * AIWC_NSKIP) {
    const int s = tid / AIWC_NSKIP, k = tid % AIWC_NSKIP;
    if (S.dist[s][k]) atomicAdd(&A.acc->distinct[s][k], S.dist[s][k]);
    // limbs -> 128 bits, then 2^-40 units -> the 2^-64 units of the trace
    const u64 *el = S.el[s][k];
    const u64 lo = el[0] + (el[1] << 32);
    const u64 hi = (el[1] >> 32) + el[2] + (lo < el[0] ? 1ull : 0ull);
    atomic_add_u128(&A.acc->ent_lo[s][k], &A.acc->ent_hi[s][k], lo << 24,
                    (hi << 24) | (lo >> 40));
  }
  if (tid < 2) {
    if (S.ur[tid]) atomicAdd(&A.acc->uniq_r[tid], S.ur[tid]);
    if (S.uw[tid]) atomicAdd(&A.acc->uniq_w[tid], S.uw[tid]);
  }
  if (tid == 0 && S.redos) atomicAdd(&A.acc->redos, S.redos);
  for (u32 i = tid; i < 2 * SPEC_SLOTS; i += BK_BLOCK) {
    const u32 s = i / SPEC_SLOTS, j = i % SPEC_SLOTS;
    if (S.spf[s][j]) global_spec_add(G, s, S.spf[s][j], S.spm[s][j]);
  }
  for (u32 i = tid; i < 2 * SPEC_LDS; i += BK_BLOCK) {
    const u32 s = i / SPEC_LDS, c = i % SPEC_LDS;
    if (S.spec[s][c]) global_spec_add(G, s, c, S.spec[s][c]);
  }
}


}  // namespace

namespace aiwc_kernels {


template <typename K>
static void allow_big_lds(K kernel) {
  hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)(MAX_PARTS * 4));
}

hipError_t launch_mem(const TraceArgs &a, const BatchDims &d, hipStream_t s, StageMarks *pm) {
  hipError_t e = launch_mem_partition(a, d, s, pm);
  if (e == hipSuccess) e = launch_mem_bucket(a, d, s, pm);
  return e;
}

hipError_t launch_mem_bucket(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                             StageMarks *pm) {
  if (!d.any_mem) return hipSuccess;
  const dim3 gb((unsigned)(d.max_parts < 512 ? d.max_parts : 512), d.n);
  const TraceArgs *b = d.batch;
  if (b) hipLaunchKernelGGL(k_mem_bucket<true>, gb, dim3(BK_BLOCK), 0, s, a, b);
  else hipLaunchKernelGGL(k_mem_bucket<false>, gb, dim3(BK_BLOCK), 0, s, a, b);
  AIWC_MARK(pm, "k_mem_bucket", s);
  return hipGetLastError();
}

hipError_t launch_mem_count(const TraceArgs &a, u32 *count, hipStream_t s) {
  if (a.n_mem == 0) return hipSuccess;
  static bool attr = false;
  if (!attr) { allow_big_lds(k_mem_count); attr = true; }
  const u64 want = (a.n_mem + 16383) / 16384;
  const unsigned g = (unsigned)(want < 1024 ? (want ? want : 1) : 1024);
  hipLaunchKernelGGL(k_mem_count, dim3(g), dim3(GRP_BLOCK), (size_t)4 << a.pbits, s, a, count);
  return hipGetLastError();
}

hipError_t launch_mem_scatter_range(const TraceArgs &a, u32 p0, u32 p1, u32 *cursor, u64 *rec,
                                    hipStream_t s) {
  if (a.n_mem == 0 || p1 <= p0) return hipSuccess;
  static bool attr = false;
  if (!attr) { allow_big_lds(k_mem_scatter_range); attr = true; }
  const u64 want = (a.n_mem + 16383) / 16384;
  const unsigned g = (unsigned)(want < 1024 ? (want ? want : 1) : 1024);
  hipLaunchKernelGGL(k_mem_scatter_range, dim3(g), dim3(GRP_BLOCK), (size_t)4 * (p1 - p0), s, a,
                     p0, p1, cursor, rec);
  return hipGetLastError();
}

hipError_t launch_mem_partition(const TraceArgs &a, const BatchDims &d, hipStream_t s,
                                StageMarks *pm) {
  if (!d.any_mem) return hipSuccess;
  static bool attrs = false;
  if (!attrs) {
    allow_big_lds(k_mem_hist<true, true>); allow_big_lds(k_mem_hist<false, true>);
    allow_big_lds(k_mem_hist<true, false>); allow_big_lds(k_mem_hist<false, false>);
    allow_big_lds(k_mem_scatter<true, true>); allow_big_lds(k_mem_scatter<false, true>);
    allow_big_lds(k_mem_scatter<true, false>); allow_big_lds(k_mem_scatter<false, false>);
    attrs = true;
  }
  const size_t lds = (size_t)d.max_parts * 4;
  const dim3 gh((unsigned)d.max_hist_blocks, d.n), gc((unsigned)((d.max_parts + 255) / 256), d.n);
  const dim3 g1(1, d.n);
  const TraceArgs *b = d.batch;
  if (b) {
    if (d.vec) hipLaunchKernelGGL((k_mem_hist<true, true>), gh, dim3(MEM_BLOCK), lds, s, a, b);
    else hipLaunchKernelGGL((k_mem_hist<false, true>), gh, dim3(MEM_BLOCK), lds, s, a, b);
  } else {
    if (d.vec) hipLaunchKernelGGL((k_mem_hist<true, false>), gh, dim3(MEM_BLOCK), lds, s, a, b);
    else hipLaunchKernelGGL((k_mem_hist<false, false>), gh, dim3(MEM_BLOCK), lds, s, a, b);
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
  if (d.any_one_level) {
    if (b) {
      if (d.vec) hipLaunchKernelGGL((k_mem_scatter<true, true>), gh, dim3(MEM_BLOCK), lds, s, a, b);
      else hipLaunchKernelGGL((k_mem_scatter<false, true>), gh, dim3(MEM_BLOCK), lds, s, a, b);
    } else {
      if (d.vec) hipLaunchKernelGGL((k_mem_scatter<true, false>), gh, dim3(MEM_BLOCK), lds, s, a, b);
      else hipLaunchKernelGGL((k_mem_scatter<false, false>), gh, dim3(MEM_BLOCK), lds, s, a, b);
    }
  }
  if (d.any_two_level) {
    // persistent tiles: two 84 KiB blocks per CU
    const dim3 gt(1024, d.n);
    if (b) {
      if (d.vec) hipLaunchKernelGGL((k_mem_scatter_a<true, true>), gt, dim3(SC_BLOCK), 0, s, a, b);
      else hipLaunchKernelGGL((k_mem_scatter_a<false, true>), gt, dim3(SC_BLOCK), 0, s, a, b);
      hipLaunchKernelGGL(k_mem_scatter_b<true>, gt, dim3(SC_BLOCK), 0, s, a, b);
    } else {
      if (d.vec) hipLaunchKernelGGL((k_mem_scatter_a<true, false>), gt, dim3(SC_BLOCK), 0, s, a, b);
      else hipLaunchKernelGGL((k_mem_scatter_a<false, false>), gt, dim3(SC_BLOCK), 0, s, a, b);
      hipLaunchKernelGGL(k_mem_scatter_b<false>, gt, dim3(SC_BLOCK), 0, s, a, b);
    }
  }
  if (d.any_hot_mem) {   // counted in the scatter's stage time
    const dim3 gp(AIWC_HOT_PMAX, d.n), gc(512, d.n);
    if (b) {
      hipLaunchKernelGGL(k_mem_hot_pick<true>, gp, dim3(1024), 0, s, a, b);
      hipLaunchKernelGGL(k_mem_hot_count<true>, gc, dim3(1024), 0, s, a, b);
    } else {
      hipLaunchKernelGGL(k_mem_hot_pick<false>, gp, dim3(1024), 0, s, a, b);
      hipLaunchKernelGGL(k_mem_hot_count<false>, gc, dim3(1024), 0, s, a, b);
    }
  }
  AIWC_MARK(pm, "k_mem_scatter", s);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
