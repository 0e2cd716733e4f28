// producer.hip -- the trace producer: a kernel program (aiwc_insn records)
// interpreted on the GPU, one thread per work-item and one workgroup per
// work-group, emitting the event arrays that the characterization reads.
//
// The paper's trace comes from a simulator that interprets a kernel's LLVM IR
// and notifies the AIWC plugin of every executed instruction, memory access
// and branch outcome (Implementation section).  Here the same notifications
// become array writes:
//   k_interp<false>  the counting run: executes the kernel and counts each
//                    work-item's instructions, memory events and branches;
//   k_count_sums / k_offsets
//                    exclusive scans of those counts (block sums added on the
//                    host between the two launches) = every work-item's
//                    output ranges; the instruction scan is wi_offsets;
//   k_interp<true>   the recording run (buffers restored first): writes the
//                    opcode ids and memory events into the work-item's
//                    ranges, branch events into a staging range, and at every
//                    barrier and at the end moves the interval's branch
//                    events into the paper's schedule order (work-items of a
//                    work-group one after another within each barrier
//                    interval).
// Barriers are taken at one block-uniform point (__syncthreads_count), never
// inside divergent code, so a program whose work-items disagree about a
// barrier ends with an error instead of waiting.  Every memory access is
// checked against its buffer, every output write against its range.
#include <algorithm>
#include <cstring>
#include <vector>

#include "abi_internal.h"

#pragma clang fp contract(off)

typedef unsigned short u16;
typedef unsigned char u8;

#define HIP_OR_RET(ctx, call)                                                   \
  do {                                                                          \
    hipError_t e__ = (call);                                                    \
    if (e__ != hipSuccess) {                                                    \
      ctx_error(ctx, "%s failed: %s", #call, hipGetErrorString(e__));           \
      return AIWC_ERR_HIP;                                                      \
    }                                                                           \
  } while (0)

namespace {

constexpr u32 E_BOUNDS = 1, E_ALIGN = 2, E_STEPS = 4, E_BARRIER = 8, E_PC = 16, E_SCHED = 32;
constexpr u32 ST_RUN = 0, ST_WAIT = 1, ST_DONE = 2;
constexpr u64 TAG_MASK = (1ull << AIWC_ADDR_TAG_SHIFT) - 1;
constexpr u32 SCAN_BLOCK = 1024;

struct ProdLaunch {
  const aiwc_insn *code;
  u32 n_insn, wg;
  u32 lsz[3], ngr[3];
  u32 local_bytes, n_args, n_buf, pad;
  u64 max_steps;
  u64 args[AIWC_MAX_KERNEL_ARGS];
  u64 buf_ptr[AIWC_MAX_KERNEL_ARGS];
  u64 buf_bytes[AIWC_MAX_KERNEL_ARGS];
  u32 *cnt;                 // counting run: 3 per work-item (instr, memory, branch)
  u32 *err;                 // [0] error bits; [2..3] u64 first (w << 20 | pc)
  const u64 *ev_off, *mem_off, *br_off;   // recording run: W + 1 each
  u16 *opcode;
  u64 *addr;
  u8 *mkind;
  u32 *bsite;
  u8 *btaken;
  u32 *ssite;               // branch staging, work-item major
  u8 *staken;
};

__device__ __forceinline__ float as_f(u64 v) { return __uint_as_float((u32)v); }
__device__ __forceinline__ u64 f_bits(float x) {
  u32 u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) u = 0x7FC00000u;   // one NaN
  return u;
}

__device__ __forceinline__ u64 int_op(u32 op, u64 x, u64 y) {
  const long long sx = (long long)x, sy = (long long)y;
  switch (op) {
    case AIWC_OP_ADD: return x + y;
    case AIWC_OP_SUB: return x - y;
    case AIWC_OP_MUL: return x * y;
    case AIWC_OP_SDIV:
      if (y == 0) return 0;
      if (sx == (long long)0x8000000000000000ull && sy == -1) return x;
      return (u64)(sx / sy);
    case AIWC_OP_SREM:
      if (y == 0 || sy == -1) return 0;
      return (u64)(sx % sy);
    case AIWC_OP_UDIV: return y ? x / y : 0;
    case AIWC_OP_UREM: return y ? x % y : 0;
    case AIWC_OP_SHL: return x << (y & 63);
    case AIWC_OP_LSHR: return x >> (y & 63);
    case AIWC_OP_ASHR: return (u64)(sx >> (y & 63));
    case AIWC_OP_AND: return x & y;
    case AIWC_OP_OR: return x | y;
    default: return x ^ y;   // AIWC_OP_XOR
  }
}

__device__ __forceinline__ u64 icmp(u32 mode, u64 x, u64 y) {
  const long long sx = (long long)x, sy = (long long)y;
  bool r;
  switch (mode) {
    case AIWC_ICMP_EQ: r = x == y; break;
    case AIWC_ICMP_NE: r = x != y; break;
    case AIWC_ICMP_SLT: r = sx < sy; break;
    case AIWC_ICMP_SLE: r = sx <= sy; break;
    case AIWC_ICMP_SGT: r = sx > sy; break;
    case AIWC_ICMP_SGE: r = sx >= sy; break;
    case AIWC_ICMP_ULT: r = x < y; break;
    case AIWC_ICMP_ULE: r = x <= y; break;
    case AIWC_ICMP_UGT: r = x > y; break;
    default: r = x >= y; break;   // AIWC_ICMP_UGE
  }
  return r ? 1 : 0;
}

__device__ __forceinline__ u64 fcmp(u32 mode, float x, float y) {
  bool r;
  switch (mode) {
    case AIWC_FCMP_OEQ: r = x == y; break;
    case AIWC_FCMP_UNE: r = !(x == y); break;
    case AIWC_FCMP_OLT: r = x < y; break;
    case AIWC_FCMP_OLE: r = x <= y; break;
    case AIWC_FCMP_OGT: r = x > y; break;
    default: r = x >= y; break;   // AIWC_FCMP_OGE
  }
  return r ? 1 : 0;
}

// fmin / fmax: a NaN operand yields the other one; -0 orders below +0
__device__ __forceinline__ float fmin_ord(float x, float y, bool is_max) {
  if (x != x) return y;
  if (y != y) return x;
  if (x < y) return is_max ? y : x;
  if (y < x) return is_max ? x : y;
  const bool xneg = (__float_as_uint(x) >> 31) != 0;   // equal values: pick by sign
  return (xneg != is_max) ? x : y;
}

// Correctly rounded square root: the hardware estimate, then moved to the
// neighbour whose rounding interval holds sqrt(x).  The midpoints between
// neighbouring binary32 values have at most 25 significant bits, so their
// squares are exact in binary64 and each comparison with x is exact.
__device__ __forceinline__ float sqrt_rn(float x) {
  float r = __fsqrt_rn(x);
  if (!(x > 0.0f) || !(r < 3.4028235e38f) || !(r > 0.0f)) return r;   // 0, -0, < 0, NaN, inf, max
  const double dx = (double)x;
  for (int it = 0; it < 2; ++it) {
    const u32 b = __float_as_uint(r);
    const double up = (double)__uint_as_float(b + 1), dn = (double)__uint_as_float(b - 1);
    const double hi = 0.5 * ((double)r + up), lo = 0.5 * ((double)r + dn);
    if (hi * hi <= dx) r = __uint_as_float(b + 1);
    else if (lo * lo > dx) r = __uint_as_float(b - 1);
    else break;
  }
  return r;
}

__device__ __forceinline__ u64 fptosi32(float x) {
  int r;
  if (x != x) r = 0;
  else if (x >= 2147483648.0f) r = 2147483647;
  else if (x < -2147483648.0f) r = (int)0x80000000u;
  else r = (int)x;   // truncates toward zero
  return (u64)(long long)r;
}

// work-item functions: mode / 3 = function, mode % 3 = dimension
__device__ __forceinline__ u64 builtin(const ProdLaunch &L, u32 mode, const u32 lid[3],
                                       const u32 gr[3]) {
  const u32 dim = mode % 3;
  switch (mode / 3) {
    case 0: return (u64)gr[dim] * L.lsz[dim] + lid[dim];
    case 1: return lid[dim];
    case 2: return gr[dim];
    case 3: return (u64)L.lsz[dim] * L.ngr[dim];
    case 4: return L.lsz[dim];
    default: return L.ngr[dim];
  }
}

__device__ __forceinline__ void set_error(const ProdLaunch &L, u32 bits, u64 w, u32 pc) {
  atomicOr(L.err, bits);
  atomicMin((unsigned long long *)(L.err + 2), (unsigned long long)((w << 20) | pc));
}

// Address of an access of `bytes` bytes aligned to `elt`, or nullptr (error
// recorded) when it leaves its buffer or is misaligned.
__device__ __forceinline__ unsigned char *resolve(const ProdLaunch &L, unsigned char *lmem, u64 va,
                                                  u32 bytes, u32 elt, bool &local, u64 w, u32 pc) {
  const u64 tag = va >> AIWC_ADDR_TAG_SHIFT, off = va & TAG_MASK;
  if (off & (elt - 1)) { set_error(L, E_ALIGN, w, pc); return nullptr; }
  if (tag == 0) {
    local = true;
    if (off + bytes > L.local_bytes) { set_error(L, E_BOUNDS, w, pc); return nullptr; }
    return lmem + off;
  }
  local = false;
  const u64 bi = tag - 1;
  if (bi >= L.n_buf || off + bytes > L.buf_bytes[bi]) { set_error(L, E_BOUNDS, w, pc); return nullptr; }
  return (unsigned char *)L.buf_ptr[bi] + off;
}

__device__ __forceinline__ u32 atomic_op(u32 mode, unsigned char *p, u32 v) {
  unsigned int *q = (unsigned int *)p;
  switch (mode) {
    case AIWC_AT_ADD: return atomicAdd(q, v);
    case AIWC_AT_SUB: return atomicSub(q, v);
    case AIWC_AT_AND: return atomicAnd(q, v);
    case AIWC_AT_OR: return atomicOr(q, v);
    case AIWC_AT_XOR: return atomicXor(q, v);
    case AIWC_AT_MIN: return (u32)atomicMin((int *)q, (int)v);
    case AIWC_AT_MAX: return (u32)atomicMax((int *)q, (int)v);
    case AIWC_AT_UMIN: return atomicMin(q, v);
    default: return atomicMax(q, v);   // AIWC_AT_UMAX
  }
}

// Inclusive block scan (Hillis-Steele over LDS; phases are rare).
__device__ u64 block_incl_scan(u64 v, u64 *tmp, u32 n, u64 &total) {
  const u32 t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (u32 off = 1; off < n; off <<= 1) {
    const u64 x = t >= off ? tmp[t - off] : 0;
    __syncthreads();
    tmp[t] += x;
    __syncthreads();
  }
  const u64 r = tmp[t];
  total = tmp[n - 1];
  __syncthreads();
  return r;
}

template <bool REC>
__global__ __launch_bounds__(1024) void k_interp(ProdLaunch L) {
  extern __shared__ __align__(16) unsigned char lmem[];
  const u32 t = threadIdx.x, wg = L.wg;
  const u64 grp = blockIdx.x;
  const u64 w = grp * wg + t;
  const u32 lbytes16 = (L.local_bytes + 15u) & ~15u;
  for (u32 i = t * 16; i < lbytes16; i += wg * 16) *(uint4 *)(lmem + i) = make_uint4(0, 0, 0, 0);
  u64 *scan_tmp = (u64 *)(lmem + lbytes16);

  u32 lid[3], gr[3];
  lid[0] = t % L.lsz[0];
  lid[1] = (t / L.lsz[0]) % L.lsz[1];
  lid[2] = t / (L.lsz[0] * L.lsz[1]);
  gr[0] = (u32)(grp % L.ngr[0]);
  gr[1] = (u32)((grp / L.ngr[0]) % L.ngr[1]);
  gr[2] = (u32)(grp / ((u64)L.ngr[0] * L.ngr[1]));

  u64 R[AIWC_NREG];
  for (u32 r = 0; r < AIWC_NREG; ++r) R[r] = r < L.n_args ? L.args[r] : 0;
  __syncthreads();   // local memory zeroed

  u32 pc = 0, state = ST_RUN;
  u64 steps = 0;
  u32 nev = 0, nmem = 0, nbr = 0;
  u64 ev_pos = 0, ev_end = 0, mem_pos = 0, mem_end = 0, st_pos = 0, st_end = 0;
  u64 st_first = 0, run_base = 0, blk_end = 0;
  u32 ph_br = 0;
  if (REC) {
    ev_pos = L.ev_off[w]; ev_end = L.ev_off[w + 1];
    mem_pos = L.mem_off[w]; mem_end = L.mem_off[w + 1];
    st_pos = st_first = L.br_off[w]; st_end = L.br_off[w + 1];
    run_base = L.br_off[grp * wg];
    blk_end = L.br_off[grp * wg + wg];
  }
  bool sched_bad = false;

  for (;;) {
    while (state == ST_RUN) {
      if (pc >= L.n_insn) { set_error(L, E_PC, w, pc); state = ST_DONE; break; }
      if (++steps > L.max_steps) { set_error(L, E_STEPS, w, pc); state = ST_DONE; break; }
      const aiwc_insn I = L.code[pc];
      if (REC) {
        if (ev_pos < ev_end) L.opcode[ev_pos] = I.id; else sched_bad = true;
        ++ev_pos;
      }
      ++nev;
      const u32 op = I.op, wd = I.width, d = I.d & 63, a = I.a & 63, b = I.b & 63, c = I.c & 63;
      const bool immb = (I.flags & AIWC_INSN_IMM_B) != 0;
      const u64 imm = (u64)I.imm;
      u32 next = pc + 1;
#define BV(i) (immb ? imm : R[(b + (i)) & 63])
      switch (op) {
        case AIWC_OP_RET: state = ST_DONE; break;
        case AIWC_OP_MOV:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = BV(i);
          break;
        case AIWC_OP_ICMP:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = icmp(I.mode, R[(a + i) & 63], BV(i));
          break;
        case AIWC_OP_FADD: case AIWC_OP_FSUB: case AIWC_OP_FMUL: case AIWC_OP_FDIV:
          for (u32 i = 0; i < wd; ++i) {
            const float x = as_f(R[(a + i) & 63]), y = as_f(BV(i));
            float r;
            if (op == AIWC_OP_FADD) r = __fadd_rn(x, y);
            else if (op == AIWC_OP_FSUB) r = __fsub_rn(x, y);
            else if (op == AIWC_OP_FMUL) r = __fmul_rn(x, y);
            else r = __fdiv_rn(x, y);
            R[(d + i) & 63] = f_bits(r);
          }
          break;
        case AIWC_OP_FCMP:
          for (u32 i = 0; i < wd; ++i)
            R[(d + i) & 63] = fcmp(I.mode, as_f(R[(a + i) & 63]), as_f(BV(i)));
          break;
        case AIWC_OP_FMA:
          for (u32 i = 0; i < wd; ++i)
            R[(d + i) & 63] = f_bits(__fmaf_rn(as_f(R[(a + i) & 63]), as_f(BV(i)), as_f(R[(c + i) & 63])));
          break;
        case AIWC_OP_FSQRT:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = f_bits(sqrt_rn(as_f(R[(a + i) & 63])));
          break;
        case AIWC_OP_FMIN: case AIWC_OP_FMAX:
          for (u32 i = 0; i < wd; ++i)
            R[(d + i) & 63] = f_bits(fmin_ord(as_f(R[(a + i) & 63]), as_f(BV(i)), op == AIWC_OP_FMAX));
          break;
        case AIWC_OP_SITOFP:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = f_bits((float)(int)(u32)R[(a + i) & 63]);
          break;
        case AIWC_OP_FPTOSI:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = fptosi32(as_f(R[(a + i) & 63]));
          break;
        case AIWC_OP_SEXT:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = (u64)(long long)(int)(u32)R[(a + i) & 63];
          break;
        case AIWC_OP_ZEXT:
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = R[(a + i) & 63] & 0xFFFFFFFFull;
          break;
        case AIWC_OP_SELECT:
          for (u32 i = 0; i < wd; ++i)
            R[(d + i) & 63] = R[(a + i) & 63] ? BV(i) : R[(c + i) & 63];
          break;
        case AIWC_OP_GEP:
          for (u32 i = 0; i < wd; ++i)
            R[(d + i) & 63] = immb ? R[(a + i) & 63] + imm : R[(a + i) & 63] + R[(b + i) & 63] * imm;
          break;
        case AIWC_OP_LOAD: case AIWC_OP_STORE: {
          const u64 va = R[a];
          const u32 elt = op == AIWC_OP_LOAD ? (I.mode == AIWC_LD_64 ? 8u : 4u)
                                             : (I.mode == AIWC_ST_64 ? 8u : 4u);
          bool local = false;
          unsigned char *p = resolve(L, lmem, va, elt * wd, elt, local, w, pc);
          if (!p) { state = ST_DONE; break; }
          if (op == AIWC_OP_LOAD) {
            for (u32 i = 0; i < wd; ++i) {
              u64 v;
              if (elt == 8) v = *(const u64 *)(p + 8 * i);
              else {
                const u32 x = *(const u32 *)(p + 4 * i);
                v = I.mode == AIWC_LD_I32 ? (u64)(long long)(int)x : (u64)x;
              }
              R[(d + i) & 63] = v;
            }
          } else {
            for (u32 i = 0; i < wd; ++i) {
              const u64 v = BV(i);
              if (elt == 8) *(u64 *)(p + 8 * i) = v;
              else *(u32 *)(p + 4 * i) = (u32)v;
            }
          }
          if (REC) {
            if (mem_pos < mem_end) {
              L.addr[mem_pos] = va;
              L.mkind[mem_pos] = (u8)((op == AIWC_OP_STORE ? AIWC_MEM_WRITE : 0u) | (local ? AIWC_MEM_LOCAL : 0u));
            } else sched_bad = true;
            ++mem_pos;
          }
          ++nmem;
          break;
        }
        case AIWC_OP_ATOMIC: {
          const u64 va = R[a];
          bool local = false;
          unsigned char *p = resolve(L, lmem, va, 4, 4, local, w, pc);
          if (!p) { state = ST_DONE; break; }
          const u32 old = atomic_op(I.mode, p, (u32)BV(0));
          R[d] = (u64)(long long)(int)old;
          if (REC) {
            const u8 lk = local ? (u8)AIWC_MEM_LOCAL : (u8)0;
            if (mem_pos + 1 < mem_end) {
              L.addr[mem_pos] = va; L.mkind[mem_pos] = lk;
              L.addr[mem_pos + 1] = va; L.mkind[mem_pos + 1] = (u8)(lk | AIWC_MEM_WRITE);
            } else sched_bad = true;
            mem_pos += 2;
          }
          nmem += 2;
          break;
        }
        case AIWC_OP_BR: {
          const bool taken = R[a] != 0;
          if (REC) {
            if (st_pos < st_end) { L.ssite[st_pos] = I.site; L.staken[st_pos] = taken ? 1 : 0; }
            else sched_bad = true;
            ++st_pos;
            ++ph_br;
          }
          ++nbr;
          next = taken ? (u32)I.imm : I.target2;
          break;
        }
        case AIWC_OP_JMP: next = (u32)I.imm; break;
        case AIWC_OP_BARRIER: state = ST_WAIT; break;
        case AIWC_OP_BUILTIN: R[d] = builtin(L, I.mode, lid, gr); break;
        default:   // the integer binary operations
          for (u32 i = 0; i < wd; ++i) R[(d + i) & 63] = int_op(op, R[(a + i) & 63], BV(i));
          break;
      }
#undef BV
      pc = next;
    }
    if (REC) {
      // move this barrier interval's branch events into schedule order
      u64 total;
      const u64 incl = block_incl_scan(ph_br, scan_tmp, wg, total);
      const u64 dst = run_base + incl - ph_br;
      for (u32 k = 0; k < ph_br; ++k) {
        const u64 s = st_first + k, o = dst + k;
        if (s < st_end && o < blk_end) { L.bsite[o] = L.ssite[s]; L.btaken[o] = L.staken[s]; }
        else sched_bad = true;
      }
      run_base += total;
      st_first += ph_br;
      ph_br = 0;
    }
    const int waiting = __syncthreads_count(state == ST_WAIT);
    if (waiting == 0) break;
    if (waiting != (int)wg) {
      if (state == ST_WAIT) set_error(L, E_BARRIER, w, pc);
      break;
    }
    state = ST_RUN;
  }
  if (!REC) {
    L.cnt[3 * w] = nev;
    L.cnt[3 * w + 1] = nmem;
    L.cnt[3 * w + 2] = nbr;
  } else if (sched_bad || ev_pos != ev_end || mem_pos != mem_end || st_pos != st_end) {
    set_error(L, E_SCHED, w, pc);
  }
}

// Block sums of the three per-work-item counts (SCAN_BLOCK work-items each).
__global__ __launch_bounds__(SCAN_BLOCK) void k_count_sums(const u32 *cnt, u64 W, u64 *bsum) {
  __shared__ u64 red[3][SCAN_BLOCK / 64];
  const u64 i = (u64)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  for (u32 j = 0; j < 3; ++j) {
    u64 v = i < W ? cnt[3 * i + j] : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    u64 s = 0;
    for (u32 k = 0; k < SCAN_BLOCK / 64; ++k) s += red[threadIdx.x][k];
    bsum[3 * (u64)blockIdx.x + threadIdx.x] = s;
  }
}

// Exclusive offsets: block offset (from the host) + exclusive scan in block.
__global__ __launch_bounds__(SCAN_BLOCK) void k_offsets(const u32 *cnt, u64 W, const u64 *boff,
                                                        u64 *ev_off, u64 *mem_off, u64 *br_off) {
  __shared__ u64 tmp[SCAN_BLOCK];
  const u64 i = (u64)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  u64 *outs[3] = {ev_off, mem_off, br_off};
  for (u32 j = 0; j < 3; ++j) {
    const u64 v = i < W ? cnt[3 * i + j] : 0;
    u64 total;
    const u64 incl = block_incl_scan(v, tmp, SCAN_BLOCK, total);
    if (i < W) outs[j][i] = boff[3 * (u64)blockIdx.x + j] + incl - v;
  }
}

}  // namespace

// ------------------------------------------------------------------- host

struct aiwc_program {
  aiwc_ctx *ctx = nullptr;
  u32 n_insn = 0, n_sites = 0;
  aiwc_insn *dev_code = nullptr;
  std::vector<aiwc_opcode_info> table;
};

struct aiwc_produced {
  aiwc_ctx *ctx = nullptr;
  std::vector<aiwc_opcode_info> table;
  u32 n_sites = 0, wg = 0;
  u64 W = 0, n_ev = 0, n_mem = 0, n_br = 0;
  u16 *opcode = nullptr;
  u64 *wi_off = nullptr, *addr = nullptr;
  u8 *mkind = nullptr, *btaken = nullptr;
  u32 *bsite = nullptr;
};

static bool op_uses_b(u32 op) {
  switch (op) {
    case AIWC_OP_RET: case AIWC_OP_FSQRT: case AIWC_OP_SITOFP: case AIWC_OP_FPTOSI:
    case AIWC_OP_SEXT: case AIWC_OP_ZEXT: case AIWC_OP_LOAD: case AIWC_OP_BR: case AIWC_OP_JMP:
    case AIWC_OP_BARRIER: case AIWC_OP_BUILTIN:
      return false;
    default:
      return true;
  }
}

static bool op_uses_a(u32 op) {
  switch (op) {
    case AIWC_OP_RET: case AIWC_OP_MOV: case AIWC_OP_JMP: case AIWC_OP_BARRIER:
    case AIWC_OP_BUILTIN:
      return false;
    default:
      return true;
  }
}

static bool op_writes_d(u32 op) {
  switch (op) {
    case AIWC_OP_RET: case AIWC_OP_STORE: case AIWC_OP_BR: case AIWC_OP_JMP: case AIWC_OP_BARRIER:
      return false;
    default:
      return true;
  }
}

// Instructions whose width must be 1 (control, work-item functions, atomics).
static bool scalar_only(u32 op) {
  return op == AIWC_OP_RET || op == AIWC_OP_ATOMIC || op == AIWC_OP_BR || op == AIWC_OP_JMP ||
         op == AIWC_OP_BARRIER || op == AIWC_OP_BUILTIN;
}

static int kind_needed(u32 op) {
  switch (op) {
    case AIWC_OP_LOAD: return AIWC_KIND_LOAD;
    case AIWC_OP_STORE: return AIWC_KIND_STORE;
    case AIWC_OP_ATOMIC: return AIWC_KIND_ATOMIC_RMW;
    case AIWC_OP_BR: return AIWC_KIND_BRANCH_COND;
    case AIWC_OP_BARRIER: return AIWC_KIND_BARRIER;
    default: return -1;   // COMPUTE or OTHER
  }
}

static u32 max_mode(u32 op) {
  switch (op) {
    case AIWC_OP_ICMP: return AIWC_ICMP_UGE;
    case AIWC_OP_FCMP: return AIWC_FCMP_OGE;
    case AIWC_OP_LOAD: return AIWC_LD_64;
    case AIWC_OP_STORE: return AIWC_ST_64;
    case AIWC_OP_ATOMIC: return AIWC_AT_UMAX;
    case AIWC_OP_BUILTIN: return AIWC_BI_NUM_GROUPS + 2;
    default: return 0;
  }
}

// register ranges [x, x+n) and [y, y+n) equal or disjoint
static bool same_or_disjoint(u32 x, u32 y, u32 n) { return x == y || x + n <= y || y + n <= x; }

static bool check_insn(const aiwc_insn &I, u32 idx, const aiwc_program_desc *d, char *why, size_t wn) {
  const u32 op = I.op, w = I.width;
  if (op >= AIWC_OP_COUNT) { snprintf(why, wn, "unknown operation %u", op); return false; }
  if (w < 1 || w > 16 || (scalar_only(op) && w != 1)) { snprintf(why, wn, "width %u not allowed", w); return false; }
  if (I.flags & ~AIWC_INSN_IMM_B) { snprintf(why, wn, "unknown flag bits"); return false; }
  if ((I.flags & AIWC_INSN_IMM_B) && !op_uses_b(op)) { snprintf(why, wn, "immediate operand on an operation without one"); return false; }
  if (I.mode > max_mode(op)) { snprintf(why, wn, "mode %u out of range", I.mode); return false; }
  if (I.id >= d->n_opcode_ids) { snprintf(why, wn, "opcode id %u >= %u", I.id, d->n_opcode_ids); return false; }
  const int need = kind_needed(op);
  const u32 kind = d->opcode_table[I.id].kind;
  if (need >= 0 ? kind != (u32)need
                : (kind != AIWC_KIND_COMPUTE && kind != AIWC_KIND_OTHER)) {
    snprintf(why, wn, "opcode id %u has kind %u, the operation needs %s", I.id, kind,
             need >= 0 ? "its own kind" : "COMPUTE or OTHER");
    return false;
  }
  // register ranges: memory addresses and branch conditions are one register
  const bool vec_a = op != AIWC_OP_LOAD && op != AIWC_OP_STORE && op != AIWC_OP_ATOMIC && op != AIWC_OP_BR;
  const u32 wa = vec_a ? w : 1;
  const bool uses_b = op_uses_b(op) && !(I.flags & AIWC_INSN_IMM_B);
  const bool uses_c = op == AIWC_OP_FMA || op == AIWC_OP_SELECT;
  const bool gep_imm = op == AIWC_OP_GEP && (I.flags & AIWC_INSN_IMM_B);
  if ((op_writes_d(op) && I.d + (op == AIWC_OP_STORE ? 1 : w) > AIWC_NREG) ||
      (op_uses_a(op) && I.a + wa > AIWC_NREG) || (uses_b && !gep_imm && I.b + w > AIWC_NREG) ||
      (uses_c && I.c + w > AIWC_NREG)) {
    snprintf(why, wn, "register range beyond r%u", AIWC_NREG - 1);
    return false;
  }
  if (op_writes_d(op) && vec_a && op != AIWC_OP_MOV) {
    if ((op_uses_a(op) && !same_or_disjoint(I.d, I.a, w)) ||
        (uses_b && !same_or_disjoint(I.d, I.b, w)) || (uses_c && !same_or_disjoint(I.d, I.c, w))) {
      snprintf(why, wn, "destination registers partly overlap an operand's");
      return false;
    }
  }
  if (op == AIWC_OP_MOV && uses_b && !same_or_disjoint(I.d, I.b, w)) {
    snprintf(why, wn, "destination registers partly overlap an operand's");
    return false;
  }
  if (op == AIWC_OP_BR) {
    if (I.site >= d->n_sites) { snprintf(why, wn, "branch site %u >= n_sites %u", I.site, d->n_sites); return false; }
    if (I.imm < 0 || (u64)I.imm >= d->n_insn || I.target2 >= d->n_insn) { snprintf(why, wn, "branch target out of range"); return false; }
  }
  if (op == AIWC_OP_JMP && (I.imm < 0 || (u64)I.imm >= d->n_insn)) { snprintf(why, wn, "jump target out of range"); return false; }
  (void)idx;
  return true;
}

extern "C" aiwc_status aiwc_program_create(aiwc_ctx *ctx, const aiwc_program_desc *d,
                                           aiwc_program **out) {
  if (!ctx || !d || !out) { ctx_error(ctx, "aiwc_program_create: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  if (d->struct_size != sizeof(aiwc_program_desc)) {
    ctx_error(ctx, "aiwc_program_create: struct_size %u != %zu", d->struct_size, sizeof(aiwc_program_desc));
    return AIWC_ERR_INVALID_ARG;
  }
  if (!d->code || d->n_insn == 0 || d->n_insn > (1u << 20)) {
    ctx_error(ctx, "aiwc_program_create: the program needs 1..2^20 instructions");
    return AIWC_ERR_INVALID_ARG;
  }
  if (!d->opcode_table || d->n_opcode_ids == 0 || d->n_opcode_ids > 65536) {
    ctx_error(ctx, "aiwc_program_create: opcode table needs 1..65536 entries");
    return AIWC_ERR_INVALID_ARG;
  }
  if (d->n_sites > 65536) { ctx_error(ctx, "aiwc_program_create: n_sites must be <= 65536"); return AIWC_ERR_INVALID_ARG; }
  for (u32 i = 0; i < d->n_opcode_ids; ++i) {
    const aiwc_opcode_info &e = d->opcode_table[i];
    if (e.op_class == 0xFFFF || e.simd_width == 0 || e.kind > AIWC_KIND_OTHER) {
      ctx_error(ctx, "aiwc_program_create: opcode table entry %u is invalid", i);
      return AIWC_ERR_INVALID_ARG;
    }
  }
  char why[160];
  for (u32 i = 0; i < d->n_insn; ++i) {
    if (!check_insn(d->code[i], i, d, why, sizeof why)) {
      ctx_error(ctx, "aiwc_program_create: instruction %u: %s", i, why);
      return AIWC_ERR_INVALID_ARG;
    }
  }
  HIP_OR_RET(ctx, hipSetDevice(ctx->device));
  aiwc_program *p = new aiwc_program();
  p->ctx = ctx;
  p->n_insn = d->n_insn;
  p->n_sites = d->n_sites;
  p->table.assign(d->opcode_table, d->opcode_table + d->n_opcode_ids);
  if (hipMalloc(&p->dev_code, sizeof(aiwc_insn) * d->n_insn) != hipSuccess) {
    delete p;
    ctx_error(ctx, "aiwc_program_create: out of device memory for the program");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(p->dev_code, d->code, sizeof(aiwc_insn) * d->n_insn, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(p->dev_code);
    delete p;
    ctx_error(ctx, "aiwc_program_create: copying the program failed");
    return AIWC_ERR_HIP;
  }
  *out = p;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_program_destroy(aiwc_program *p) {
  if (!p) return AIWC_OK;
  hipSetDevice(p->ctx->device);
  hipFree(p->dev_code);
  delete p;
  return AIWC_OK;
}

static void free_produced(aiwc_produced *r) {
  hipFree(r->opcode); hipFree(r->wi_off); hipFree(r->addr);
  hipFree(r->mkind); hipFree(r->bsite); hipFree(r->btaken);
  delete r;
}

extern "C" aiwc_status aiwc_produced_destroy(aiwc_produced *r) {
  if (!r) return AIWC_OK;
  hipSetDevice(r->ctx->device);
  free_produced(r);
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_produced_desc(const aiwc_produced *r, aiwc_trace_desc *o) {
  if (!r || !o) { ctx_error(nullptr, "aiwc_produced_desc: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  std::memset(o, 0, sizeof *o);
  o->struct_size = sizeof(aiwc_trace_desc);
  o->n_events = r->n_ev;
  o->opcode = r->opcode;
  o->n_workitems = r->W;
  o->wi_offsets = (const uint64_t *)r->wi_off;
  o->wg_size = r->wg;
  o->n_opcode_ids = (u32)r->table.size();
  o->opcode_table = r->table.data();
  o->n_mem = r->n_mem;
  o->addr = (const uint64_t *)r->addr;
  o->mem_kind = r->mkind;
  o->n_branch = r->n_br;
  o->br_site = r->bsite;
  o->br_taken = r->btaken;
  o->n_sites = r->n_sites ? r->n_sites : 1;
  o->history_len = 16;
  o->max_lsb_skip = 10;
  return AIWC_OK;
}

extern "C" aiwc_status aiwc_produced_to_host(const aiwc_produced *r, uint16_t *opcode,
                                             uint64_t *wi_offsets, uint64_t *addr, uint8_t *mem_kind,
                                             uint32_t *br_site, uint8_t *br_taken) {
  if (!r) { ctx_error(nullptr, "aiwc_produced_to_host: NULL argument"); return AIWC_ERR_INVALID_ARG; }
  aiwc_ctx *ctx = r->ctx;
  HIP_OR_RET(ctx, hipSetDevice(ctx->device));
  const struct { void *dst; const void *src; u64 bytes; } parts[6] = {
      {opcode, r->opcode, 2 * r->n_ev},  {wi_offsets, r->wi_off, 8 * (r->W + 1)},
      {addr, r->addr, 8 * r->n_mem},     {mem_kind, r->mkind, r->n_mem},
      {br_site, r->bsite, 4 * r->n_br},  {br_taken, r->btaken, r->n_br}};
  for (const auto &x : parts)
    if (x.dst && x.bytes) HIP_OR_RET(ctx, hipMemcpy(x.dst, x.src, x.bytes, hipMemcpyDeviceToHost));
  return AIWC_OK;
}

namespace {

// Device allocations of one aiwc_produce call that do not outlive it.
struct Temps {
  std::vector<void *> ptrs;
  ~Temps() { for (void *p : ptrs) hipFree(p); }
  template <class T> bool get(T **out, u64 bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return false;
    ptrs.push_back(p);
    *out = (T *)p;
    return true;
  }
};

const char *error_text(u32 bits) {
  if (bits & E_BOUNDS) return "a memory access left its buffer";
  if (bits & E_ALIGN) return "a memory access was misaligned";
  if (bits & E_STEPS) return "a work-item ran more than max_steps instructions";
  if (bits & E_PC) return "a work-item ran past the end of the program";
  if (bits & E_BARRIER) return "work-items of a work-group waited at a barrier that others never reached";
  return "the counting and recording runs disagree";
}

}  // namespace

extern "C" aiwc_status aiwc_produce(aiwc_program *prog, const aiwc_ndrange *nd,
                                    const aiwc_kernel_arg *args, uint32_t n_args, uint64_t max_steps,
                                    void *stream, aiwc_produced **out) {
  if (!prog || !nd || !out || (n_args && !args)) {
    ctx_error(prog ? prog->ctx : nullptr, "aiwc_produce: NULL argument");
    return AIWC_ERR_INVALID_ARG;
  }
  aiwc_ctx *ctx = prog->ctx;
  if (nd->dims < 1 || nd->dims > 3) { ctx_error(ctx, "aiwc_produce: dims must be 1..3"); return AIWC_ERR_INVALID_ARG; }
  ProdLaunch L;
  std::memset(&L, 0, sizeof L);
  u64 W = 1, groups = 1;
  for (u32 i = 0; i < 3; ++i) {
    const u32 g = i < nd->dims ? nd->global[i] : 1, l = i < nd->dims ? nd->local[i] : 1;
    if (g == 0 || l == 0 || g % l) {
      ctx_error(ctx, "aiwc_produce: dimension %u: global %u is not a positive multiple of local %u", i, g, l);
      return AIWC_ERR_INVALID_ARG;
    }
    L.lsz[i] = l;
    L.ngr[i] = g / l;
    W *= g;
    groups *= g / l;
  }
  const u64 wg = (u64)L.lsz[0] * L.lsz[1] * L.lsz[2];
  if (wg > 1024) { ctx_error(ctx, "aiwc_produce: work-group size %llu > 1024", (unsigned long long)wg); return AIWC_ERR_INVALID_ARG; }
  if (groups > 0x7FFFFFFFull || W > (1ull << 32)) { ctx_error(ctx, "aiwc_produce: ND-range too large"); return AIWC_ERR_INVALID_ARG; }
  if (n_args > AIWC_MAX_KERNEL_ARGS) { ctx_error(ctx, "aiwc_produce: more than %d arguments", AIWC_MAX_KERNEL_ARGS); return AIWC_ERR_INVALID_ARG; }
  if (max_steps == 0) max_steps = 1ull << 20;
  if (max_steps > 0x7FFFFFFFull) { ctx_error(ctx, "aiwc_produce: max_steps must be < 2^31"); return AIWC_ERR_INVALID_ARG; }
  u64 local_bytes = 0, snap_bytes = 0;
  u32 n_buf = 0;
  for (u32 i = 0; i < n_args; ++i) {
    const aiwc_kernel_arg &A = args[i];
    if (A.kind == AIWC_ARG_GLOBAL) {
      if (!A.ptr || A.bytes == 0 || A.bytes > TAG_MASK || ((uintptr_t)A.ptr & 15)) {
        ctx_error(ctx, "aiwc_produce: argument %u: a global buffer needs a 16-byte aligned pointer "
                  "and 1..2^40-1 bytes", i);
        return AIWC_ERR_INVALID_ARG;
      }
      L.args[i] = (u64)(n_buf + 1) << AIWC_ADDR_TAG_SHIFT;
      L.buf_ptr[n_buf] = (u64)(uintptr_t)A.ptr;
      L.buf_bytes[n_buf] = A.bytes;
      snap_bytes += (A.bytes + 255) & ~255ull;
      ++n_buf;
    } else if (A.kind == AIWC_ARG_LOCAL) {
      if (A.bytes == 0) { ctx_error(ctx, "aiwc_produce: argument %u: empty local buffer", i); return AIWC_ERR_INVALID_ARG; }
      local_bytes = (local_bytes + 15) & ~15ull;
      L.args[i] = local_bytes;
      local_bytes += A.bytes;
    } else if (A.kind == AIWC_ARG_SCALAR) {
      L.args[i] = A.value;
    } else {
      ctx_error(ctx, "aiwc_produce: argument %u: unknown kind %u", i, A.kind);
      return AIWC_ERR_INVALID_ARG;
    }
  }
  if (local_bytes > 65536) { ctx_error(ctx, "aiwc_produce: %llu bytes of local memory > 65536", (unsigned long long)local_bytes); return AIWC_ERR_INVALID_ARG; }
  HIP_OR_RET(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  L.code = prog->dev_code;
  L.n_insn = prog->n_insn;
  L.wg = (u32)wg;
  L.local_bytes = (u32)local_bytes;
  L.n_args = n_args;
  L.n_buf = n_buf;
  L.max_steps = max_steps;

  Temps tmp;
  unsigned char *snap = nullptr;
  const u64 nblk = (W + SCAN_BLOCK - 1) / SCAN_BLOCK;
  u64 *bsum = nullptr, *ev_off = nullptr, *mem_off = nullptr, *br_off = nullptr;
  if (!tmp.get(&snap, snap_bytes) || !tmp.get(&L.cnt, 12 * W) || !tmp.get(&L.err, 16) ||
      !tmp.get(&bsum, 24 * nblk) || !tmp.get(&mem_off, 8 * (W + 1)) || !tmp.get(&br_off, 8 * (W + 1))) {
    ctx_error(ctx, "aiwc_produce: out of device memory for the buffer copy and counts");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  auto copy_buffers = [&](bool to_snap) -> hipError_t {
    u64 o = 0;
    for (u32 j = 0; j < n_buf; ++j) {
      void *buf = (void *)(uintptr_t)L.buf_ptr[j];
      hipError_t e = to_snap ? hipMemcpyAsync(snap + o, buf, L.buf_bytes[j], hipMemcpyDeviceToDevice, s)
                             : hipMemcpyAsync(buf, snap + o, L.buf_bytes[j], hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      o += (L.buf_bytes[j] + 255) & ~255ull;
    }
    return hipSuccess;
  };
  const u32 err_init[4] = {0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu};
  const u64 lds_count = (local_bytes + 15) & ~15ull, lds_rec = lds_count + 8 * wg;
  HIP_OR_RET(ctx, hipFuncSetAttribute((const void *)k_interp<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024));
  HIP_OR_RET(ctx, hipFuncSetAttribute((const void *)k_interp<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024));
  auto read_err = [&](u32 e[4]) -> hipError_t {
    hipError_t x = hipMemcpyAsync(e, L.err, 16, hipMemcpyDeviceToHost, s);
    if (x == hipSuccess) x = hipStreamSynchronize(s);
    return x;
  };
  auto fail = [&](const u32 e[4], aiwc_status st) {
    const u64 at = ((u64)e[3] << 32) | e[2];
    ctx_error(ctx, "aiwc_produce: %s (work-item %llu, instruction %llu)", error_text(e[0]),
              (unsigned long long)(at >> 20), (unsigned long long)(at & 0xFFFFF));
    copy_buffers(false);   // leave the buffers as they were before the call
    hipStreamSynchronize(s);
    return st;
  };

  // counting run
  HIP_OR_RET(ctx, copy_buffers(true));
  HIP_OR_RET(ctx, hipMemcpyAsync(L.err, err_init, 16, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_interp<false>, dim3((u32)groups), dim3((u32)wg), lds_count, s, L);
  HIP_OR_RET(ctx, hipGetLastError());
  u32 e[4];
  HIP_OR_RET(ctx, read_err(e));
  if (e[0]) return fail(e, AIWC_ERR_INVALID_ARG);

  // offsets: block sums on the device, their scan on the host, then in-block scans
  hipLaunchKernelGGL(k_count_sums, dim3((u32)nblk), dim3(SCAN_BLOCK), 0, s, L.cnt, W, bsum);
  HIP_OR_RET(ctx, hipGetLastError());
  std::vector<u64> hb(3 * nblk);
  HIP_OR_RET(ctx, hipMemcpyAsync(hb.data(), bsum, 24 * nblk, hipMemcpyDeviceToHost, s));
  HIP_OR_RET(ctx, hipStreamSynchronize(s));
  u64 tot[3] = {0, 0, 0};
  for (u64 b = 0; b < nblk; ++b)
    for (u32 j = 0; j < 3; ++j) { const u64 v = hb[3 * b + j]; hb[3 * b + j] = tot[j]; tot[j] += v; }

  aiwc_produced *r = new aiwc_produced();
  r->ctx = ctx;
  r->table = prog->table;
  r->n_sites = prog->n_sites;
  r->wg = (u32)wg;
  r->W = W;
  r->n_ev = tot[0];
  r->n_mem = tot[1];
  r->n_br = tot[2];
  u32 *ssite = nullptr;
  u8 *staken = nullptr;
  if (hipMalloc(&r->opcode, 2 * tot[0] + 16) != hipSuccess || hipMalloc(&r->wi_off, 8 * (W + 1)) != hipSuccess ||
      hipMalloc(&r->addr, 8 * tot[1] + 16) != hipSuccess || hipMalloc(&r->mkind, tot[1] + 16) != hipSuccess ||
      hipMalloc(&r->bsite, 4 * tot[2] + 16) != hipSuccess || hipMalloc(&r->btaken, tot[2] + 16) != hipSuccess ||
      !tmp.get(&ssite, 4 * tot[2]) || !tmp.get(&staken, tot[2])) {
    free_produced(r);
    ctx_error(ctx, "aiwc_produce: out of device memory for a trace of %llu events",
              (unsigned long long)tot[0]);
    copy_buffers(false);
    hipStreamSynchronize(s);
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  ev_off = r->wi_off;
  hipError_t he = hipMemcpyAsync(bsum, hb.data(), 24 * nblk, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) {
    hipLaunchKernelGGL(k_offsets, dim3((u32)nblk), dim3(SCAN_BLOCK), 0, s, L.cnt, W, bsum, ev_off,
                       mem_off, br_off);
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = hipMemcpyAsync(ev_off + W, &tot[0], 8, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(mem_off + W, &tot[1], 8, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(br_off + W, &tot[2], 8, hipMemcpyHostToDevice, s);

  // recording run, from the buffers as they were
  if (he == hipSuccess) he = copy_buffers(false);
  if (he == hipSuccess) he = hipMemcpyAsync(L.err, err_init, 16, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) {
    L.ev_off = ev_off; L.mem_off = mem_off; L.br_off = br_off;
    L.opcode = r->opcode; L.addr = r->addr; L.mkind = r->mkind;
    L.bsite = r->bsite; L.btaken = r->btaken; L.ssite = ssite; L.staken = staken;
    hipLaunchKernelGGL(k_interp<true>, dim3((u32)groups), dim3((u32)wg), lds_rec, s, L);
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = read_err(e);
  if (he != hipSuccess) {
    free_produced(r);
    ctx_error(ctx, "aiwc_produce: %s", hipGetErrorString(he));
    return AIWC_ERR_HIP;
  }
  if (e[0]) {
    free_produced(r);
    return fail(e, (e[0] & E_SCHED) && !(e[0] & ~E_SCHED) ? AIWC_ERR_UNSUPPORTED : AIWC_ERR_INVALID_ARG);
  }
  *out = r;
  return AIWC_OK;
}
