/*
 * producer.c -- CPU oracle of the trace producer.  TEST INFRASTRUCTURE ONLY:
 * the tests, the smoke check and the benchmark's CPU leg may call it; the
 * product never does.
 *
 * It runs a kernel program the way the paper's simulator runs an OpenCL
 * kernel (Implementation section): work-groups one after another; inside a
 * work-group, each work-item in turn runs until it reaches a barrier or
 * returns, and once every work-item waits at the barrier they all continue.
 * Each executed instruction appends its opcode id to its work-item's
 * stream; loads and stores append one memory event, atomics a read and a
 * write event (the memoryLoad / memoryStore / memoryAtomicLoad /
 * memoryAtomicStore notifications); a conditional branch appends its site and
 * whether its condition held.  Memory and branch events are kept in the order
 * they happen; each memory event also keeps its work-item, so that a test
 * can compare per work-item sequences with a producer that orders memory
 * events differently (their order does not change any metric).
 *
 * The instruction record and its operations are the producer's input
 * format: 24 bytes, fields in this order -- op, mode, width, flags, d, a, b,
 * c (one byte each), id, site (two bytes each), target2 (four), imm (eight,
 * signed).  Operation numbers and semantics are restated below from that
 * format's definition; no code is shared with the GPU producer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint8_t op, mode, width, flags, d, a, b, c;
  uint16_t id, site;
  uint32_t target2;
  int64_t imm;
} pinsn;

typedef struct {
  uint32_t kind; /* 0 global buffer, 1 local bytes, 2 scalar */
  uint32_t pad;
  void *host;
  uint64_t bytes;
  uint64_t value;
} parg;

typedef struct {
  uint64_t n_events, n_wi, n_mem, n_branch;
  uint16_t *opcode;
  uint64_t *wi_offsets;
  uint64_t *addr;
  uint8_t *mem_kind;
  uint64_t *mem_wi;
  uint32_t *br_site;
  uint8_t *br_taken;
  uint32_t error;  /* 0 ok; else one of the PERR_* codes */
  uint64_t error_wi;
} pout;

enum { PERR_BOUNDS = 1, PERR_ALIGN = 2, PERR_STEPS = 4, PERR_BARRIER = 8, PERR_PC = 16,
       PERR_PROGRAM = 64 /* a register range or jump target outside the machine */ };

/* operation numbers of the input format */
enum {
  RET, MOV, ADD, SUB, MUL, SDIV, SREM, UDIV, UREM, SHL, LSHR, ASHR, AND, OR, XOR, ICMP,
  FADD, FSUB, FMUL, FDIV, FCMP, FMA, FSQRT, FMIN, FMAX, SITOFP, FPTOSI, SEXT, ZEXT, SELECT,
  GEP, LOAD, STORE, ATOMIC, BR, JMP, BARRIER, BUILTIN
};

#define NREG 64
#define TAG_SHIFT 40

/* growable arrays */
typedef struct { void *p; size_t n, cap, esz; } vec;
static int vpush(vec *v, const void *x) {
  if (v->n == v->cap) {
    size_t nc = v->cap ? 2 * v->cap : 1024;
    void *q = realloc(v->p, nc * v->esz);
    if (!q) return 0;
    v->p = q;
    v->cap = nc;
  }
  memcpy((char *)v->p + v->n * v->esz, x, v->esz);
  v->n++;
  return 1;
}

static float f_of(uint64_t r) { uint32_t u = (uint32_t)r; float f; memcpy(&f, &u, 4); return f; }
static uint64_t bits_of(float f) {
  uint32_t u;
  if (isnan(f)) return 0x7FC00000u;
  memcpy(&u, &f, 4);
  return u;
}

typedef struct {
  uint64_t R[NREG];
  uint32_t pc;
  int state;  /* 0 running, 1 at a barrier, 2 finished */
  uint64_t steps;
  vec ops;    /* this work-item's opcode ids */
} witem;

typedef struct {
  const pinsn *code;
  uint32_t n_insn;
  uint32_t lsize[3], ngroups[3];
  parg *args;
  uint32_t n_args;
  void *gbuf[64];
  uint64_t gbytes[64];
  uint32_t n_gbuf;
  uint8_t *lmem;
  uint64_t lbytes;
  uint64_t max_steps;
  vec mem_addr, mem_kind, mem_wi, br_site, br_taken;
  uint32_t error;
  uint64_t error_wi;
} machine;

/* host address of an access, or NULL after recording the error */
static uint8_t *where(machine *M, uint64_t va, uint64_t size, uint64_t elt, int *is_local, uint64_t wi) {
  uint64_t tag = va >> TAG_SHIFT, off = va & ((1ull << TAG_SHIFT) - 1);
  if (off % elt != 0) { M->error = PERR_ALIGN; M->error_wi = wi; return NULL; }
  if (tag == 0) {
    *is_local = 1;
    if (off + size > M->lbytes) { M->error = PERR_BOUNDS; M->error_wi = wi; return NULL; }
    return M->lmem + off;
  }
  *is_local = 0;
  if (tag - 1 >= M->n_gbuf || off + size > M->gbytes[tag - 1]) {
    M->error = PERR_BOUNDS;
    M->error_wi = wi;
    return NULL;
  }
  return (uint8_t *)M->gbuf[tag - 1] + off;
}

static int add_mem(machine *M, uint64_t va, uint8_t kind, uint64_t wi) {
  return vpush(&M->mem_addr, &va) && vpush(&M->mem_kind, &kind) && vpush(&M->mem_wi, &wi);
}

/* signed 64-bit view */
static int64_t S(uint64_t x) { return (int64_t)x; }

static uint64_t integer_op(int op, uint64_t x, uint64_t y) {
  unsigned sh = (unsigned)(y % 64);
  if (op == ADD) return x + y;
  if (op == SUB) return x - y;
  if (op == MUL) return x * y;
  if (op == SDIV) {
    if (y == 0) return 0;
    if (S(x) == INT64_MIN && S(y) == -1) return (uint64_t)INT64_MIN;
    return (uint64_t)(S(x) / S(y));
  }
  if (op == SREM) {
    if (y == 0 || S(y) == -1) return 0;
    return (uint64_t)(S(x) % S(y));
  }
  if (op == UDIV) return y == 0 ? 0 : x / y;
  if (op == UREM) return y == 0 ? 0 : x % y;
  if (op == SHL) return x << sh;
  if (op == LSHR) return x >> sh;
  if (op == ASHR) return (uint64_t)(S(x) >> sh);
  if (op == AND) return x & y;
  if (op == OR) return x | y;
  return x ^ y;
}

static uint64_t int_compare(int pred, uint64_t x, uint64_t y) {
  switch (pred) {
    case 0: return x == y;
    case 1: return x != y;
    case 2: return S(x) < S(y);
    case 3: return S(x) <= S(y);
    case 4: return S(x) > S(y);
    case 5: return S(x) >= S(y);
    case 6: return x < y;
    case 7: return x <= y;
    case 8: return x > y;
    default: return x >= y;
  }
}

static uint64_t float_compare(int pred, float x, float y) {
  if (isnan(x) || isnan(y)) return pred == 1;  /* only "unordered or not equal" holds */
  switch (pred) {
    case 0: return x == y;
    case 1: return x != y;
    case 2: return x < y;
    case 3: return x <= y;
    case 4: return x > y;
    default: return x >= y;
  }
}

/* fmin / fmax with NaN -> the other operand and -0 below +0 */
static float min_or_max(float x, float y, int want_max) {
  if (isnan(x)) return y;
  if (isnan(y)) return x;
  if (x == y) {
    int xn = signbit(x) != 0, yn = signbit(y) != 0;
    if (xn == yn) return x;
    /* one is -0, the other +0 */
    return want_max ? (xn ? y : x) : (xn ? x : y);
  }
  if (want_max) return x > y ? x : y;
  return x < y ? x : y;
}

static uint64_t float_to_int32(float x) {
  int32_t r;
  if (isnan(x)) r = 0;
  else if (x >= 2147483648.0f) r = INT32_MAX;
  else if (x < -2147483648.0f) r = INT32_MIN;
  else r = (int32_t)truncf(x);
  return (uint64_t)(int64_t)r;
}

static uint64_t work_item_function(const machine *M, int mode, const uint32_t lid[3], const uint32_t grp[3]) {
  int dim = mode % 3;
  switch (mode / 3) {
    case 0: return (uint64_t)grp[dim] * M->lsize[dim] + lid[dim];   /* get_global_id  */
    case 1: return lid[dim];                                         /* get_local_id   */
    case 2: return grp[dim];                                         /* get_group_id   */
    case 3: return (uint64_t)M->lsize[dim] * M->ngroups[dim];        /* get_global_size*/
    case 4: return M->lsize[dim];                                    /* get_local_size */
    default: return M->ngroups[dim];                                 /* get_num_groups */
  }
}

/* Run one work-item until it waits at a barrier, returns or fails. */
static int run_item(machine *M, witem *W, uint64_t wi, const uint32_t lid[3], const uint32_t grp[3]) {
  while (W->state == 0) {
    if (W->pc >= M->n_insn) { M->error = PERR_PC; M->error_wi = wi; return 0; }
    if (W->steps == M->max_steps) { M->error = PERR_STEPS; M->error_wi = wi; return 0; }
    W->steps++;
    const pinsn *I = &M->code[W->pc];
    uint16_t id = I->id;
    if (!vpush(&W->ops, &id)) return 0;
    uint32_t next = W->pc + 1;
    int n = I->width;
    int immb = I->flags & 1;
    uint64_t *R = W->R;
    /* operand b of element i */
#define OPB(i) (immb ? (uint64_t)I->imm : R[I->b + (i)])
    switch (I->op) {
      case RET:
        W->state = 2;
        break;
      case MOV:
        for (int i = 0; i < n; i++) R[I->d + i] = OPB(i);
        break;
      case ADD: case SUB: case MUL: case SDIV: case SREM: case UDIV: case UREM:
      case SHL: case LSHR: case ASHR: case AND: case OR: case XOR:
        for (int i = 0; i < n; i++) R[I->d + i] = integer_op(I->op, R[I->a + i], OPB(i));
        break;
      case ICMP:
        for (int i = 0; i < n; i++) R[I->d + i] = int_compare(I->mode, R[I->a + i], OPB(i));
        break;
      case FADD:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of(f_of(R[I->a + i]) + f_of(OPB(i)));
        break;
      case FSUB:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of(f_of(R[I->a + i]) - f_of(OPB(i)));
        break;
      case FMUL:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of(f_of(R[I->a + i]) * f_of(OPB(i)));
        break;
      case FDIV:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of(f_of(R[I->a + i]) / f_of(OPB(i)));
        break;
      case FCMP:
        for (int i = 0; i < n; i++) R[I->d + i] = float_compare(I->mode, f_of(R[I->a + i]), f_of(OPB(i)));
        break;
      case FMA:
        for (int i = 0; i < n; i++)
          R[I->d + i] = bits_of(fmaf(f_of(R[I->a + i]), f_of(OPB(i)), f_of(R[I->c + i])));
        break;
      case FSQRT:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of(sqrtf(f_of(R[I->a + i])));
        break;
      case FMIN: case FMAX:
        for (int i = 0; i < n; i++)
          R[I->d + i] = bits_of(min_or_max(f_of(R[I->a + i]), f_of(OPB(i)), I->op == FMAX));
        break;
      case SITOFP:
        for (int i = 0; i < n; i++) R[I->d + i] = bits_of((float)(int32_t)(uint32_t)R[I->a + i]);
        break;
      case FPTOSI:
        for (int i = 0; i < n; i++) R[I->d + i] = float_to_int32(f_of(R[I->a + i]));
        break;
      case SEXT:
        for (int i = 0; i < n; i++) R[I->d + i] = (uint64_t)(int64_t)(int32_t)(uint32_t)R[I->a + i];
        break;
      case ZEXT:
        for (int i = 0; i < n; i++) R[I->d + i] = R[I->a + i] & 0xFFFFFFFFull;
        break;
      case SELECT:
        for (int i = 0; i < n; i++) R[I->d + i] = R[I->a + i] != 0 ? OPB(i) : R[I->c + i];
        break;
      case GEP:
        for (int i = 0; i < n; i++)
          R[I->d + i] = immb ? R[I->a + i] + (uint64_t)I->imm : R[I->a + i] + R[I->b + i] * (uint64_t)I->imm;
        break;
      case LOAD: {
        uint64_t va = R[I->a];
        uint64_t elt = I->mode == 2 ? 8 : 4;
        int loc;
        uint8_t *p = where(M, va, elt * n, elt, &loc, wi);
        if (!p) return 0;
        uint64_t vals[16];
        for (int i = 0; i < n; i++) {
          if (elt == 8) {
            memcpy(&vals[i], p + 8 * i, 8);
          } else {
            uint32_t x;
            memcpy(&x, p + 4 * i, 4);
            vals[i] = I->mode == 0 ? (uint64_t)(int64_t)(int32_t)x : (uint64_t)x;
          }
        }
        for (int i = 0; i < n; i++) R[I->d + i] = vals[i];
        if (!add_mem(M, va, (uint8_t)(loc ? 2 : 0), wi)) return 0;
        break;
      }
      case STORE: {
        uint64_t va = R[I->a];
        uint64_t elt = I->mode == 1 ? 8 : 4;
        int loc;
        uint8_t *p = where(M, va, elt * n, elt, &loc, wi);
        if (!p) return 0;
        for (int i = 0; i < n; i++) {
          uint64_t v = OPB(i);
          if (elt == 8) memcpy(p + 8 * i, &v, 8);
          else { uint32_t x = (uint32_t)v; memcpy(p + 4 * i, &x, 4); }
        }
        if (!add_mem(M, va, (uint8_t)(1 | (loc ? 2 : 0)), wi)) return 0;
        break;
      }
      case ATOMIC: {
        uint64_t va = R[I->a];
        int loc;
        uint8_t *p = where(M, va, 4, 4, &loc, wi);
        if (!p) return 0;
        uint32_t old, v = (uint32_t)OPB(0), nv;
        memcpy(&old, p, 4);
        switch (I->mode) {
          case 0: nv = old + v; break;
          case 1: nv = old - v; break;
          case 2: nv = old & v; break;
          case 3: nv = old | v; break;
          case 4: nv = old ^ v; break;
          case 5: nv = (int32_t)old < (int32_t)v ? old : v; break;
          case 6: nv = (int32_t)old > (int32_t)v ? old : v; break;
          case 7: nv = old < v ? old : v; break;
          default: nv = old > v ? old : v; break;
        }
        memcpy(p, &nv, 4);
        R[I->d] = (uint64_t)(int64_t)(int32_t)old;
        if (!add_mem(M, va, (uint8_t)(loc ? 2 : 0), wi)) return 0;          /* the read  */
        if (!add_mem(M, va, (uint8_t)(1 | (loc ? 2 : 0)), wi)) return 0;    /* the write */
        break;
      }
      case BR: {
        uint8_t taken = R[I->a] != 0;
        uint32_t site = I->site;
        if (!vpush(&M->br_site, &site) || !vpush(&M->br_taken, &taken)) return 0;
        next = taken ? (uint32_t)I->imm : I->target2;
        break;
      }
      case JMP:
        next = (uint32_t)I->imm;
        break;
      case BARRIER:
        W->state = 1;
        break;
      case BUILTIN:
        R[I->d] = work_item_function(M, I->mode, lid, grp);
        break;
      default:
        M->error = PERR_PC;
        M->error_wi = wi;
        return 0;
    }
#undef OPB
    W->pc = next;
  }
  return 1;
}

void orc_produce_free(pout *o) {
  free(o->opcode); free(o->wi_offsets); free(o->addr); free(o->mem_kind);
  free(o->mem_wi); free(o->br_site); free(o->br_taken);
  memset(o, 0, sizeof *o);
}

/* Returns 0 on success (out filled), -1 when memory ran out; a kernel that
 * fails (out of bounds, misaligned, step limit, barrier mismatch, running
 * off the program) returns 0 with out->error set and no arrays. */
int orc_produce(const pinsn *code, uint32_t n_insn, uint32_t dims, const uint32_t *global,
                const uint32_t *local, parg *args, uint32_t n_args, uint64_t max_steps, pout *out) {
  memset(out, 0, sizeof *out);
  for (uint32_t i = 0; i < n_insn; i++) {
    const pinsn *I = &code[i];
    int w = I->width;
    if (w < 1 || w > 16 || I->d + w > NREG || I->a + w > NREG || I->b + w > NREG || I->c + w > NREG ||
        ((I->op == BR || I->op == JMP) && (I->imm < 0 || (uint64_t)I->imm >= n_insn)) ||
        (I->op == BR && I->target2 >= n_insn)) {
      out->error = PERR_PROGRAM;
      return 0;
    }
  }
  machine M;
  memset(&M, 0, sizeof M);
  M.code = code;
  M.n_insn = n_insn;
  M.args = args;
  M.n_args = n_args;
  M.max_steps = max_steps ? max_steps : (1ull << 20);
  M.mem_addr.esz = 8; M.mem_kind.esz = 1; M.mem_wi.esz = 8; M.br_site.esz = 4; M.br_taken.esz = 1;
  uint64_t n_groups = 1, wg = 1;
  for (int i = 0; i < 3; i++) {
    uint32_t g = i < (int)dims ? global[i] : 1, l = i < (int)dims ? local[i] : 1;
    M.lsize[i] = l;
    M.ngroups[i] = g / l;
    n_groups *= g / l;
    wg *= l;
  }
  /* argument registers and memory */
  uint64_t argreg[64];
  uint64_t loff = 0;
  for (uint32_t i = 0; i < n_args; i++) {
    if (args[i].kind == 0) {
      M.gbuf[M.n_gbuf] = args[i].host;
      M.gbytes[M.n_gbuf] = args[i].bytes;
      argreg[i] = (uint64_t)(M.n_gbuf + 1) << TAG_SHIFT;
      M.n_gbuf++;
    } else if (args[i].kind == 1) {
      loff = (loff + 15) / 16 * 16;
      argreg[i] = loff;
      loff += args[i].bytes;
    } else {
      argreg[i] = args[i].value;
    }
  }
  M.lbytes = loff;
  M.lmem = (uint8_t *)malloc(loff ? loff : 1);
  witem *items = (witem *)calloc(wg, sizeof(witem));
  vec ops_all = {0}, offs = {0};
  ops_all.esz = 2;
  offs.esz = 8;
  int ok = M.lmem && items;
  uint64_t zero = 0;
  ok = ok && vpush(&offs, &zero);
  for (uint64_t g = 0; ok && g < n_groups && !M.error; g++) {
    uint32_t grp[3] = {(uint32_t)(g % M.ngroups[0]), (uint32_t)((g / M.ngroups[0]) % M.ngroups[1]),
                       (uint32_t)(g / ((uint64_t)M.ngroups[0] * M.ngroups[1]))};
    memset(M.lmem, 0, loff ? loff : 1);
    for (uint64_t l = 0; l < wg; l++) {
      witem *W = &items[l];
      memset(W->R, 0, sizeof W->R);
      for (uint32_t i = 0; i < n_args; i++) W->R[i] = argreg[i];
      W->pc = 0;
      W->state = 0;
      W->steps = 0;
      W->ops.n = 0;
      W->ops.esz = 2;
    }
    for (;;) {
      /* every work-item in turn, until it waits or ends */
      for (uint64_t l = 0; ok && l < wg && !M.error; l++) {
        uint32_t lid[3] = {(uint32_t)(l % M.lsize[0]), (uint32_t)((l / M.lsize[0]) % M.lsize[1]),
                           (uint32_t)(l / ((uint64_t)M.lsize[0] * M.lsize[1]))};
        if (items[l].state == 0 && !run_item(&M, &items[l], g * wg + l, lid, grp) && !M.error) ok = 0;
      }
      if (!ok || M.error) break;
      uint64_t waiting = 0;
      for (uint64_t l = 0; l < wg; l++) waiting += items[l].state == 1;
      if (waiting == 0) break;
      if (waiting != wg) {
        M.error = PERR_BARRIER;
        for (uint64_t l = 0; l < wg; l++)
          if (items[l].state == 1) { M.error_wi = g * wg + l; break; }
        break;
      }
      for (uint64_t l = 0; l < wg; l++) items[l].state = 0;   /* the barrier clears */
    }
    /* the work-group's opcode streams, work-item major */
    for (uint64_t l = 0; ok && !M.error && l < wg; l++) {
      for (size_t k = 0; k < items[l].ops.n && ok; k++) ok = vpush(&ops_all, (uint16_t *)items[l].ops.p + k);
      uint64_t end = ops_all.n;
      ok = ok && vpush(&offs, &end);
    }
  }
  for (uint64_t l = 0; items && l < wg; l++) free(items[l].ops.p);
  free(items);
  free(M.lmem);
  if (!ok || M.error) {
    free(ops_all.p); free(offs.p);
    free(M.mem_addr.p); free(M.mem_kind.p); free(M.mem_wi.p); free(M.br_site.p); free(M.br_taken.p);
    out->error = M.error;
    out->error_wi = M.error_wi;
    return ok || M.error ? 0 : -1;
  }
  out->n_events = ops_all.n;
  out->n_wi = n_groups * wg;
  out->n_mem = M.mem_addr.n;
  out->n_branch = M.br_site.n;
  out->opcode = (uint16_t *)ops_all.p;
  out->wi_offsets = (uint64_t *)offs.p;
  out->addr = (uint64_t *)M.mem_addr.p;
  out->mem_kind = (uint8_t *)M.mem_kind.p;
  out->mem_wi = (uint64_t *)M.mem_wi.p;
  out->br_site = (uint32_t *)M.br_site.p;
  out->br_taken = (uint8_t *)M.br_taken.p;
  return 0;
}
