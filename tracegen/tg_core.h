/*
 * tg_core.h -- the synthetic trace recipe, shared by the host generator
 * (tg_host.c) and the device generator (tg_dev.hip).
 *
 * This module only *produces inputs*: it holds none of the characterization
 * arithmetic.  Everything here is integer-only (splitmix64 counter-based
 * hashing plus integer tables computed once by the caller), so the host and
 * the device produce byte-identical traces.
 *
 * The includer must define TG_FN (e.g. "static inline" on the host,
 * "__device__ static inline" in HIP code) before including this file.
 *
 * Event recipe for work-item w at 1-based position p of its L_w events:
 *   p == L_w                      -> RET       (kind OTHER)
 *   period > 0 and p % period == 0 -> BARRIER
 *   else u = hash32(kind stream):  u < p_mem            -> LOAD or STORE, or
 *                                                          ATOMIC_RMW with
 *                                                          probability p_atomic
 *                                  u < p_mem + p_branch -> BRANCH_COND
 *                                  else                 -> compute id (Zipf CDF)
 * An ATOMIC_RMW instruction issues two memory events at one address: a read,
 * then a write.
 * Memory and branch events are emitted in the simulator's schedule order:
 * work-group by work-group, barrier phase by phase, work-item by work-item.
 */
#ifndef TG_CORE_H
#define TG_CORE_H

#include <stdint.h>

#ifndef TG_FN
#error "define TG_FN before including tg_core.h"
#endif

enum { TG_S_LEN = 1, TG_S_KIND = 2, TG_S_VAL = 3, TG_S_ADDR = 4, TG_S_ATOM = 5 };
enum { TG_EV_COMPUTE = 0, TG_EV_MEM = 1, TG_EV_BRANCH = 2, TG_EV_BARRIER = 3,
       TG_EV_RET = 4 };

typedef struct tg_params {
  uint64_t seed;
  uint64_t n_wi;
  uint32_t wg_size;
  uint32_t len_min, len_max;
  uint32_t barrier_period;       /* 0 = no explicit barriers                */
  uint32_t p_mem_q32;            /* probabilities scaled by 2^32            */
  uint32_t p_branch_q32;
  uint32_t p_store_q32;
  uint32_t p_local_q32;
  uint32_t t_sweep_q32;          /* global pattern: u < t_sweep -> sweep,    */
  uint32_t t_stencil_q32;        /*   u < t_stencil -> stencil, else random  */
  uint64_t sweep_base, sweep_stride, sweep_words;
  uint64_t stencil_base;
  uint64_t stencil_dim;          /* grid side G (4-byte elements), >= 3     */
  uint64_t random_base, random_words;
  uint64_t local_words;
  uint32_t n_compute_ids;        /* compute ids are 0 .. n_compute_ids-1    */
  uint32_t id_load, id_store, id_branch, id_barrier, id_ret;
  uint32_t n_sites;
  uint32_t n_phases;             /* (len_max - 1) / period + 1, or 1        */
  uint32_t p_atomic_q32;         /* share of memory instructions that are
                                    atomic read-modify-writes               */
  uint32_t id_atomic;
} tg_params;

TG_FN uint64_t tg_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

TG_FN uint64_t tg_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return tg_mix(tg_mix(tg_mix(seed ^ (stream * 0xD1B54A32D192ED03ull)) ^ a) ^ b);
}

TG_FN uint32_t tg_len(const tg_params *P, uint64_t w) {
  uint64_t span = (uint64_t)(P->len_max - P->len_min) + 1u;
  return P->len_min + (uint32_t)(tg_hash(P->seed, TG_S_LEN, w, 0) % span);
}

TG_FN uint32_t tg_phase(const tg_params *P, uint32_t p) {
  return P->barrier_period ? (p - 1u) / P->barrier_period : 0u;
}

/* slot of (work-item, phase) in schedule order */
TG_FN uint64_t tg_sched_slot(const tg_params *P, uint64_t w, uint32_t phase) {
  uint64_t g = w / P->wg_size;
  return (g * P->n_phases + phase) * P->wg_size + (w - g * P->wg_size);
}

TG_FN int tg_event_type(const tg_params *P, uint64_t w, uint32_t p, uint32_t L) {
  if (p == L) return TG_EV_RET;
  if (P->barrier_period && (p % P->barrier_period) == 0u) return TG_EV_BARRIER;
  uint32_t u = (uint32_t)tg_hash(P->seed, TG_S_KIND, w, p);
  if (u < P->p_mem_q32) return TG_EV_MEM;
  if ((uint64_t)u < (uint64_t)P->p_mem_q32 + P->p_branch_q32) return TG_EV_BRANCH;
  return TG_EV_COMPUTE;
}

/* Whether the memory instruction at (w, p) is an atomic read-modify-write
 * (two memory events); never drawn when p_atomic is 0, so traces without
 * atomics do not depend on this stream.                                     */
TG_FN int tg_is_atomic(const tg_params *P, uint64_t w, uint32_t p) {
  return P->p_atomic_q32 != 0u &&
         (uint32_t)tg_hash(P->seed, TG_S_ATOM, w, p) < P->p_atomic_q32;
}

TG_FN uint32_t tg_compute_id(const tg_params *P, const uint32_t *zipf_cdf,
                             uint64_t w, uint32_t p) {
  uint32_t u = (uint32_t)(tg_hash(P->seed, TG_S_VAL, w, p) >> 32);
  uint32_t i = 0;
  while (i + 1u < P->n_compute_ids && u >= zipf_cdf[i]) ++i;
  return i;
}

/* Memory event: returns the address, writes the mem_kind bits.  jsw / jst
 * are the work-item's running counters of sweep and stencil events; they are
 * advanced when used.                                                       */
TG_FN uint64_t tg_mem_event(const tg_params *P, uint64_t w, uint32_t p,
                            uint32_t *jsw, uint32_t *jst, uint8_t *kind) {
  uint64_t r = tg_hash(P->seed, TG_S_VAL, w, p);
  uint64_t r2 = tg_hash(P->seed, TG_S_ADDR, w, p);
  uint8_t k = ((uint32_t)r < P->p_store_q32) ? 1u : 0u;
  if ((uint32_t)(r >> 32) < P->p_local_q32) {
    *kind = (uint8_t)(k | 2u);
    return 4ull * (r2 % P->local_words);
  }
  *kind = k;
  uint32_t u = (uint32_t)(r2 >> 32);
  if (u < P->t_sweep_q32) {
    uint64_t j = (*jsw)++;
    return P->sweep_base + ((j * P->n_wi + w) % P->sweep_words) * P->sweep_stride;
  }
  if (u < P->t_stencil_q32) {
    uint64_t j = (*jst)++;
    uint64_t inner = P->stencil_dim - 2u;
    uint64_t q = ((j / 5u) * P->n_wi + w) % (inner * inner);
    uint64_t row = 1u + q / inner, col = 1u + q % inner;
    switch ((uint32_t)(j % 5u)) {
      case 1: row -= 1u; break;
      case 2: row += 1u; break;
      case 3: col += 1u; break;
      case 4: col -= 1u; break;
      default: break;
    }
    return P->stencil_base + 4ull * (row * P->stencil_dim + col);
  }
  return P->random_base + 4ull * ((uint32_t)r2 % P->random_words);
}

TG_FN void tg_branch_event(const tg_params *P, const uint32_t *site_thr,
                           uint64_t w, uint32_t p, uint32_t *site,
                           uint8_t *taken) {
  uint64_t r = tg_hash(P->seed, TG_S_VAL, w, p);
  uint32_t s = (uint32_t)((r >> 32) % P->n_sites);
  *site = s;
  *taken = ((uint32_t)r < site_thr[s]) ? 1u : 0u;
}

#endif /* TG_CORE_H */
