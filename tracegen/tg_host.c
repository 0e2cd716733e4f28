/*
 * tg_host.c -- host (CPU) generator for the synthetic traces of tg_core.h.
 *
 * Two calls: tg_host_plan() draws every work-item's length and counts its
 * memory and branch events per barrier phase, then lays the streams out in
 * schedule order; tg_host_fill() writes the arrays.  Both run on `threads`
 * POSIX threads over disjoint work-item ranges, so the bytes do not depend
 * on the thread count.
 */
#define TG_FN static inline
#include "tg_core.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct tg_plan {
  tg_params P;
  uint32_t *zipf_cdf;   /* owned copies of the tables */
  uint32_t *site_thr;
  uint64_t *wi_off;     /* [n_wi + 1] */
  uint64_t *mem_off;    /* [slots]: schedule-order offsets */
  uint64_t *br_off;
  uint64_t slots;
  uint64_t n_events, n_mem, n_branch;
} tg_plan;

typedef struct {
  tg_plan *pl;
  uint64_t w0, w1;
  int stage; /* 0 = lengths, 1 = counts, 2 = fill */
  uint16_t *opcode; uint64_t *addr; uint8_t *kind; uint32_t *site; uint8_t *taken;
} tg_job;

static void walk_count(tg_plan *pl, uint64_t w) {
  const tg_params *P = &pl->P;
  uint32_t L = (uint32_t)(pl->wi_off[w + 1] - pl->wi_off[w]);
  for (uint32_t p = 1; p <= L; ++p) {
    int t = tg_event_type(P, w, p, L);
    uint64_t s = tg_sched_slot(P, w, tg_phase(P, p));
    if (t == TG_EV_MEM) pl->mem_off[s] += tg_is_atomic(P, w, p) ? 2u : 1u;
    else if (t == TG_EV_BRANCH) pl->br_off[s]++;
  }
}

static void walk_fill(tg_plan *pl, uint64_t w, tg_job *j) {
  const tg_params *P = &pl->P;
  uint64_t base = pl->wi_off[w];
  uint32_t L = (uint32_t)(pl->wi_off[w + 1] - base);
  uint32_t jsw = 0, jst = 0;
  uint32_t cur_phase = 0xFFFFFFFFu;
  uint64_t mo = 0, bo = 0;
  for (uint32_t p = 1; p <= L; ++p) {
    uint32_t ph = tg_phase(P, p);
    if (ph != cur_phase) {
      uint64_t s = tg_sched_slot(P, w, ph);
      mo = pl->mem_off[s];
      bo = pl->br_off[s];
      cur_phase = ph;
    }
    int t = tg_event_type(P, w, p, L);
    uint16_t id;
    switch (t) {
      case TG_EV_RET: id = (uint16_t)P->id_ret; break;
      case TG_EV_BARRIER: id = (uint16_t)P->id_barrier; break;
      case TG_EV_MEM: {
        uint8_t k;
        uint64_t a = tg_mem_event(P, w, p, &jsw, &jst, &k);
        if (tg_is_atomic(P, w, p)) {
          /* the read, then the write, of one address */
          j->addr[mo] = a; j->kind[mo] = (uint8_t)(k & 2u); ++mo;
          j->addr[mo] = a; j->kind[mo] = (uint8_t)((k & 2u) | 1u); ++mo;
          id = (uint16_t)P->id_atomic;
          break;
        }
        j->addr[mo] = a;
        j->kind[mo] = k;
        ++mo;
        id = (uint16_t)((k & 1u) ? P->id_store : P->id_load);
        break;
      }
      case TG_EV_BRANCH: {
        uint32_t s; uint8_t y;
        tg_branch_event(P, pl->site_thr, w, p, &s, &y);
        j->site[bo] = s;
        j->taken[bo] = y;
        ++bo;
        id = (uint16_t)P->id_branch;
        break;
      }
      default: id = (uint16_t)tg_compute_id(P, pl->zipf_cdf, w, p); break;
    }
    j->opcode[base + p - 1] = id;
  }
}

static void *job_main(void *arg) {
  tg_job *j = (tg_job *)arg;
  for (uint64_t w = j->w0; w < j->w1; ++w) {
    if (j->stage == 0) j->pl->wi_off[w + 1] = tg_len(&j->pl->P, w);
    else if (j->stage == 1) walk_count(j->pl, w);
    else walk_fill(j->pl, w, j);
  }
  return NULL;
}

/* Work-items of one work-group touch the same schedule slots; ranges are cut
 * at work-group boundaries so counting needs no atomics.                    */
static void run_stage(tg_plan *pl, int stage, int threads, tg_job *proto) {
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  uint64_t n = pl->P.n_wi, wg = pl->P.wg_size;
  uint64_t ngroups = (n + wg - 1) / wg;
  if ((uint64_t)threads > ngroups) threads = (int)(ngroups ? ngroups : 1);
  pthread_t tid[256];
  tg_job jobs[256];
  for (int t = 0; t < threads; ++t) {
    jobs[t] = *proto;
    jobs[t].pl = pl;
    jobs[t].stage = stage;
    uint64_t g0 = ngroups * (uint64_t)t / (uint64_t)threads;
    uint64_t g1 = ngroups * (uint64_t)(t + 1) / (uint64_t)threads;
    jobs[t].w0 = g0 * wg;
    jobs[t].w1 = g1 * wg < n ? g1 * wg : n;
  }
  for (int t = 1; t < threads; ++t) pthread_create(&tid[t], NULL, job_main, &jobs[t]);
  job_main(&jobs[0]);
  for (int t = 1; t < threads; ++t) pthread_join(tid[t], NULL);
}

void tg_host_free(tg_plan *pl) {
  if (!pl) return;
  free(pl->zipf_cdf); free(pl->site_thr); free(pl->wi_off);
  free(pl->mem_off); free(pl->br_off); free(pl);
}

/* Returns NULL on allocation failure or invalid parameters. */
tg_plan *tg_host_plan(const tg_params *P, const uint32_t *zipf_cdf,
                      const uint32_t *site_thr, int threads, uint64_t *n_events,
                      uint64_t *n_mem, uint64_t *n_branch) {
  if (!P || P->wg_size == 0 || P->len_max < P->len_min || P->n_compute_ids == 0 ||
      P->n_sites == 0 || P->sweep_words == 0 || P->random_words == 0 ||
      P->local_words == 0 || P->stencil_dim < 3)
    return NULL;
  tg_plan *pl = (tg_plan *)calloc(1, sizeof(tg_plan));
  if (!pl) return NULL;
  pl->P = *P;
  pl->P.n_phases = P->barrier_period ? (P->len_max ? (P->len_max - 1u) / P->barrier_period + 1u : 1u) : 1u;
  uint64_t ngroups = (P->n_wi + P->wg_size - 1) / P->wg_size;
  pl->slots = ngroups * pl->P.n_phases * P->wg_size;
  pl->zipf_cdf = (uint32_t *)malloc(sizeof(uint32_t) * P->n_compute_ids);
  pl->site_thr = (uint32_t *)malloc(sizeof(uint32_t) * P->n_sites);
  pl->wi_off = (uint64_t *)calloc(P->n_wi + 1, sizeof(uint64_t));
  pl->mem_off = (uint64_t *)calloc(pl->slots + 1, sizeof(uint64_t));
  pl->br_off = (uint64_t *)calloc(pl->slots + 1, sizeof(uint64_t));
  if (!pl->zipf_cdf || !pl->site_thr || !pl->wi_off || !pl->mem_off || !pl->br_off) {
    tg_host_free(pl);
    return NULL;
  }
  memcpy(pl->zipf_cdf, zipf_cdf, sizeof(uint32_t) * P->n_compute_ids);
  memcpy(pl->site_thr, site_thr, sizeof(uint32_t) * P->n_sites);
  tg_job proto;
  memset(&proto, 0, sizeof proto);
  run_stage(pl, 0, threads, &proto);
  for (uint64_t w = 0; w < P->n_wi; ++w) pl->wi_off[w + 1] += pl->wi_off[w];
  run_stage(pl, 1, threads, &proto);
  uint64_t am = 0, ab = 0;
  for (uint64_t s = 0; s < pl->slots; ++s) {
    uint64_t cm = pl->mem_off[s], cb = pl->br_off[s];
    pl->mem_off[s] = am; pl->br_off[s] = ab;
    am += cm; ab += cb;
  }
  pl->n_events = pl->wi_off[P->n_wi];
  pl->n_mem = am;
  pl->n_branch = ab;
  *n_events = pl->n_events;
  *n_mem = am;
  *n_branch = ab;
  return pl;
}

void tg_host_wi_offsets(const tg_plan *pl, uint64_t *out) {
  memcpy(out, pl->wi_off, sizeof(uint64_t) * (pl->P.n_wi + 1));
}

/* Schedule-order offsets of the memory and branch streams ([slots] each),
 * used by the device generator so it shares the exact layout.              */
uint64_t tg_host_slots(const tg_plan *pl) { return pl->slots; }
const uint64_t *tg_host_mem_offsets(const tg_plan *pl) { return pl->mem_off; }
const uint64_t *tg_host_br_offsets(const tg_plan *pl) { return pl->br_off; }
uint32_t tg_host_n_phases(const tg_plan *pl) { return pl->P.n_phases; }

void tg_host_fill(tg_plan *pl, int threads, uint16_t *opcode, uint64_t *addr,
                  uint8_t *kind, uint32_t *site, uint8_t *taken) {
  tg_job proto;
  memset(&proto, 0, sizeof proto);
  proto.opcode = opcode; proto.addr = addr; proto.kind = kind;
  proto.site = site; proto.taken = taken;
  run_stage(pl, 2, threads, &proto);
}
