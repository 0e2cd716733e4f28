// tg_dev.hip -- device (gfx950) generator for the synthetic traces of
// tg_core.h; writes the same bytes as tg_host.c, straight into HBM.
//
// tg_dev_plan(): lengths and per-(work-item, phase) event counts on the GPU,
// prefix sums on the host (the generator is not a timed path).
// tg_dev_fill(): one thread per work-item writes its events.
#include <hip/hip_runtime.h>

#define TG_FN __device__ static inline
#include "tg_core.h"

#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

__global__ void k_len(tg_params P, uint64_t *wi_len) {
  uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < P.n_wi) wi_len[w] = tg_len(&P, w);
}

__global__ void k_count(tg_params P, const uint64_t *wi_off, uint64_t *mem_cnt,
                        uint64_t *br_cnt) {
  uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= P.n_wi) return;
  uint32_t L = (uint32_t)(wi_off[w + 1] - wi_off[w]);
  uint32_t cur = 0xFFFFFFFFu;
  uint64_t cm = 0, cb = 0, slot = 0;
  for (uint32_t p = 1; p <= L; ++p) {
    uint32_t ph = tg_phase(&P, p);
    if (ph != cur) {
      if (cur != 0xFFFFFFFFu) { mem_cnt[slot] = cm; br_cnt[slot] = cb; }
      slot = tg_sched_slot(&P, w, ph);
      cm = cb = 0;
      cur = ph;
    }
    int t = tg_event_type(&P, w, p, L);
    cm += (t == TG_EV_MEM) ? (tg_is_atomic(&P, w, p) ? 2u : 1u) : 0u;
    cb += (t == TG_EV_BRANCH);
  }
  if (cur != 0xFFFFFFFFu) { mem_cnt[slot] = cm; br_cnt[slot] = cb; }
}

__global__ void k_fill(tg_params P, const uint32_t *zipf_cdf,
                       const uint32_t *site_thr, const uint64_t *wi_off,
                       const uint64_t *mem_off, const uint64_t *br_off,
                       uint16_t *opcode, uint64_t *addr, uint8_t *kind,
                       uint32_t *site, uint8_t *taken) {
  uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= P.n_wi) return;
  uint64_t base = wi_off[w];
  uint32_t L = (uint32_t)(wi_off[w + 1] - base);
  uint32_t jsw = 0, jst = 0, cur = 0xFFFFFFFFu;
  uint64_t mo = 0, bo = 0;
  for (uint32_t p = 1; p <= L; ++p) {
    uint32_t ph = tg_phase(&P, p);
    if (ph != cur) {
      uint64_t s = tg_sched_slot(&P, w, ph);
      mo = mem_off[s];
      bo = br_off[s];
      cur = ph;
    }
    int t = tg_event_type(&P, w, p, L);
    uint16_t id;
    if (t == TG_EV_RET) {
      id = (uint16_t)P.id_ret;
    } else if (t == TG_EV_BARRIER) {
      id = (uint16_t)P.id_barrier;
    } else if (t == TG_EV_MEM) {
      uint8_t k;
      uint64_t a = tg_mem_event(&P, w, p, &jsw, &jst, &k);
      if (tg_is_atomic(&P, w, p)) {
        // the read, then the write, of one address
        addr[mo] = a; kind[mo] = (uint8_t)(k & 2u); ++mo;
        addr[mo] = a; kind[mo] = (uint8_t)((k & 2u) | 1u); ++mo;
        id = (uint16_t)P.id_atomic;
      } else {
        addr[mo] = a;
        kind[mo] = k;
        ++mo;
        id = (uint16_t)((k & 1u) ? P.id_store : P.id_load);
      }
    } else if (t == TG_EV_BRANCH) {
      uint32_t s;
      uint8_t y;
      tg_branch_event(&P, site_thr, w, p, &s, &y);
      site[bo] = s;
      taken[bo] = y;
      ++bo;
      id = (uint16_t)P.id_branch;
    } else {
      id = (uint16_t)tg_compute_id(&P, zipf_cdf, w, p);
    }
    opcode[base + p - 1] = id;
  }
}

struct DevPlan {
  tg_params P;
  uint64_t slots = 0;
  uint32_t *zipf = nullptr, *thr = nullptr;
  uint64_t *wi_off = nullptr, *mem_off = nullptr, *br_off = nullptr;
  uint64_t n_events = 0, n_mem = 0, n_branch = 0;
};

void free_plan(DevPlan *d) {
  if (!d) return;
  hipFree(d->zipf); hipFree(d->thr); hipFree(d->wi_off);
  hipFree(d->mem_off); hipFree(d->br_off);
  delete d;
}

}  // namespace

extern "C" {

void tg_dev_free(void *h) { free_plan(static_cast<DevPlan *>(h)); }

// Returns an opaque plan, or NULL on error.  All sizes are written on success.
void *tg_dev_plan(const tg_params *Pin, const uint32_t *zipf_cdf,
                  const uint32_t *site_thr, uint64_t *n_events, uint64_t *n_mem,
                  uint64_t *n_branch) {
  if (!Pin || Pin->wg_size == 0 || Pin->len_max < Pin->len_min ||
      Pin->n_compute_ids == 0 || Pin->n_sites == 0 || Pin->sweep_words == 0 ||
      Pin->random_words == 0 || Pin->local_words == 0 || Pin->stencil_dim < 3)
    return nullptr;
  (void)hipGetLastError();   // an error left by an earlier, unrelated call is not ours
  DevPlan *d = new DevPlan();
  d->P = *Pin;
  tg_params &P = d->P;
  P.n_phases = P.barrier_period ? (P.len_max ? (P.len_max - 1u) / P.barrier_period + 1u : 1u) : 1u;
  uint64_t ngroups = (P.n_wi + P.wg_size - 1) / P.wg_size;
  d->slots = ngroups * P.n_phases * P.wg_size;
  bool ok = hipMalloc(&d->zipf, 4 * P.n_compute_ids) == hipSuccess &&
            hipMalloc(&d->thr, 4ull * P.n_sites) == hipSuccess &&
            hipMalloc(&d->wi_off, 8 * (P.n_wi + 1)) == hipSuccess &&
            hipMalloc(&d->mem_off, 8 * (d->slots + 1)) == hipSuccess &&
            hipMalloc(&d->br_off, 8 * (d->slots + 1)) == hipSuccess;
  if (!ok) { free_plan(d); return nullptr; }
  hipMemcpy(d->zipf, zipf_cdf, 4 * P.n_compute_ids, hipMemcpyHostToDevice);
  hipMemcpy(d->thr, site_thr, 4ull * P.n_sites, hipMemcpyHostToDevice);
  const int B = 256;
  unsigned grid = (unsigned)((P.n_wi + B - 1) / B);
  std::vector<uint64_t> h(P.n_wi + 1, 0);
  if (P.n_wi) {
    k_len<<<grid, B>>>(P, d->wi_off + 1);
    hipMemcpy(h.data() + 1, d->wi_off + 1, 8 * P.n_wi, hipMemcpyDeviceToHost);
  }
  for (uint64_t w = 0; w < P.n_wi; ++w) h[w + 1] += h[w];
  hipMemcpy(d->wi_off, h.data(), 8 * (P.n_wi + 1), hipMemcpyHostToDevice);
  d->n_events = h[P.n_wi];
  hipMemset(d->mem_off, 0, 8 * (d->slots + 1));
  hipMemset(d->br_off, 0, 8 * (d->slots + 1));
  if (P.n_wi) k_count<<<grid, B>>>(P, d->wi_off, d->mem_off, d->br_off);
  std::vector<uint64_t> cm(d->slots), cb(d->slots);
  hipMemcpy(cm.data(), d->mem_off, 8 * d->slots, hipMemcpyDeviceToHost);
  hipMemcpy(cb.data(), d->br_off, 8 * d->slots, hipMemcpyDeviceToHost);
  uint64_t am = 0, ab = 0;
  for (uint64_t s = 0; s < d->slots; ++s) {
    uint64_t a = cm[s], b = cb[s];
    cm[s] = am; cb[s] = ab;
    am += a; ab += b;
  }
  hipMemcpy(d->mem_off, cm.data(), 8 * d->slots, hipMemcpyHostToDevice);
  hipMemcpy(d->br_off, cb.data(), 8 * d->slots, hipMemcpyHostToDevice);
  if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) {
    free_plan(d);
    return nullptr;
  }
  d->n_mem = am;
  d->n_branch = ab;
  *n_events = d->n_events;
  *n_mem = am;
  *n_branch = ab;
  return d;
}

// Writes the trace into caller-allocated device arrays (sizes from the plan)
// and wi_offsets[n_wi + 1].  Returns 0 on success.
int tg_dev_fill(void *h, uint64_t *wi_offsets, uint16_t *opcode, uint64_t *addr,
                uint8_t *kind, uint32_t *site, uint8_t *taken) {
  DevPlan *d = static_cast<DevPlan *>(h);
  if (!d) return 1;
  const tg_params &P = d->P;
  hipMemcpy(wi_offsets, d->wi_off, 8 * (P.n_wi + 1), hipMemcpyDeviceToDevice);
  const int B = 256;
  if (P.n_wi)
    k_fill<<<(unsigned)((P.n_wi + B - 1) / B), B>>>(P, d->zipf, d->thr, d->wi_off,
                                                    d->mem_off, d->br_off, opcode,
                                                    addr, kind, site, taken);
  if (hipDeviceSynchronize() != hipSuccess) return 2;
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
