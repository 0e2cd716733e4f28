// k_validate.hip -- optional device-side check of a trace's arrays at
// aiwc_trace_create time (AIWC_VALIDATE_ON_DEVICE).
#include <cstring>

#include "abi_internal.h"

namespace {

// flags[0]: offsets, [1]: opcode ids, [2]: mem_kind, [3]: addr sentinel,
// [4]: branch outcomes / sites, [5..8]: #load, #store, #atomic, #branch
__global__ void k_validate(TraceArgs A, u64 *flags) {
  const u64 tid = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u64 bad_off = 0, bad_id = 0, bad_kind = 0, bad_addr = 0, bad_br = 0;
  u64 nl = 0, ns = 0, na = 0, nb = 0;
  for (u64 w = tid; w < A.n_wi; w += stride)
    bad_off += A.wi_off[w + 1] < A.wi_off[w];
  if (tid == 0) bad_off += (A.wi_off[0] != 0) + (A.wi_off[A.n_wi] != A.n_events);
  for (u64 i = tid; i < A.n_events; i += stride) {
    const u32 id = A.opcode[i];
    if (id >= A.n_ids) { bad_id++; continue; }
    const u32 k = A.op_info[id] & 0xFFu;
    nl += k == AIWC_KIND_LOAD;
    ns += k == AIWC_KIND_STORE;
    na += k == AIWC_KIND_ATOMIC_RMW;
    nb += k == AIWC_KIND_BRANCH_COND;
  }
  for (u64 i = tid; i < A.n_mem; i += stride) {
    bad_kind += (A.mem_kind[i] & ~3u) != 0;
    bad_addr += A.addr[i] == ~0ull;
  }
  for (u64 i = tid; i < A.n_branch; i += stride)
    bad_br += (A.br_taken[i] > 1u) || (A.br_site[i] >= A.n_sites);
  u64 v[9] = {bad_off, bad_id, bad_kind, bad_addr, bad_br, nl, ns, na, nb};
  for (int j = 0; j < 9; ++j) {
    u64 s = wave_sum_u64(v[j]);
    if (lane_id() == 0 && s) atomicAdd(&flags[j], s);
  }
}

}  // namespace

aiwc_status validate_on_device(aiwc_ctx *ctx, const aiwc_trace *t) {
  TraceArgs a;
  memset(&a, 0, sizeof a);
  const aiwc_trace_desc &d = t->d;
  a.opcode = d.opcode; a.wi_off = (const u64 *)d.wi_offsets; a.addr = (const u64 *)d.addr;
  a.mem_kind = d.mem_kind; a.br_site = d.br_site; a.br_taken = d.br_taken;
  a.op_info = t->dev_info; a.n_events = d.n_events; a.n_wi = d.n_workitems;
  a.n_mem = d.n_mem; a.n_branch = d.n_branch; a.n_ids = d.n_opcode_ids; a.n_sites = d.n_sites;
  u64 *flags = nullptr;
  if (hipMalloc(&flags, 9 * sizeof(u64)) != hipSuccess) {
    hipGetLastError();
    ctx_error(ctx, "out of device memory for validation");
    return AIWC_ERR_OUT_OF_MEMORY;
  }
  hipMemset(flags, 0, 9 * sizeof(u64));
  hipLaunchKernelGGL(k_validate, dim3(1024), dim3(256), 0, 0, a, flags);
  u64 h[9] = {0};
  hipError_t e = hipMemcpy(h, flags, sizeof h, hipMemcpyDeviceToHost);
  hipFree(flags);
  if (e != hipSuccess) { ctx_error(ctx, "validation kernel failed: %s", hipGetErrorString(e)); return AIWC_ERR_HIP; }
  static const char *what[5] = {"work-item offsets", "opcode ids", "mem_kind bits",
                                "reserved address UINT64_MAX", "branch sites / outcomes"};
  for (int j = 0; j < 5; ++j)
    if (h[j]) { ctx_error(ctx, "invalid trace: %llu bad %s", (unsigned long long)h[j], what[j]); return AIWC_ERR_INVALID_ARG; }
  if (h[5] + h[6] + 2 * h[7] != d.n_mem || h[8] != d.n_branch) {
    ctx_error(ctx, "inconsistent trace: %llu loads + %llu stores + 2 x %llu atomics vs n_mem %llu; "
              "%llu branches vs n_branch %llu", (unsigned long long)h[5], (unsigned long long)h[6],
              (unsigned long long)h[7], (unsigned long long)d.n_mem, (unsigned long long)h[8],
              (unsigned long long)d.n_branch);
    return AIWC_ERR_INCONSISTENT;
  }
  return AIWC_OK;
}
