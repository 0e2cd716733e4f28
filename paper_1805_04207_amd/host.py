"""Helpers that move traces into device memory (torch is plumbing only)."""
from __future__ import annotations

import numpy as np


def host_to_device(tr, device: int = 0):
    """Copy a host trace (numpy arrays) into torch CUDA tensors."""
    import torch
    dev = torch.device("cuda", device)

    def t(a, dt):
        a = np.ascontiguousarray(a)
        return torch.from_numpy(a.view(dt)).to(dev) if a.size else torch.empty(0, dtype=torch.from_numpy(np.zeros(1, dt)).dtype, device=dev)

    return {
        "opcode": t(tr.opcode, np.int16),
        "wi_offsets": t(tr.wi_offsets.astype(np.uint64), np.int64),
        "addr": t(tr.addr.astype(np.uint64), np.int64),
        "mem_kind": t(tr.mem_kind.astype(np.uint8), np.uint8),
        "br_site": t(tr.br_site.astype(np.uint32), np.int32),
        "br_taken": t(tr.br_taken.astype(np.uint8), np.uint8),
    }


def device_trace(ctx, tensors, table, n_sites: int, history_len: int, wg_size: int = 0,
                 validate: bool = False, branch_flags: int = 0):
    """aiwc_trace over a dict of device tensors (opcode, wi_offsets, addr,
    mem_kind, br_site, br_taken); empty streams may be omitted / empty."""
    g = tensors.get
    n_ev = g("n_events")
    op = g("opcode")
    if n_ev is not None:
        op = op[:n_ev]
    addr, kind = g("addr"), g("mem_kind")
    if g("n_mem") is not None:
        addr, kind = addr[:g("n_mem")], kind[:g("n_mem")]
    site, taken = g("br_site"), g("br_taken")
    if g("n_branch") is not None:
        site, taken = site[:g("n_branch")], taken[:g("n_branch")]
    return ctx.trace(op, g("wi_offsets"), addr, kind, site, taken, table, n_sites,
                     history_len, wg_size, validate, branch_flags)
