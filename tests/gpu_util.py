"""Helpers for the GPU tests: run libaiwc on a host trace."""
import json

import numpy as np

import paper_1805_04207_amd as aiwc

_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        _ctx = aiwc.Context(0)
    return _ctx


def run(tr, validate=False, wg_size=0):
    """Copy a host trace to the GPU, characterize it, return (metrics, handle)."""
    c = ctx()
    dev = aiwc.host_to_device(tr, 0)
    t = aiwc.device_trace(c, dev, tr.table, int(tr.n_sites), int(tr.history_len), wg_size,
                          validate=validate, branch_flags=int(getattr(tr, "branch_flags", 0)))
    m = c.characterize(t)
    r = m.read()
    return r, m, t, dev


def same(a, b, drop=("overflow_redos", "partitions")):
    """Identical metrics apart from the sizing diagnostics; NaN values (the
    ratios of an empty space, an unrequested pattern entropy) compare equal."""
    dump = lambda d: json.dumps({k: v for k, v in d.items() if k not in drop}, sort_keys=True)
    return dump(a) == dump(b)
