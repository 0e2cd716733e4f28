"""Stage timers (aiwc_profile_*) in the two-stream stage order, for one
trace and for an eager batch (run with -m gpu)."""
import numpy as np
import pytest

from helpers import random_trace

pytestmark = pytest.mark.gpu

# "join": the caller's stream waiting for the side stream, before the bucket
STAGES = {"k_zero", "k_ops", "k_mem_hist", "k_mem_scan", "k_mem_scatter", "join", "k_mem_bucket",
          "k_br_pack", "k_br_sort", "k_br_segments", "k_br_windows", "k_finalize"}


def test_stage_timers_single_and_batch():
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    rng = np.random.default_rng(71)
    ts = [random_trace(rng, 30, 3000, 60, 8, addr_bits=20) for _ in range(3)]
    keep, hs = [], []
    for t in ts:
        dev = aiwc.host_to_device(t, 0)
        keep.append(dev)
        hs.append(aiwc.device_trace(c, dev, t.table, int(t.n_sites), 8))
    c.profile_enable(True)
    try:
        for call in (lambda: c.characterize(hs[0]).read(),
                     lambda: [m.read() for m in c.characterize_batch(hs)]):
            for _ in range(2):           # the marks of one call only, each time
                call()
                stages = c.profile_read()
                names = [n for n, _ in stages]
                assert set(names) == STAGES and len(names) == len(STAGES), names
                assert all(ms >= 0.0 for _, ms in stages)
    finally:
        c.profile_enable(False)
