"""aiwc_characterize_static, the entry point that allocates nothing, against
aiwc_characterize on the same traces: identical metrics and class
histograms, on consecutive calls that reuse the GPU's static scratch array
(the second call with a smaller trace), and its size checks."""
import numpy as np
import pytest

import tracegen as tg
from gpu_util import ctx, same

pytestmark = pytest.mark.gpu


def static_run(c, t, n_classes, nbytes=None):
    import torch
    import paper_1805_04207_amd.aiwc as A
    n = A.static_result_bytes(n_classes) if nbytes is None else nbytes
    # poison the block, so that a field the kernels failed to write shows
    out = torch.full((n,), 0xAB, dtype=torch.uint8, device="cuda")
    c.characterize_static(t, out)
    torch.cuda.synchronize()
    return A.static_result(out.cpu().numpy().tobytes(), n_classes)


def plain_run(c, t, n_classes):
    m = c.characterize(t)
    return m.read(), m.class_hist(n_classes).tolist()


def traces():
    """The config1 trace, then a smaller trace of another seed and shape."""
    big = tg.config1()
    small = tg.config1(seed=7)
    small.n_wi = 64
    small.len_min, small.len_max = 300, 900
    small.p_atomic = 0.1
    return [tg.generate_host(big), tg.generate_host(small)]


def test_static_equals_characterize_on_consecutive_calls():
    import paper_1805_04207_amd as aiwc
    c = ctx()
    hs = traces()
    assert hs[1].addr.size < hs[0].addr.size and hs[1].opcode.size < hs[0].opcode.size
    devs = [aiwc.host_to_device(h, 0) for h in hs]
    trs = [aiwc.device_trace(c, d, h.table, h.spec.n_sites, h.spec.history_len, h.spec.wg_size)
           for d, h in zip(devs, hs)]
    want = [plain_run(c, t, tg.N_CLASSES) for t in trs]
    # big, big again (the array holds the first call's contents), then small
    for i in (0, 0, 1):
        print(f"[static] call on trace {i}: {hs[i].opcode.size} events", flush=True)
        got, cls = static_run(c, trs[i], tg.N_CLASSES)
        assert same(got, want[i][0], drop=()), f"metrics differ on trace {i}"
        assert cls == want[i][1], f"class histogram differs on trace {i}"
    # the plain path is unaffected by the static calls
    again = plain_run(c, trs[0], tg.N_CLASSES)
    assert same(again[0], want[0][0], drop=()) and again[1] == want[0][1]



def test_static_with_hot_partitions():
    """A memory stream whose accesses pile onto two local pages (the hot-page
    path: candidate tables and compacted records in the static array) and a
    global one: the static entry equals aiwc_characterize, on two calls in a
    row, the second on a smaller trace."""
    import paper_1805_04207_amd as aiwc
    from helpers import mem_trace
    c = ctx()
    rng = np.random.default_rng(21)
    hs = []
    for n, pages, local in ((1200000, [0, 1], True), (700000, [77], False)):
        k = int(n * 0.9)
        a_hot = rng.choice(np.asarray(pages, dtype=np.uint64), size=k) * np.uint64(1024) + \
            rng.integers(0, 1024, size=k, dtype=np.uint64)
        a = np.concatenate([a_hot, rng.integers(0, 1 << 26, size=n - k, dtype=np.uint64)])
        kinds = (rng.random(n) < 0.3).astype(np.uint8)
        if local:
            kinds[:k] |= 2
        order = rng.permutation(n)
        hs.append(mem_trace(a[order], kinds[order]))
    assert hs[0].addr.size >= 1 << 18 and hs[1].addr.size >= 1 << 18
    n_cls = int(hs[0].table["op_class"].max()) + 1
    devs = [aiwc.host_to_device(h, 0) for h in hs]
    trs = [aiwc.device_trace(c, d, h.table, int(h.n_sites), int(h.history_len), 0)
           for d, h in zip(devs, hs)]
    want = [plain_run(c, t, n_cls) for t in trs]
    for i in (0, 1):
        print(f"[static] hot-page trace {i}: {hs[i].addr.size} memory events", flush=True)
        got, cls = static_run(c, trs[i], n_cls)
        assert same(got, want[i][0], drop=()), f"metrics differ on hot-page trace {i}"
        assert cls == want[i][1], f"class histogram differs on hot-page trace {i}"


def test_static_size_checks():
    import paper_1805_04207_amd as aiwc
    import paper_1805_04207_amd.aiwc as A
    c = ctx()
    h = tg.generate_host(tg.config1(seed=3))
    t = aiwc.device_trace(c, aiwc.host_to_device(h, 0), h.table, h.spec.n_sites,
                          h.spec.history_len, h.spec.wg_size)
    with pytest.raises(aiwc.AiwcError) as e:
        static_run(c, t, tg.N_CLASSES, nbytes=A.static_result_bytes(tg.N_CLASSES) - 8)
    assert e.value.status == A.AIWC_ERR_INVALID_ARG
    # a trace whose scratch exceeds the static array is refused before any
    # launch (about 1e7 memory events need ~115 MiB)
    d = tg.generate_device(tg.config2(n_wi=1 << 15), 0)
    assert d["n_mem"] > 8_000_000
    tb = aiwc.device_trace(c, d, tg.opcode_table(), d["spec"].n_sites, d["spec"].history_len,
                           d["spec"].wg_size)
    with pytest.raises(aiwc.AiwcError) as e:
        static_run(c, tb, tg.N_CLASSES)
    assert e.value.status == A.AIWC_ERR_UNSUPPORTED
    assert "scratch" in str(e.value)
    # and the plain path still takes it; the static path still works after
    assert c.characterize(tb).read()["space"][0]["total_accesses"] > 0
    got, cls = static_run(c, t, tg.N_CLASSES)
    want = plain_run(c, t, tg.N_CLASSES)
    assert same(got, want[0], drop=()) and cls == want[1]
    assert int(np.sum(cls)) == h.opcode.size
