"""Parity at the full sizes of the benchmarked workloads (run with -m gpu).

* The plain large trace (2^20 work-items, ~1.07e9 events) through the same
  plan and launches that bench.py times, against the vectorised oracle
  (oracle/bulk.py) on the byte-identical host trace: every field, the class
  histogram and the level-0 spectrum.  The batched path with learned sizing
  and a replayed graph must give the identical metrics.
* The uneven batch (512 traces of 1e4..1e8 events, ~5e9 in total) in one
  batched call with learned sizing, autotuning and a replayed graph: every
  trace identical to its plain per-trace result, the three smallest against
  the C oracle and a mid-size one against the vectorised oracle.
* The aggregate over invocations: the plain large trace cut into 8
  invocations (work-items at random boundaries, memory and branch streams at
  random points) and merged must equal the plain path on the whole; the 512
  uneven invocations merged must satisfy every relation between an aggregate
  and its parts, and the 256 smallest merged must match the vectorised oracle
  on their concatenation.
* Streaming: the plain large trace appended in 16 chunks and finished must
  equal the plain path on the whole.
* The stress batch (64 traces, 2^32 addresses in total, up to 2^28 per trace,
  history 32 over 2^16 sites) in one batched call with learned sizing and a
  200 GiB admission cap: the two smallest traces against the C oracle, every
  trace against the invariants that hold at any size, and a sample of traces
  against the plain per-trace path.
"""
import json
import time

import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle import bulk
from oracle.compare import compare

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[fullsize] {msg}", flush=True)


def same(a, b):
    """Identical metrics (NaN ratios of an empty space compare equal)."""
    drop = ("overflow_redos", "partitions")
    dump = lambda d: json.dumps({k: v for k, v in d.items() if k not in drop}, sort_keys=True)
    return dump(a) == dump(b)


def spectrum_of(counts0):
    """{f: m_f} of the level-0 counts."""
    if counts0.size == 0:
        return {}
    b = np.bincount(counts0)
    f = np.flatnonzero(b)
    return {int(x): int(b[x]) for x in f}


def spectrum_of_host(h, space):
    """{f: m_f} of one space's level-0 counts, from the host trace."""
    a = np.asarray(h.addr)[((np.asarray(h.mem_kind) >> 1) & 1) == space]
    if a.size == 0:
        return {}
    _, c = np.unique(a, return_counts=True)
    return spectrum_of(c)


def res_spectrum(ctx, t, space):
    """The spectrum pairs of the plain path on trace t."""
    return ctx.characterize(t).spectrum(space)


def invariants(r, n_mem_space):
    """Relations that hold for any trace (Metrics section definitions)."""
    for s in (0, 1):
        sp = r["space"][s]
        d, h = sp["distinct"], sp["entropy"]
        assert sp["total_accesses"] == n_mem_space[s]
        assert sp["total_reads"] + sp["total_writes"] == sp["total_accesses"]
        assert sp["footprint"] == d[0]
        assert sp["footprint_90"] <= d[0]
        for k in range(10):
            assert d[k + 1] <= d[k] <= 2 * d[k + 1]
            assert h[k + 1] <= h[k] * (1 + 1e-12) + 1e-12
            assert h[k] <= h[k + 1] + 1.0 + 1e-9
        if d[0]:
            assert h[0] <= np.log2(d[0]) + 1e-9
    assert 0.0 <= r["yokota_entropy"] <= 1.0 + 1e-12
    assert 0.0 <= r["linear_branch_entropy"] <= 1.0


@pytest.mark.timeout(1200)
def test_plain_large_trace_full_size():
    import torch
    import paper_1805_04207_amd as aiwc

    spec = tg.config2(n_wi=1 << 20)
    t0 = time.time()
    h = tg.generate_host(spec)
    log(f"host trace: {h.opcode.size} events, {h.addr.size} memory, {h.br_site.size} branch "
        f"({time.time() - t0:.1f}s)")
    ctx = aiwc.Context(0)
    dev = aiwc.host_to_device(h, 0)
    tr = aiwc.device_trace(ctx, dev, h.table, int(h.n_sites), int(h.history_len), spec.wg_size)
    stream = torch.cuda.current_stream()
    m = ctx.characterize(tr, stream)
    got = m.read()
    ncls = int(np.asarray(h.table)["op_class"].max()) + 1
    got_cls = m.class_hist(ncls)
    got_spec = [dict(m.spectrum(s)) for s in (0, 1)]
    log(f"plain path done: partitions {got['partitions']}, redos {got['overflow_redos']}")
    from paper_1805_04207_amd.train_sizer import DEFAULT_WEIGHTS
    ctx.sizer_load(DEFAULT_WEIGHTS)
    for rep in range(2):
        gb = ctx.characterize_batch([tr], sizing=aiwc.SIZING_LEARNED, use_graph=True,
                                    stream=stream)[0].read()
        assert same(gb, got), f"batched replay {rep} differs from the plain path"
    log("batched path identical")
    del tr, dev
    torch.cuda.empty_cache()
    t0 = time.time()
    want = bulk.characterize(h, progress=log)
    log(f"vectorised oracle ({time.time() - t0:.1f}s)")
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])
    assert np.array_equal(np.asarray(got_cls)[:len(want["_class_hist"])], want["_class_hist"])
    for s in (0, 1):
        assert got_spec[s] == spectrum_of(want["space"][s]["_counts0"]), f"spectrum space {s}"
    kinds = np.asarray(h.mem_kind)
    loc = int(np.count_nonzero((kinds >> 1) & 1))
    invariants(got, (kinds.size - loc, loc))


@pytest.mark.timeout(1200)
def test_stress_batch_full_size():
    import torch
    import paper_1805_04207_amd as aiwc
    from paper_1805_04207_amd.train_sizer import DEFAULT_WEIGHTS

    specs = tg.config5_specs()
    ctx = aiwc.Context(0)
    ctx.sizer_load(DEFAULT_WEIGHTS)
    keep, trs, n_mem = [], [], []
    t0 = time.time()
    for sp in specs:
        d = tg.generate_device(sp, 0)
        keep.append(d)
        n_mem.append(d["n_mem"])
        trs.append(aiwc.device_trace(ctx, d, tg.opcode_table(), sp.n_sites, sp.history_len,
                                     sp.wg_size))
    torch.cuda.synchronize()
    log(f"{len(trs)} traces, {sum(n_mem)} addresses, generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    res = [m.read() for m in ctx.characterize_batch(
        trs, sizing=aiwc.SIZING_LEARNED, admission_cap_bytes=200 << 30, use_graph=False)]
    st = ctx.batch_stats()
    log(f"batched: {time.time() - t0:.1f}s, waves {st['waves']}, redo partitions "
        f"{st['redo_partitions']} of {st['total_partitions']}")
    # the recipe targets 2^32 addresses; the realised count (memory events are
    # drawn per instruction) lies within a percent of it
    assert abs(sum(n_mem) - (1 << 32)) < 0.02 * (1 << 32)
    assert max(n_mem) < 1.02 * (1 << 28)
    for r, nm in zip(res, n_mem):
        invariants(r, (nm, 0))
        assert r["space"][0]["distinct"][0] <= min(nm, 1 << 28)
    order = np.argsort(n_mem)
    # the two smallest traces against the C oracle (byte-identical host copies)
    for i in (int(order[0]), int(order[1])):
        hh = tg.generate_host(specs[i])
        want = oracle.characterize(hh)
        bad = compare(res[i], want)
        assert not bad, f"batched, trace {i}:\n" + "\n".join(bad[:20])
        bad = compare(ctx.characterize(trs[i]).read(), want)
        assert not bad, f"plain, trace {i}:\n" + "\n".join(bad[:20])
    log("oracle parity on the two smallest traces")
    # the largest trace (2^28 uniform addresses, 4.5e7 branches at history
    # 32 over 2^16 sites) against the vectorised oracle, element by element
    top = int(order[-1])
    log(f"vectorised oracle on the largest trace {top} ({n_mem[top]} addresses)")
    hh = tg.generate_host(specs[top])
    want = bulk.characterize(hh)
    bad = compare(res[top], want)
    assert not bad, f"batched, trace {top}:\n" + "\n".join(bad[:20])
    assert spectrum_of_host(hh, 0) == dict(res_spectrum(ctx, trs[top], 0)), "spectrum"
    log(f"oracle parity on the largest trace {top}")
    del hh, want
    # the plain per-trace path on a sample (median, largest)
    for i in (int(order[len(order) // 2]), int(order[-1])):
        assert same(ctx.characterize(trs[i]).read(), res[i]), f"trace {i}"
    log("plain path identical on the sample")


@pytest.mark.timeout(1200)
def test_uneven_batch_full_size():
    import torch
    import paper_1805_04207_amd as aiwc
    from paper_1805_04207_amd.train_sizer import DEFAULT_WEIGHTS

    specs = tg.config3_specs(seed=2, n_traces=512, scale=1.0)
    ctx = aiwc.Context(0)
    ctx.sizer_load(DEFAULT_WEIGHTS)
    keep, trs, n_ev, n_mem = [], [], [], []
    t0 = time.time()
    for sp in specs:
        d = tg.generate_device(sp, 0)
        keep.append(d)
        n_ev.append(d["n_events"])
        n_mem.append(d["n_mem"])
        trs.append(aiwc.device_trace(ctx, d, tg.opcode_table(), sp.n_sites, sp.history_len,
                                     sp.wg_size))
    torch.cuda.synchronize()
    log(f"{len(trs)} traces, {sum(n_ev)} events, generated in {time.time() - t0:.1f}s")
    opts = dict(sizing=aiwc.SIZING_LEARNED, autotune=aiwc.AUTOTUNE_SEARCH, use_graph=True)
    res = [m.read() for m in ctx.characterize_batch(trs, **opts)]
    res2 = [m.read() for m in ctx.characterize_batch(trs, **opts)]     # graph replay
    st = ctx.batch_stats()
    log(f"batched: waves {st['waves']}, redo partitions {st['redo_partitions']} of "
        f"{st['total_partitions']}")
    for i, t in enumerate(trs):
        p = ctx.characterize(t).read()
        assert same(p, res[i]) and same(p, res2[i]), f"trace {i}"
        loc = p["space"][1]["total_accesses"]
        invariants(p, (n_mem[i] - loc, loc))
    log("every trace identical to the plain path")
    order = np.argsort(n_ev)
    for i in (int(order[0]), int(order[1]), int(order[2])):
        bad = compare(res[i], oracle.characterize(tg.generate_host(specs[i])))
        assert not bad, f"trace {i}:\n" + "\n".join(bad[:20])
    mid = int(order[len(order) // 2])
    bad = compare(res[mid], bulk.characterize(tg.generate_host(specs[mid])))
    assert not bad, f"trace {mid}:\n" + "\n".join(bad[:20])
    log(f"oracle parity on traces {int(order[0])}, {int(order[1])}, {int(order[2])} and {mid} "
        f"({n_ev[mid]} events)")
    # the largest trace (about 1e8 events) against the vectorised oracle
    top = int(order[-1])
    log(f"vectorised oracle on the largest trace {top} ({n_ev[top]} events)")
    hh = tg.generate_host(specs[top])
    want = bulk.characterize(hh)
    bad = compare(res[top], want)
    assert not bad, f"trace {top}:\n" + "\n".join(bad[:20])
    for s in (0, 1):
        assert spectrum_of_host(hh, s) == dict(res_spectrum(ctx, trs[top], s)), f"spectrum {s}"
    log(f"oracle parity on the largest trace {top}")


@pytest.mark.timeout(1200)
def test_merged_pieces_of_the_large_trace():
    import torch
    import paper_1805_04207_amd as aiwc

    spec = tg.config2(n_wi=1 << 20)
    d = tg.generate_device(spec, 0)
    ctx = aiwc.Context(0)
    tab = tg.opcode_table()
    whole = aiwc.device_trace(ctx, d, tab, spec.n_sites, spec.history_len, spec.wg_size)
    plain = ctx.characterize(whole).read()
    rng = np.random.default_rng(77)
    k = 8
    wcut = np.sort(rng.choice(np.arange(1, spec.n_wi), size=k - 1, replace=False))
    wcut = np.concatenate([[0], wcut, [spec.n_wi]]).astype(np.int64)
    off = d["wi_offsets"]
    ecut = off[torch.from_numpy(wcut).to(off.device)].cpu().numpy()
    mcut = np.concatenate([[0], np.sort(rng.integers(0, d["n_mem"] + 1, size=k - 1)),
                           [d["n_mem"]]])
    bcut = np.concatenate([[0], np.sort(rng.integers(0, d["n_branch"] + 1, size=k - 1)),
                           [d["n_branch"]]])
    keep, pieces = [], []
    for i in range(k):
        p = {"opcode": d["opcode"][ecut[i]:ecut[i + 1]],
             "wi_offsets": (off[wcut[i]:wcut[i + 1] + 1] - off[wcut[i]]).contiguous(),
             "addr": d["addr"][mcut[i]:mcut[i + 1]], "mem_kind": d["mem_kind"][mcut[i]:mcut[i + 1]],
             "br_site": d["br_site"][bcut[i]:bcut[i + 1]],
             "br_taken": d["br_taken"][bcut[i]:bcut[i + 1]]}
        keep.append(p)
        pieces.append(aiwc.device_trace(ctx, p, tab, spec.n_sites, spec.history_len, spec.wg_size))
    torch.cuda.synchronize()
    log(f"{k} pieces: work-item cuts {wcut.tolist()}")
    got = ctx.characterize_merged(pieces).read()
    assert same(got, plain), "merged pieces differ from the whole"
    log("merged pieces identical to the plain path on the whole")


@pytest.mark.timeout(1200)
def test_merged_uneven_invocations_full_size():
    import torch
    import paper_1805_04207_amd as aiwc

    specs = tg.config3_specs(seed=2, n_traces=512, scale=1.0)
    ctx = aiwc.Context(0)
    keep, trs, n_ev = [], [], []
    for sp in specs:
        d = tg.generate_device(sp, 0)
        keep.append(d)
        n_ev.append(d["n_events"])
        trs.append(aiwc.device_trace(ctx, d, tg.opcode_table(), sp.n_sites, sp.history_len,
                                     sp.wg_size))
    torch.cuda.synchronize()
    m = ctx.characterize_merged(trs)
    r = m.read()
    ncls = int(np.asarray(tg.opcode_table())["op_class"].max()) + 1
    cls = np.asarray(m.class_hist(ncls))
    log(f"merged {len(trs)} invocations, {sum(n_ev)} events")
    parts, pcls = [], np.zeros(ncls, dtype=np.uint64)
    for t in trs:
        pm = ctx.characterize(t)
        parts.append(pm.read())
        pcls += np.asarray(pm.class_hist(ncls), dtype=np.uint64)
    # relations between an aggregate and its parts
    tot = lambda f: sum(p[f] for p in parts)
    for f in ("total_instructions", "work_items", "barriers_hit", "itb_count", "itb_sum",
              "simd_sum", "total_branches"):
        assert r[f] == tot(f), f
    assert r["simd_max"] == max(p["simd_max"] for p in parts)
    assert r["itb_min"] == min(p["itb_min"] for p in parts)
    assert r["itb_max"] == max(p["itb_max"] for p in parts)
    assert r["ipt_min"] == min(p["ipt_min"] for p in parts)
    assert r["ipt_max"] == max(p["ipt_max"] for p in parts)
    assert r["load_imbalance"] == r["ipt_max"] - r["ipt_min"]
    assert np.array_equal(cls, pcls)
    assert max(p["unique_branches"] for p in parts) <= r["unique_branches"] <= tot("unique_branches")
    assert tot("n_windows") <= r["n_windows"] <= r["total_branches"]
    for s in (0, 1):
        sp = r["space"][s]
        for f in ("total_accesses", "total_reads", "total_writes"):
            assert sp[f] == sum(p["space"][s][f] for p in parts), (s, f)
        for f in ("unique_reads", "unique_writes"):
            vals = [p["space"][s][f] for p in parts]
            assert max(vals) <= sp[f] <= sum(vals), (s, f)
        for kk in range(11):
            vals = [p["space"][s]["distinct"][kk] for p in parts]
            assert max(vals) <= sp["distinct"][kk] <= sum(vals), (s, kk)
    loc = r["space"][1]["total_accesses"]
    invariants(r, (r["space"][0]["total_accesses"], loc))
    log("aggregate consistent with its 512 parts")
    # exact parity on the 256 smallest invocations merged
    order = np.argsort(n_ev)[:256]
    sub = [trs[i] for i in order]
    got = ctx.characterize_merged(sub).read()
    want = bulk.characterize(oracle.MergedTrace([tg.generate_host(specs[i]) for i in order]))
    bad = compare(got, want)
    assert not bad, "\n".join(bad[:20])
    log(f"256 smallest merged ({sum(n_ev[i] for i in order)} events) match the oracle")


@pytest.mark.timeout(1200)
def test_stream_of_the_large_trace():
    import torch
    import paper_1805_04207_amd as aiwc

    spec = tg.config2(n_wi=1 << 20)
    d = tg.generate_device(spec, 0)
    ctx = aiwc.Context(0)
    tab = tg.opcode_table()
    plain = ctx.characterize(aiwc.device_trace(ctx, d, tab, spec.n_sites, spec.history_len,
                                               spec.wg_size)).read()
    k = 16
    wcut = np.linspace(0, spec.n_wi, k + 1).astype(np.int64)
    off = d["wi_offsets"]
    ecut = off[torch.from_numpy(wcut).to(off.device)].cpu().numpy()
    mcut = np.linspace(0, d["n_mem"], k + 1).astype(np.int64)
    bcut = np.linspace(0, d["n_branch"], k + 1).astype(np.int64)
    st = ctx.stream(d["n_mem"] // 3)     # reserved below the need: moves happen too
    for i in range(k):
        p = {"opcode": d["opcode"][ecut[i]:ecut[i + 1]],
             "wi_offsets": (off[wcut[i]:wcut[i + 1] + 1] - off[wcut[i]]).contiguous(),
             "addr": d["addr"][mcut[i]:mcut[i + 1]], "mem_kind": d["mem_kind"][mcut[i]:mcut[i + 1]],
             "br_site": d["br_site"][bcut[i]:bcut[i + 1]],
             "br_taken": d["br_taken"][bcut[i]:bcut[i + 1]]}
        st.append(aiwc.device_trace(ctx, p, tab, spec.n_sites, spec.history_len, spec.wg_size))
    got = st.finish().read()
    assert same(got, plain), "stream of 16 chunks differs from the whole"
    log("stream of 16 chunks identical to the plain path on the whole")
    st.close()
    st = ctx.stream(host_retain=True)
    for i in range(k):
        p = {"opcode": d["opcode"][ecut[i]:ecut[i + 1]],
             "wi_offsets": (off[wcut[i]:wcut[i + 1] + 1] - off[wcut[i]]).contiguous(),
             "addr": d["addr"][mcut[i]:mcut[i + 1]], "mem_kind": d["mem_kind"][mcut[i]:mcut[i + 1]],
             "br_site": d["br_site"][bcut[i]:bcut[i + 1]],
             "br_taken": d["br_taken"][bcut[i]:bcut[i + 1]]}
        st.append(aiwc.device_trace(ctx, p, tab, spec.n_sites, spec.history_len, spec.wg_size))
    got = st.finish().read()
    assert same(got, plain), "host-retained stream differs from the whole"
    log("host-retained stream identical to the plain path on the whole")
    st.close()
    # out of core: the memory stream stays in pinned host memory and the
    # device holds a quarter of its partition records at a time
    st = ctx.stream(host_retain=True)
    st.set_device_budget(12 * (d["n_mem"] // 4))
    for i in range(k):
        p = {"opcode": d["opcode"][ecut[i]:ecut[i + 1]],
             "wi_offsets": (off[wcut[i]:wcut[i + 1] + 1] - off[wcut[i]]).contiguous(),
             "addr": d["addr"][mcut[i]:mcut[i + 1]], "mem_kind": d["mem_kind"][mcut[i]:mcut[i + 1]],
             "br_site": d["br_site"][bcut[i]:bcut[i + 1]],
             "br_taken": d["br_taken"][bcut[i]:bcut[i + 1]]}
        st.append(aiwc.device_trace(ctx, p, tab, spec.n_sites, spec.history_len, spec.wg_size))
    got = st.finish().read()
    s = st.stats()
    assert s["groups"] >= 4 and s["device_records"] < d["n_mem"] // 3, s
    assert same(got, plain), "out-of-core stream differs from the whole"
    log(f"out-of-core stream ({s['groups']} partition groups, {s['device_records']} of "
        f"{d['n_mem']} records on the device at once) identical to the plain path")
