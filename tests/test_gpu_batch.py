"""Batched path: bit-identical to the single-trace path and to the oracle,
with and without a captured hipGraph, across admission waves and forced
partition overflow (run with -m gpu)."""
import dataclasses

import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle.compare import compare
from gpu_util import same
from helpers import COMPUTE, DEFAULT_TABLE, random_trace, table

pytestmark = pytest.mark.gpu


def _traces(n, scale=2e-3, seed=2):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    specs = tg.config3_specs(seed=seed, n_traces=n, scale=scale)
    hosts, trs, keep = [], [], []
    for sp in specs:
        h = tg.generate_host(sp)
        dev = aiwc.host_to_device(h, 0)
        keep.append(dev)
        hosts.append(h)
        trs.append(aiwc.device_trace(ctx(), dev, h.table, sp.n_sites, sp.history_len, sp.wg_size))
    return hosts, trs, keep


@pytest.fixture(scope="module")
def batch12():
    return _traces(12)


def test_batch_equals_single_and_oracle(batch12):
    from gpu_util import ctx
    hosts, trs, _ = batch12
    print("batch sizes", [h.opcode.size for h in hosts], flush=True)
    c = ctx()
    got = [m.read() for m in c.characterize_batch(trs)]
    single = [c.characterize(t).read() for t in trs]
    for g, s in zip(got, single):
        assert same(g, s, drop=())
    for h, g in list(zip(hosts, got))[:6]:
        bad = compare(g, oracle.characterize(h))
        assert not bad, "\n".join(bad[:10])


def test_graph_replays_are_identical(batch12):
    from gpu_util import ctx
    hosts, trs, _ = batch12
    c = ctx()
    ref = [m.read() for m in c.characterize_batch(trs)]
    for rep in range(3):
        got = [m.read() for m in c.characterize_batch(trs, use_graph=True)]
        assert all(same(g, r, drop=()) for g, r in zip(got, ref)), f"replay {rep}"
        # eager work between replays
        c.characterize(trs[0]).read()


def test_admission_waves_and_forced_redo(batch12):
    from gpu_util import ctx
    hosts, trs, _ = batch12
    c = ctx()
    ref = [m.read() for m in c.characterize_batch(trs)]
    got = [m.read() for m in c.characterize_batch(trs, admission_cap_bytes=8 << 20)]
    assert all(same(g, r, drop=()) for g, r in zip(got, ref))
    assert c.batch_stats()["waves"] >= 2
    # add a trace with ~6e5 memory events: 16 forced partitions overflow
    import paper_1805_04207_amd as aiwc
    sp = tg.config2(n_wi=2048)
    d = tg.generate_device(sp, 0)
    big = aiwc.device_trace(c, d, tg.opcode_table(), sp.n_sites, sp.history_len, sp.wg_size)
    trs2 = list(trs) + [big]
    ref = [m.read() for m in c.characterize_batch(trs2)]
    got = [m.read() for m in c.characterize_batch(trs2, force_partition_log2=4)]
    for g, r in zip(got, ref):
        assert same(g, r)
    assert c.batch_stats()["redo_partitions"] > 0


def test_autotune_search_keeps_results(batch12, tmp_path, monkeypatch):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    monkeypatch.setenv("AIWC_TUNE_CACHE", str(tmp_path / "tune.json"))
    hosts, trs, _ = batch12
    c = ctx()
    ref = [m.read() for m in c.characterize_batch(trs)]
    got = [m.read() for m in c.characterize_batch(trs, autotune=aiwc.AUTOTUNE_SEARCH)]
    for g, r in zip(got, ref):
        assert same(g, r)


def test_graph_cache_after_destroy_and_recreate():
    # a cached batch graph belongs to the traces it was built for: a trace
    # destroyed and another created (possibly at the same host address, with
    # other arrays and sizes) must not replay the old graph
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    for rep in range(4):
        sp = tg.config3_specs(seed=40 + rep, n_traces=1, scale=2e-3)[0]
        h = tg.generate_host(sp)
        dev = aiwc.host_to_device(h, 0)
        t = aiwc.device_trace(c, dev, h.table, sp.n_sites, sp.history_len, sp.wg_size)
        got = c.characterize_batch([t], use_graph=True)[0].read()
        assert same(got, c.characterize(t).read(), drop=()), f"rep {rep}"
        bad = compare(got, oracle.characterize(h))
        assert not bad, "\n".join(bad[:10])
        t.close()
        del dev


def _wide(tr, n_ids, rng):
    """The trace with half of its compute instructions moved to the compute
    ids 10 .. n_ids - 1 of a wider table (kinds unchanged, so still consistent)."""
    if n_ids == len(DEFAULT_TABLE):
        return tr
    tab = table([tuple(e) for e in DEFAULT_TABLE.tolist()] +
                [(4 + i % 5, 1 + i % 7, COMPUTE) for i in range(n_ids - len(DEFAULT_TABLE))])
    op = tr.opcode.copy()
    move = (op < 4) & (rng.random(op.size) < 0.5)
    op[move] = rng.integers(len(DEFAULT_TABLE), n_ids, size=int(move.sum()))
    return dataclasses.replace(tr, opcode=op, table=tab)


@pytest.mark.parametrize("with_global", [False, True])
def test_batch_mixed_opcode_tables(with_global):
    # one batch over traces whose opcode tables differ in size: the ops
    # kernel's LDS is sized for the largest need of any trace (the counter
    # copies per id shrink as a table grows), and a table above 8192 ids
    # sends the whole batch to the global-memory histogram
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    sizes = [10, 66, 300, 520, 4100] + ([10000] if with_global else [])
    rng = np.random.default_rng(31)
    hosts = [_wide(random_trace(rng, 200, 300, 7, 5), n, rng) for n in sizes]
    c = ctx()
    keep, trs = [], []
    for h in hosts:
        dev = aiwc.host_to_device(h, 0)
        keep.append(dev)
        trs.append(aiwc.device_trace(c, dev, h.table, int(h.n_sites), int(h.history_len), 0))
    got = [m.read() for m in c.characterize_batch(trs)]
    for n, h, t, g in zip(sizes, hosts, trs, got):
        assert same(g, c.characterize(t).read(), drop=()), f"{n} ids: batch differs from single"
        bad = compare(g, oracle.characterize(h))
        assert not bad, f"{n} ids:\n" + "\n".join(bad[:10])
