"""Learned sizing: prefix features vs a numpy restatement, MLP gradients vs
the FP64 reference, training on exact-path labels, and the gain of LEARNED
over BOUND sizing with identical metrics, and of the shipped network over
the heuristic (run with -m gpu)."""
import numpy as np
import pytest

import tracegen as tg
from oracle import mlp
from gpu_util import same

pytestmark = pytest.mark.gpu


def _dev_traces(specs):
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    out = []
    for sp in specs:
        d = tg.generate_device(sp, 0)
        t = aiwc.device_trace(ctx(), d, tg.opcode_table(), sp.n_sites, sp.history_len, sp.wg_size)
        out.append((sp, d, t))
    return out


def test_prefix_features_match_numpy():
    import torch
    from gpu_util import ctx
    sp = tg.config2(n_wi=512)
    h = tg.generate_host(sp)
    import paper_1805_04207_amd as aiwc
    dev = aiwc.host_to_device(h, 0)
    t = aiwc.device_trace(ctx(), dev, h.table, sp.n_sites, sp.history_len, sp.wg_size)
    f = torch.zeros((1, 40), dtype=torch.float32, device="cuda")
    ctx().sizer_features([t], f)
    f = f.cpu().numpy()[0]
    a, k = h.addr[:8192], h.mem_kind[:8192]
    for s in (0, 1):
        sel = a[((k >> 1) & 1) == s]
        for lsb in range(11):
            want = np.log2(1 + np.unique(sel >> np.uint64(lsb)).size)
            assert abs(f[8 + 11 * s + lsb] - want) < 1e-5, (s, lsb)
    assert abs(f[1] - np.log2(1 + h.addr.size)) < 1e-5
    assert abs(f[6] - ((k >> 1) & 1).mean()) < 1e-6


def test_mlp_gradients_match_fp64_reference():
    import torch
    from gpu_util import ctx
    c = ctx()
    rng = np.random.default_rng(42)
    p = c.sizer_params()
    p[:mlp.NPARAM] = rng.normal(0, 0.25, size=mlp.NPARAM).astype(np.float32)
    c.sizer_set_params(p)
    pb = c.sizer_params()[:mlp.NPARAM].astype(np.float64)   # bf16-rounded weights
    x = rng.normal(size=(48, 40)).astype(np.float32)
    y = rng.normal(size=(48, 11)).astype(np.float32)
    loss, g = c.sizer_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    lr, gr = mlp.loss_and_grad(pb, x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lr) <= 1e-4 * abs(lr)
    g = g[:mlp.NPARAM]
    err = np.abs(g - gr)
    assert np.all(err <= 1e-4 * np.abs(gr) + 1e-6), float(np.max(err / (np.abs(gr) + 1e-6)))


def test_train_and_learned_sizing_gain(tmp_path):
    import torch
    import paper_1805_04207_amd as aiwc
    from gpu_util import ctx
    c = ctx()
    train = _dev_traces(tg.config2_family(3, 192, 6, 11, len_min=256, len_max=512))
    evals = _dev_traces(tg.config2_family(4, 24, 7, 12, len_min=256, len_max=512))
    trs = [t for _, _, t in train]
    labels = []
    for m in c.characterize_batch(trs):
        r = m.read()
        labels.append([np.log2(1.0 + r["space"][0]["distinct"][k]) for k in range(11)])
    y = torch.tensor(np.array(labels, dtype=np.float32), device="cuda")
    x = torch.zeros((len(trs), 40), dtype=torch.float32, device="cuda")
    c.sizer_features(trs, x)
    loss = c.sizer_train(x, y, epochs=60, batch=64, lr=2e-3, seed=1)
    print("final train mse (normalized)", loss, flush=True)
    assert loss < 0.2
    path = str(tmp_path / "sizer.bin")
    c.sizer_save(path)
    c.sizer_load(path)
    etr = [t for _, _, t in evals]
    bound = [m.read() for m in c.characterize_batch(etr, sizing=aiwc.SIZING_BOUND)]
    sb = c.batch_stats()
    learned = [m.read() for m in c.characterize_batch(etr, sizing=aiwc.SIZING_LEARNED)]
    sl = c.batch_stats()
    for a, b in zip(bound, learned):
        assert same(a, b)
    print("bound", sb, "learned", sl, flush=True)
    assert sl["total_partitions"] < sb["total_partitions"]
    assert sl["reserved_bytes"] <= sb["reserved_bytes"]


def test_shipped_network_beats_the_heuristic():
    # the shipped weights on held-out traces of the family they were trained
    # on (another seed): fewer partitions than the heuristic (the sizing
    # without the network) and than the bound, identical metrics under all
    # three policies
    from paper_1805_04207_amd.train_sizer import DEFAULT_WEIGHTS, evaluate
    from gpu_util import ctx
    c = ctx()
    c.sizer_load(DEFAULT_WEIGHTS)
    out = evaluate(c, 48, 5, 12.0, 16.0)
    print({k: out[k]["partitions"] for k in ("bound", "heuristic", "learned")}, flush=True)
    for k in ("bound", "heuristic", "learned"):
        assert out[k]["identical_metrics"], k
    assert out["learned"]["partitions"] < out["heuristic"]["partitions"] < out["bound"]["partitions"]
