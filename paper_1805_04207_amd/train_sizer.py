"""Train the sizing network on the GPU and save its weights.

Traces of the config2 family (tracegen.config2_family: log-uniform
work-item counts over 2^8..2^16 by default, work-items of 768..1280 events,
per-trace pattern mix, stride and gather range) are
generated on the device, characterized exactly by libaiwc (labels =
log2(1 + distinct_k) of the global space, k = 0..10), featurized by the
library's prefix-feature kernel, and the 40->64->64->64->11 network is
trained by the library's own forward / backward / Adam kernels.  The margin
added to predictions before sizing is calibrated on a held-out split so that
at most `--overflow-target` of the held-out traces would be undersized at
skip 10 (the page count that sizes the partitions).

    python -m paper_1805_04207_amd.train_sizer --traces 20000 --out sizer_weights.bin
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "sizer_weights.bin")


def build_dataset(ctx, n: int, seed: int, wi_lo: float, wi_hi: float, batch: int = 64):
    """Features and exact labels of n generated traces (device tensors)."""
    import torch
    import tracegen as tg
    from . import device_trace

    specs = tg.config2_family(seed, n, wi_lo, wi_hi, len_min=768, len_max=1280)
    feats, labels = [], []
    for b0 in range(0, n, batch):
        keep, trs = [], []
        for sp in specs[b0:b0 + batch]:
            d = tg.generate_device(sp, ctx.device)
            keep.append(d)
            trs.append(device_trace(ctx, d, tg.opcode_table(), sp.n_sites, sp.history_len,
                                    sp.wg_size))
        x = torch.zeros((len(trs), 40), dtype=torch.float32, device=f"cuda:{ctx.device}")
        ctx.sizer_features(trs, x)
        for m in ctx.characterize_batch(trs):
            r = m.read()
            labels.append([np.log2(1.0 + r["space"][0]["distinct"][k]) for k in range(11)])
        feats.append(x)
        del keep, trs
        if (b0 // batch) % 8 == 7:
            print(f"# labelled {min(n, b0 + batch)} / {n} traces", file=sys.stderr, flush=True)
    x = torch.cat(feats)
    y = torch.tensor(np.array(labels, dtype=np.float32), device=x.device)
    return x, y


def evaluate(ctx, n: int, seed: int, wi_lo: float, wi_hi: float, repeats: int = 1):
    """What the network gains: one batch of held-out traces under each sizing
    mode -- partitions (device memory and work), partitions redone after an
    overflow, and the time of the batched call; metrics must not change."""
    import torch
    import tracegen as tg
    from . import SIZING_BOUND, SIZING_HEURISTIC, SIZING_LEARNED, device_trace

    specs = tg.config2_family(seed, n, wi_lo, wi_hi, len_min=768, len_max=1280)
    keep, trs, events = [], [], 0
    for sp in specs:
        d = tg.generate_device(sp, ctx.device)
        keep.append(d)
        events += d["n_events"]
        trs.append(device_trace(ctx, d, tg.opcode_table(), sp.n_sites, sp.history_len,
                                sp.wg_size))
    out, ref = {"traces": n, "events": events}, None
    for name, mode in (("bound", SIZING_BOUND), ("heuristic", SIZING_HEURISTIC),
                       ("learned", SIZING_LEARNED)):
        ctx.characterize_batch(trs, sizing=mode)
        dts = []
        for _ in range(max(1, repeats)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = [m.read() for m in ctx.characterize_batch(trs, sizing=mode)]
            torch.cuda.synchronize()
            dts.append(time.perf_counter() - t0)
        dt = float(np.median(dts))
        st = ctx.batch_stats()
        key = [json.dumps({k: v for k, v in r.items() if k not in ("overflow_redos", "partitions")},
                          sort_keys=True) for r in res]
        if ref is None:
            ref = key
        out[name] = {"ms": 1e3 * dt, "partitions": st["total_partitions"],
                     "redo_partitions": st["redo_partitions"],
                     "redo_rate": st["redo_partitions"] / max(1, st["total_partitions"]),
                     "reserved_bytes": st["reserved_bytes"], "waves": st["waves"],
                     "identical_metrics": key == ref}
        print(f"# eval {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--traces", type=int, default=20000)
    ap.add_argument("--val-frac", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--wi-log2", type=float, nargs=2, default=(8.0, 16.0))
    ap.add_argument("--overflow-target", type=float, default=0.02)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None, help="write a JSON report here")
    ap.add_argument("--eval-traces", type=int, default=256,
                    help="held-out family traces run under BOUND / HEURISTIC / LEARNED sizing")
    ap.add_argument("--eval-wi-log2", type=float, nargs=2, default=(10.0, 16.0))
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="load these weights and only run the evaluation")
    args = ap.parse_args(argv)

    import torch
    from . import Context

    ctx = Context(0)
    if args.eval_only:
        ctx.sizer_load(args.eval_only)
        rep = {"weights": args.eval_only,
               "eval": evaluate(ctx, args.eval_traces, args.seed + 1, *args.eval_wi_log2)}
        print(json.dumps(rep))
        return 0
    t0 = time.time()
    x, y = build_dataset(ctx, args.traces, args.seed, *args.wi_log2)
    t_data = time.time() - t0
    n_val = max(1, int(args.traces * args.val_frac))
    xt, yt, xv, yv = x[n_val:], y[n_val:], x[:n_val], y[:n_val]
    t0 = time.time()
    loss = ctx.sizer_train(xt.contiguous(), yt.contiguous(), epochs=args.epochs,
                           batch=args.batch, lr=args.lr, seed=args.seed)
    t_train = time.time() - t0
    pv = torch.zeros_like(yv)
    ctx.sizer_predict(xv.contiguous(), pv)
    err = (pv - yv).cpu().numpy()
    # margin: the (1 - target) quantile of the under-prediction at skip 10
    under = -err[:, 10]
    margin = float(max(0.0, np.quantile(under, 1.0 - args.overflow_target)))
    ctx.sizer_set_margin(margin)
    ctx.sizer_save(args.out)
    rep = {"traces": args.traces, "train_mse_normalized": loss,
           "val_mae_log2": [float(v) for v in np.abs(err).mean(0)],
           "margin_log2": margin, "data_s": t_data, "train_s": t_train, "weights": args.out}
    if args.eval_traces:
        rep["eval"] = evaluate(ctx, args.eval_traces, args.seed + 1, *args.eval_wi_log2)
    print(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
