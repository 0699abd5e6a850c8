"""Train the warm-start network on solver-generated steady states and
compare warm and cold starts on held-out geometries.

    python -m paper_1711_11468_amd.train_warmstart --train 2000 --n 64 \\
        --epochs 20 --eval 20 --eval-n 128 --out weights.npz --summary eval.json

Training data: seeds 0 .. train-1 at edge n (porosity uniform in
[0.35, 0.70], sphere radii in [4, 8]), each solved by the FP64 list sweep to
residual 1e-6; labels are u * nu / (g * kc_scale(porosity)).
Evaluation: seeds 100000 .. 100000+eval-1 at edge eval-n; each geometry is
solved from rest and from the network's prediction (inference included in
the warm time); both runs stop at residual 1e-6.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def log(msg):
    print("[warmstart %s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--eval", type=int, default=20)
    ap.add_argument("--eval-n", type=int, default=128)
    ap.add_argument("--out", default="unet_porous.npz")
    ap.add_argument("--summary", default=None)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--load", default=None, help="skip training, evaluate these weights")
    args = ap.parse_args(argv)

    import numpy as np
    import torch
    from . import warmstart as WS
    from .surrogate import UNet

    summary = {"args": vars(args)}
    if args.load:
        net = UNet.load(args.load)
    else:
        t0 = time.perf_counter()
        masks, labels, info = WS.make_dataset(list(range(args.train)), args.n,
                                              workers=args.workers, log=log)
        t_data = time.perf_counter() - t0
        steps = [r["steps"] for r in info]
        log("dataset: %d geometries in %.1f s, solver steps median %d (max %d)"
            % (args.train, t_data, int(np.median(steps)), max(steps)))
        net = UNet(seed=0)
        t0 = time.perf_counter()
        hist = WS.train(net, masks, labels, args.n, args.epochs, args.batch, args.lr, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        net.save(args.out)
        log("trained %d epochs in %.1f s, saved %s" % (args.epochs, t_train, args.out))
        summary.update({"dataset_seconds": t_data, "train_seconds": t_train, "loss_history": hist,
                        "dataset_steps_median": float(np.median(steps))})
        del masks, labels
        torch.cuda.empty_cache()
    rows = []
    for k in range(args.eval):
        r = WS.compare(net, 100000 + k, args.eval_n)
        rows.append(r)
        log("eval %d: cold %d steps %.3f s | warm %d steps %.3f s (inference %.4f s) | "
            "prediction err %.3f | warm-vs-cold %.2e" % (
                r["seed"], r["cold_steps"], r["cold_s"], r["warm_steps"], r["warm_s"],
                r["inference_s"], r["prediction_rel_l2"], r["warm_vs_cold_rel_l2"]))
    if rows:
        step_ratio = [r["cold_steps"] / r["warm_steps"] for r in rows]
        time_ratio = [r["cold_s"] / r["warm_s"] for r in rows]
        summary["eval"] = rows
        summary["median_step_speedup"] = float(np.median(step_ratio))
        summary["median_time_speedup"] = float(np.median(time_ratio))
        summary["median_prediction_rel_l2"] = float(np.median([r["prediction_rel_l2"] for r in rows]))
        summary["max_warm_vs_cold_rel_l2"] = float(max(r["warm_vs_cold_rel_l2"] for r in rows))
        log("median speed-up: steps %.2fx, wall time %.2fx; median prediction error %.3f"
            % (summary["median_step_speedup"], summary["median_time_speedup"],
               summary["median_prediction_rel_l2"]))
    if args.summary:
        with open(args.summary, "w") as fh:
            json.dump(summary, fh, indent=1)
    return summary


if __name__ == "__main__":
    main(sys.argv[1:])
