"""Kernel studies on the paper's benchmark geometries (one GPU).

1. Every sweep form on the paper's channel of 500 x 100 x 100 nodes
   (Sect. 4.2 uses it for all kernel comparisons; 4,802,000 fluid nodes).
2. The staircase pipe of the same size (Sect. 2), every form but AoS.
3. The `blocks` geometry (Sect. 2; the paper's Fig. 4 study): cubic
   obstacles of growing edge inside the same 500 x 100 x 100 channel, gap
   equal to the edge, for the direct and list kernels.

    python -m paper_1711_11468_amd.study [--steps 200] [--out study.json]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs as I
from . import lbm

PHYS = dict(tau_plus=0.8, magic=3.0 / 16.0, g=(1e-6, 0.0, 0.0))

FORMS = [
    ("os-pull-soa", dict()),
    ("os-pull-aos", dict(layout="aos")),
    ("os-pull-soa-halfway", dict(bounce="halfway")),
    ("os-push-soa", dict(propagation="push")),
    ("list-os-pull-soa", dict(addressing="list", bounce="halfway")),
    ("list-os-push-soa", dict(addressing="list", bounce="halfway", propagation="push")),
    ("list-os-pull-aos", dict(addressing="list", bounce="halfway", layout="aos")),
    ("list-ria-os-pull-soa", dict(addressing="ria", bounce="halfway")),
    ("aa-soa", dict(propagation="aa")),
    ("list-aa-soa", dict(addressing="list", bounce="halfway", propagation="aa")),
    ("list-aa-ria-soa", dict(addressing="ria", bounce="halfway", propagation="aa")),
]


def time_form(mask, steps, warmup, **kw):
    import torch
    lat = lbm.Lattice(mask, residual=False, **PHYS, **kw)
    lat.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nf = lat.n_fluid
    bytes_step = lat.sizes.bytes_per_update * lat.sizes.n_sites
    out = {"ms_per_step": ms, "mflups": nf / (ms * 1e-3) / 1e6,
           "gbs": bytes_step / (ms * 1e-3) / 1e9,
           "bytes_per_fluid_update": bytes_step / nf, "fluid_nodes": nf}
    del lat
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch  # noqa: F401
    res = {"channel_500x100x100": {}, "pipe_500x100x100": {}, "blocks_500x100x100": []}
    ch = I.channel_mask(500, 100, 100)
    for name, kw in FORMS:
        r = time_form(ch, args.steps, args.warmup, **kw)
        res["channel_500x100x100"][name] = r
        print("channel %-20s %8.1f MFLUP/s  %6.0f GB/s  %.1f B/FLUP" % (
            name, r["mflups"], r["gbs"], r["bytes_per_fluid_update"]), flush=True)
    pipe = I.pipe_mask(500, 100, 100)
    for name, kw in FORMS:
        if name in ("os-pull-aos", "list-os-pull-aos"):
            continue
        r = time_form(pipe, args.steps, args.warmup, **kw)
        res["pipe_500x100x100"][name] = r
        print("pipe    %-20s %8.1f MFLUP/s  %6.0f GB/s  %.1f B/FLUP" % (
            name, r["mflups"], r["gbs"], r["bytes_per_fluid_update"]), flush=True)
    for edge in (1, 2, 4, 8, 16):
        m = I.blocks_mask(500, 100, 100, block=edge, gap=edge)
        row = {"block": edge, "gap": edge, "fluid_fraction": float((m == 0).mean())}
        for name, kw in FORMS:
            if name in ("os-pull-aos", "list-os-pull-aos"):
                continue
            row[name] = time_form(m, args.steps, args.warmup, **kw)
        res["blocks_500x100x100"].append(row)
        print("blocks %2d: fluid %.3f | " % (edge, row["fluid_fraction"]) + " | ".join(
            "%s %.0f" % (k, v["mflups"]) for k, v in row.items() if isinstance(v, dict)), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
