#!/usr/bin/env python3
"""Throughput of the fused D3Q19 TRT pull sweep on one MI355X.

Workload (the headline line): channel of 512 x 512 x 512 nodes (walls on the
y and z faces, x periodic), body force g_x = 1e-6, tau+ = 0.8,
Lambda = 3/16, double-precision populations, structure-of-arrays, direct
addressing, full-way bounce-back, started at rest.  A step is one fused
stream-collide launch (A -> B, swap); every 100th step is the same sweep with
the diagnostics (mass, momentum, max |u|, residual, non-finite count) of the
state it reads fused in, inside the timed region.

Reported: MFLUP/s (fluid lattice updates per second), the HBM roofline of
the sweep kernel (algorithmic bytes per launch / mean launch time from HIP
events recorded on the sweep's stream, against the 8 TB/s HBM3E peak), the
memory micro-benchmarks (copy, copy-19, copy-19-nt, update-19), secondary
variants (AoS, list addressing on a porous box, shifted FP32/FP16 storage)
and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--headline-only]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MFLUP/s + % HBM roofline; time-to-steady-state, surrogate warm vs cold"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
PHYS = dict(tau_plus=0.8, magic=3.0 / 16.0, g=(1e-6, 0.0, 0.0))


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_sweeps(lat, steps, warmup, diag_every=100):
    """Warm up, then time `steps` sweeps; every `diag_every`-th one also
    returns the diagnostics (fused into the sweep where the form allows it).
    Returns (total_ms, per-launch ms of the plain sweeps)."""
    import torch
    stream = lat.stream
    lat.step(warmup)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    timed = []
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(steps):
        if diag_every and (k + 1) % diag_every == 0:
            lat.step_diag()
            continue
        ev[k][0].record(stream)
        lat.step(1)
        ev[k][1].record(stream)
        timed.append(k)
    t1.record(stream)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1)
    per = [ev[k][0].elapsed_time(ev[k][1]) for k in timed]
    return total, per


def run_variant(mask, steps, warmup, diag=True, **kw):
    from paper_1711_11468_amd import lbm
    import torch
    lat = lbm.Lattice(mask, **PHYS, **kw)
    total, per = time_sweeps(lat, steps, warmup, 100 if diag else 0)
    st = lat.macroscopic()
    nf = lat.n_fluid
    res = {
        "mflups": nf * steps / (total * 1e-3) / 1e6,
        "ms_per_step": total / steps,
        "kernel_ms": float(np.mean(per)),
        "bytes_per_update": lat.sizes.bytes_per_update,
        "n_sites": lat.sizes.n_sites,
        "n_runs": lat.sizes.n_runs,
        "n_fluid": nf,
        "mass_rel_drift": abs(st["mass"] - lat.sizes.n_sites) / lat.sizes.n_sites
        if kw.get("addressing", "direct") == "direct" and kw.get("bounce", "fullway") == "fullway" else None,
    }
    algo_bytes = lat.sizes.bytes_per_update * lat.sizes.n_sites
    res["achieved_gbs"] = algo_bytes / (res["kernel_ms"] * 1e-3) / 1e9
    res["b_per_fluid_update"] = algo_bytes / nf
    return lat, res


def membench(lat, reps=20):
    """Memory micro-benchmarks on the lattice's own A/B buffers."""
    import torch
    from paper_1711_11468_amd import lbm
    s = lat.sizes
    a = lat._t["pdf_a"]
    b = lat._t["pdf_b"]
    n = int(s.n_sites)
    stride = int(s.stride)
    out = {}
    # kind: (name, threads per workgroup, accesses per element: 2 = read and
    # write, 1 = read or write only)
    kinds = {0: ("copy", 256, 2), 1: ("copy-19", 256, 2), 2: ("copy-19-nt", 256, 2),
             3: ("update-19", 256, 2), 4: ("copy-v", 256, 2), 5: ("copy-4-v", 256, 2),
             6: ("copy-19-v", 256, 2), 7: ("copy-19-vp", 256, 2), 8: ("read-19-v", 256, 1),
             9: ("write-19-v", 256, 1)}
    for kind, (name, block, acc) in kinds.items():
        nn = n * 19 if kind in (0, 4) else n
        st = stride
        if kind == 5:  # four arrays spanning the same buffers
            st = stride * 19 // 4 // 2 * 2
            nn = st
        src = None if kind == 9 else a
        for _ in range(3):
            lbm.membench(kind, src, b, nn, st, block, lat.stream.cuda_stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        for _ in range(reps):
            lbm.membench(kind, src, b, nn, st, block, lat.stream.cuda_stream)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        elems = nn * (4 if kind == 5 else (1 if kind in (0, 4) else 19))
        out[name] = round(acc * 8.0 * elems / (ms * 1e-3) / 1e9, 1)
    return out


def warm_vs_cold(n=128, seeds=(100000, 100001, 100002)):
    """Time to steady state (residual 1e-6) on held-out 128^3 porous boxes,
    cold start versus the learned warm start (inference included)."""
    from paper_1711_11468_amd import warmstart as WS
    from paper_1711_11468_amd.surrogate import UNet
    path = os.path.join(ROOT, "paper_1711_11468_amd", "weights", "unet_porous64.npz")
    if not os.path.exists(path):
        return None
    net = UNet.load(path)
    rows = [WS.compare(net, s, n) for s in seeds]
    log("warm vs cold: %s" % [(r["cold_steps"], r["warm_steps"]) for r in rows])
    return {"workload": "porous box %d^3, overlapping spheres r in [4,8], porosity U[0.35,0.7], "
                        "list FP64, tau+=0.8, Lambda=3/16, g_x=1e-6, residual 1e-6" % n,
            "cold_steps_median": float(np.median([r["cold_steps"] for r in rows])),
            "warm_steps_median": float(np.median([r["warm_steps"] for r in rows])),
            "cold_s_median": float(np.median([r["cold_s"] for r in rows])),
            "warm_s_median": float(np.median([r["warm_s"] for r in rows])),
            "step_speedup_median": float(np.median([r["cold_steps"] / r["warm_steps"] for r in rows])),
            "prediction_rel_l2_median": float(np.median([r["prediction_rel_l2"] for r in rows]))}


def cnn_throughput(steps=10, which=("infer_128", "train_64x4")):
    """The warm-start network's BF16 MFMA convolutions: inference on one
    128^3 box and a training step on four 64^3 boxes (random weights and
    inputs; the work does not depend on the values), timed with HIP events
    on torch's current stream, where the network kernels run."""
    import torch
    from paper_1711_11468_amd.surrogate import UNet
    dev = torch.device("cuda")
    net = UNet(device=dev, seed=0)
    g = torch.Generator().manual_seed(0)
    out = {}
    for key, (B, n, train) in (("infer_128", (1, 128, False)), ("train_64x4", (4, 64, True))):
        if key not in which:
            continue
        mask = (torch.rand(B * n ** 3, generator=g) < 0.4).to(torch.uint8).to(dev)
        tgt = torch.randn(B * n ** 3 * 3, generator=g).to(dev)

        def once():
            if train:
                net.train_step(mask, tgt, B, n, lr=1e-4)
            else:
                net.forward(mask, B, n, fuse_concat=True)  # as predict_velocity runs it
        for _ in range(3):
            once()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            once()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        fl = net.conv_flops(B, n, train)
        tf = fl / (ms * 1e-3) / 1e12
        out[key] = {"ms": round(ms, 3), "conv_gflop": round(fl / 1e9, 2), "tflops": round(tf, 2),
                    "frac_bf16_dense_peak": round(tf / BF16_PEAK_TFLOPS, 5)}
    log("cnn: %s" % out)
    return out


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel), or None
    when the sweep sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sweep_soa_f64_channel512_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256_16"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    h = hashlib.sha256()
    for f in ("paper_1711_11468_amd/csrc/sweep.hip", "paper_1711_11468_amd/csrc/d3q19.hpp",
              "paper_1711_11468_amd/csrc/launch.hpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != vals.get("source_sha256_16"):
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline():
    """The oracle (plain C, as it stands) on bounded samples of the headline
    workload: sections of the same 512 x 512 channel cross-section (the duct
    flow is x-invariant, so every node does the same work), 12 updates each.
    Timed twice: the serial build on one core, and the OpenMP build of the
    same source (a parallel loop over nodes, identical results) on all the
    host cores this process may use (OMP_NUM_THREADS if set)."""
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)  # read when the OpenMP build loads
    from oracle import oracle as O
    from paper_1711_11468_amd import inputs as I
    steps = 12
    rows = {}
    for key, nx, omp in (("serial", 16, False), ("openmp", 64, True)):
        mask = I.channel_mask(nx, 512, 512)
        secs = O.time_run(mask, steps, PHYS["tau_plus"], PHYS["magic"], PHYS["g"], 0, omp=omp)
        nf = int((mask == 0).sum())
        rows[key] = (nf * steps / secs / 1e6, secs, nx)
        del mask
    model = cpu_model()
    v, secs, nx = rows["openmp"]
    v1, secs1, nx1 = rows["serial"]
    log("cpu baseline: %.2f MFLUP/s on %d threads, %.2f on one (%s)" % (v, threads, v1, model))
    return {"value": round(v, 3), "unit": "MFLUP/s", "cores": threads, "kind": "oracle",
            "sample": "channel %dx512x512 (same cross-section as 512^3), %d updates, %.1f s, "
                      "OpenMP build on %d threads; serial build: channel %dx512x512, %d updates, "
                      "%.1f s" % (nx, steps, secs, threads, nx1, steps, secs1),
            "single_thread_value": round(v1, 3), "nproc": os.cpu_count(), "cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="channel edge (headline: 512)")
    ap.add_argument("--headline-only", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cnn-only", choices=["infer_128", "train_64x4", "both"], default=None,
                    help="time only the warm-start network (for kernel traces)")
    ap.add_argument("--variants", default=None,
                    help="comma-separated variant names to run after the headline "
                         "(for counter runs); skips the warm-start and network sections")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; the multi-GPU path is not implemented "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_11468_amd import inputs as I
    from paper_1711_11468_amd import lbm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    lbm.load()
    if args.cnn_only:
        which = ("infer_128", "train_64x4") if args.cnn_only == "both" else (args.cnn_only,)
        print(json.dumps({"warm_start_network": cnn_throughput(which=which)}), flush=True)
        return
    n = args.n
    mask = I.channel_mask(n, n, n)
    log("headline: channel %d^3 SoA fp64" % n)
    lat, head = run_variant(mask, args.steps, args.warmup)
    log("headline done: %.0f MFLUP/s, kernel %.3f ms" % (head["mflups"], head["kernel_ms"]))
    mb = membench(lat)
    log("membench %s" % mb)
    del lat
    torch.cuda.empty_cache()

    variants = {}
    only = set(args.variants.split(",")) if args.variants else None
    wanted = lambda name: only is None or name in only  # noqa: E731
    if not args.headline_only:
        for name, kw in [("aos_f64", dict(layout="aos")),
                         ("soa_f32_shifted", dict(storage="f32s")),
                         ("soa_f16_shifted", dict(storage="f16s")),
                         ("soa_f16_shifted_stochastic", dict(storage="f16sr")),
                         ("soa_f64_halfway", dict(bounce="halfway")),
                         ("aa_soa_f64", dict(propagation="aa")),
                         ("push_soa_f64", dict(propagation="push")),
                         ("push_aos_f64", dict(propagation="push", layout="aos")),
                         ("aa_aos_f64", dict(propagation="aa", layout="aos"))]:
            if not wanted(name):
                continue
            log("variant %s" % name)
            lat, r = run_variant(mask, args.steps, args.warmup, **kw)
            variants[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
            del lat
            torch.cuda.empty_cache()
        spheres = [("list_spheres384_f64", dict(addressing="list", bounce="halfway")),
                   ("aa_list_spheres384_f64", dict(addressing="list", bounce="halfway",
                                                   propagation="aa")),
                   ("push_list_spheres384_f64", dict(addressing="list", bounce="halfway",
                                                     propagation="push")),
                   ("ria_spheres384_f64", dict(addressing="ria", bounce="halfway")),
                   ("aa_ria_spheres384_f64", dict(addressing="ria", bounce="halfway",
                                                  propagation="aa")),
                   ("direct_spheres384_f64", dict(addressing="direct", bounce="halfway")),
                   ("list_aos_spheres384_f64", dict(addressing="list", bounce="halfway",
                                                    layout="aos")),
                   ("aa_list_aos_spheres384_f64", dict(addressing="list", bounce="halfway",
                                                       layout="aos", propagation="aa")),
                   ("push_list_aos_spheres384_f64", dict(addressing="list", bounce="halfway",
                                                         layout="aos", propagation="push"))]
        spheres = [(name, kw) for name, kw in spheres if wanted(name)]
        if spheres:
            log("variant list 384^3 spheres")
            smask, phi, _ = I.spheres_mask(384, 384, 384, seed=0, porosity=0.4, rmin=8, rmax=16)
        for name, kw in spheres:
            lat, r = run_variant(smask, args.steps, args.warmup, **kw)
            r["porosity"] = phi
            variants[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
            del lat
            torch.cuda.empty_cache()

    extras = not args.headline_only and only is None
    steady = warm_vs_cold() if extras else None
    cnn = cnn_throughput() if extras else None
    cpu = None if args.no_cpu else cpu_baseline()
    achieved = head["achieved_gbs"]
    traffic = measured_traffic() if n == 512 else None
    line = {
        "metric": METRIC,
        "value": round(head["mflups"], 1),
        "unit": "MFLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "channel %dx%dx%d D3Q19 TRT fp64 pull sweep, SoA direct "
                               "addressing, full-way bounce-back walls, g_x=1e-6, tau+=0.8, "
                               "Lambda=3/16, rest start" % (n, n, n),
                   "nodes": n ** 3, "fluid_nodes": head["n_fluid"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_sweep_soa<StoreF64, FULLWAY>",
                     "algorithmic_bytes_per_launch": head["bytes_per_update"] * head["n_sites"],
                     "kernel_ms": round(head["kernel_ms"], 4),
                     "frac_of_copy19nt": round(achieved / mb["copy-19-nt"], 4)},
        "membench_gbs": mb,
        "variants": variants,
        "steady_state": steady,
        "warm_start_network": cnn,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
