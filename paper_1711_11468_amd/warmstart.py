"""Learned warm start pipeline: porous geometries, steady-state labels from
the solver itself, training of the U-Net with the library's kernels, and the
warm-versus-cold comparison of time to steady state.

Geometries: fully periodic boxes of overlapping spheres (radii uniform in
[4, 8] lattice units) placed until a target porosity, the porosity itself
drawn uniformly from [0.35, 0.70] per seed.  Physics: D3Q19 TRT,
tau+ = 0.8, Lambda = 3/16, body force g_x = 1e-6, half-way bounce-back on
the fluid-node list, FP64 populations.  Steady state: velocity residual
||u(t) - u(t-100)|| / ||u(t)|| < 1e-6, checked every 100 steps.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import lbm

PHYS = dict(tau_plus=0.8, magic=3.0 / 16.0, g=(1e-6, 0.0, 0.0))
NU = (PHYS["tau_plus"] - 0.5) / 3.0
G_OVER_NU = PHYS["g"][0] / NU
TOL = 1e-6


def geometry(seed: int, n: int, lo=0.35, hi=0.70, rmin=4.0, rmax=8.0):
    """Porous box of edge n for a seed: (mask uint8 (n,n,n), porosity)."""
    phi_target = lo + (hi - lo) * I.SplitMix64(seed ^ 0x5EED5EED).uniform()
    mask, phi, _ = I.spheres_mask(n, n, n, seed, phi_target, rmin, rmax)
    return mask, phi


def _geometry_star(args):
    return geometry(*args)


def geometries(seeds, n, workers=8):
    """Masks for many seeds, generated in a process pool (host work)."""
    if workers <= 1:
        return [geometry(s, n) for s in seeds]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_geometry_star, [(s, n) for s in seeds], chunksize=8)


def solve(mask, u0=None, tol=TOL, max_steps=200_000, storage="f64"):
    """Run the solver from rest (u0 None) or from equilibrium at velocity
    u0 ([3][N] float64 device tensor) to the residual target.
    Returns (lattice, steps, seconds, residual, reason)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = lbm.Lattice(mask, addressing="list", bounce="halfway", storage=storage, **PHYS)
    if u0 is not None:
        lat.init_fields(None, u0)
    steps, r, why = lat.run_to_steady(tol, max_steps=max_steps)
    torch.cuda.synchronize()
    return lat, steps, time.perf_counter() - t0, r, why


def labels_from(lat, u_scale):
    """Steady velocity of a solved lattice in network units
    (u * nu / g / u_scale), float32 [N][3] on the device."""
    st = lat.macroscopic(fields=True)
    u = st["u"]                                     # [3][N] float64
    return (u.t().contiguous() / (G_OVER_NU * u_scale)).float().reshape(-1)


def make_dataset(seeds, n, u_scale, workers=8, log=None):
    """Masks (uint8 [S][n^3]) and labels (float32 [S][n^3*3]) on the GPU."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    geo = geometries(seeds, n, workers)
    masks = torch.empty((len(seeds), n ** 3), dtype=torch.uint8, device=dev)
    labels = torch.empty((len(seeds), n ** 3 * 3), dtype=torch.float32, device=dev)
    info = []
    for k, (m, phi) in enumerate(geo):
        lat, steps, secs, r, why = solve(m)
        masks[k].copy_(torch.from_numpy(m.reshape(-1)))
        labels[k].copy_(labels_from(lat, u_scale))
        info.append({"seed": int(seeds[k]), "porosity": phi, "steps": steps, "seconds": secs,
                     "reason": why})
        del lat
        if log and (k % 100 == 0 or k == len(geo) - 1):
            log("dataset %d/%d: porosity %.3f, %d steps, %.3f s" % (k + 1, len(geo), phi, steps, secs))
    return masks, labels, info


def train(net, masks, labels, n, epochs, batch=4, lr=1e-3, seed=0, log=None):
    """Adam on shuffled mini-batches; returns the per-epoch mean losses."""
    import torch
    S = masks.shape[0]
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        order = rng.permutation(S)
        losses = []
        step_lr = lr * (0.5 ** (ep // max(1, epochs // 3)))
        for i in range(0, S - batch + 1, batch):
            idx = torch.from_numpy(order[i:i + batch]).to(masks.device)
            m = masks.index_select(0, idx).reshape(-1)
            t = labels.index_select(0, idx).reshape(-1)
            loss = net.train_step(m, t, batch, n, lr=step_lr)
            losses.append(loss.clone())
        mean = float(torch.stack(losses).mean().item()) if losses else float("nan")
        history.append(mean)
        if log:
            log("epoch %d: loss %.5f (lr %.1e)" % (ep, mean, step_lr))
    return history


def compare(net, seed, n):
    """Cold (rest) versus warm (network prediction) start on one geometry."""
    import torch
    mask, phi = geometry(seed, n)
    lat_c, steps_c, secs_c, r_c, why_c = solve(mask)
    u_cold = lat_c.macroscopic(fields=True)["u"].clone()
    del lat_c
    dev = u_cold.device
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = torch.from_numpy(mask.reshape(-1)).to(dev)
    u_pred = net.predict_velocity(m, n, G_OVER_NU)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    lat_w, steps_w, secs_w, r_w, why_w = solve(mask, u0=u_pred)
    u_warm = lat_w.macroscopic(fields=True)["u"]
    fl = torch.from_numpy(mask.reshape(-1) == 0).to(dev)
    pred_err = float(((u_pred.view(3, -1) - u_cold)[:, fl].norm() / u_cold[:, fl].norm()).item())
    agree = float(((u_warm - u_cold)[:, fl].norm() / u_cold[:, fl].norm()).item())
    return {"seed": seed, "porosity": phi, "cold_steps": steps_c, "cold_s": secs_c,
            "warm_steps": steps_w, "warm_s": secs_w + t_inf, "inference_s": t_inf,
            "prediction_rel_l2": pred_err, "warm_vs_cold_rel_l2": agree,
            "cold_reason": why_c, "warm_reason": why_w}
