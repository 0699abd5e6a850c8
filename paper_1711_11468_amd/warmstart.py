"""Learned warm start pipeline: porous geometries, steady-state labels from
the solver itself, training of the U-Net with the library's kernels, and the
warm-versus-cold comparison of time to steady state.

Geometries: fully periodic boxes of overlapping spheres (radii uniform in
[4, 8] lattice units) placed until a target porosity, the porosity itself
drawn uniformly from [0.35, 0.70] per seed.  Physics: D3Q19 TRT,
tau+ = 0.8, Lambda = 3/16, body force g_x = 1e-6, half-way bounce-back on
the fluid-node list, FP64 populations.  Steady state: velocity residual
||u(t) - u(t-100)|| / ||u(t)|| < 1e-6, checked every 100 steps and
confirmed over the next 37 (so that an acoustic oscillation whose period
divides 100 cannot pass for convergence).
Labels: u * nu / (g * kc_scale(porosity)), formed on the device by the
library's label kernel.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import lbm
from . import nn
from .surrogate import kc_scale

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


def labels_into(lat, mask_dev, porosity, out):
    """Steady velocity of a solved lattice in network units,
    u * nu / (g * kc_scale(porosity)), written by the label kernel into the
    float32 [N][3] device tensor ``out`` (0 on solids)."""
    u = lat.macroscopic(fields=True)["u"]           # [3][N] float64
    nn.velocity_labels(u, mask_dev, 1.0 / (G_OVER_NU * kc_scale(porosity)), out)


def make_dataset(seeds, n, workers=8, log=None, tol=TOL):
    """Masks (uint8 [S][n^3]) and labels (float32 [S][n^3*3]) on the GPU."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    geo = geometries(seeds, n, workers)
    masks = torch.empty((len(seeds), n ** 3), dtype=torch.uint8, device=dev)
    labels = torch.empty((len(seeds), n ** 3 * 3), dtype=torch.float32, device=dev)
    info = []
    for k, (m, phi) in enumerate(geo):
        lat, steps, secs, r, why = solve(m, tol=tol)
        masks[k].copy_(torch.from_numpy(m.reshape(-1)))
        labels_into(lat, masks[k], phi, labels[k])
        info.append({"seed": int(seeds[k]), "porosity": phi, "steps": steps, "seconds": secs,
                     "reason": why})
        del lat
        if log and (k % 100 == 0 or k == len(geo) - 1):
            log("dataset %d/%d: porosity %.3f, %d steps, %.3f s" % (k + 1, len(geo), phi, steps, secs))
    return masks, labels, info


def train(net, masks, labels, n, epochs, batch=4, lr=3e-4, seed=0, log=None, warmup=300):
    """Adam on shuffled mini-batches, the learning rate ramped up linearly
    over the first ``warmup`` steps and then following a cosine decay to
    zero; returns the per-epoch mean losses."""
    import torch
    S = masks.shape[0]
    rng = np.random.default_rng(seed)
    history = []
    per_epoch = max(1, (S - batch) // batch + 1)
    total = epochs * per_epoch
    it = 0
    for ep in range(epochs):
        order = rng.permutation(S)
        losses = []
        for i in range(0, S - batch + 1, batch):
            frac = it / max(1, total - 1)
            step_lr = lr * min(1.0, (it + 1) / warmup) * 0.5 * (1.0 + np.cos(np.pi * frac))
            it += 1
            idx = torch.from_numpy(order[i:i + batch]).to(masks.device)
            m = masks.index_select(0, idx).reshape(-1)
            t = labels.index_select(0, idx).reshape(-1)
            loss = net.train_step(m, t, batch, n, lr=step_lr)
            losses.append(loss.clone())
        # the per-step losses come back to the host once per epoch and are
        # averaged there
        mean = float(np.mean(torch.cat(losses).cpu().numpy())) if losses else float("nan")
        history.append(mean)
        if log:
            log("epoch %d: loss %.5f (lr now %.1e)" % (ep, mean, step_lr))
    return history


def cycle_mean_velocity(lat, k=4):
    """Velocity [3*N] averaged over the next k updates (the lattice moves on
    by k).  On porous geometries the converged state carries a corner limit
    cycle of period 2 (half-way bounce-back) or 4 (full-way) whose
    amplitude depends on the initial state; the mean over 4 updates
    removes it, so two converged runs can be compared."""
    acc = None
    for _ in range(k):
        lat.step(1)
        u = lat.macroscopic(fields=True)["u"].reshape(-1)
        acc = u.clone() if acc is None else acc.add_(u)
    return acc.div_(k)


def compare(net, seed, n):
    """Cold (rest) versus warm (network prediction) start on one geometry.
    The warm time includes the inference; both runs stop by the same
    convergence test.  Errors are relative L2 velocity norms against the cold-start
    steady field: the prediction's (the library's verify kernel on a
    lattice initialised with it, before any update) and the warm run's
    converged field's (4-update means of both, see cycle_mean_velocity)."""
    import torch
    mask, phi = geometry(seed, n)
    lat_c, steps_c, secs_c, r_c, why_c = solve(mask)
    u_cold = lat_c.macroscopic(fields=True)["u"].reshape(-1).clone()
    u_cold_mean = cycle_mean_velocity(lat_c)
    del lat_c
    dev = u_cold.device
    m = torch.from_numpy(mask.reshape(-1)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u_pred = net.predict_velocity(m, n, G_OVER_NU, phi)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    probe = lbm.Lattice(mask, addressing="list", bounce="halfway", **PHYS)
    probe.init_fields(None, u_pred)
    pred_err = probe.verify(lbm.VERIFY_REFERENCE, u_cold)["rel_l2"]
    del probe
    lat_w, steps_w, secs_w, r_w, why_w = solve(mask, u0=u_pred)
    agree_inst = lat_w.verify(lbm.VERIFY_REFERENCE, u_cold)["rel_l2"]
    u_warm_mean = cycle_mean_velocity(lat_w)
    fl = torch.from_numpy(mask.reshape(-1) == 0).to(dev).repeat(3)
    agree = float(((u_warm_mean - u_cold_mean)[fl].norm() / u_cold_mean[fl].norm()).item())
    return {"seed": seed, "porosity": phi, "cold_steps": steps_c, "cold_s": secs_c,
            "warm_steps": steps_w, "warm_s": secs_w + t_inf, "inference_s": t_inf,
            "prediction_rel_l2": pred_err, "warm_vs_cold_rel_l2": agree,
            "warm_vs_cold_rel_l2_instantaneous": agree_inst,
            "cold_reason": why_c, "warm_reason": why_w}
