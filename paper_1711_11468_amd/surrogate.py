"""Learned warm start: a 4-level 3D U-Net that maps a solid mask to the
steady velocity field of the body-force-driven flow, trained on the GPU by
the library's own BF16 MFMA kernels (forward, data gradient, weight
gradient, Adam), and used to start the solver from equilibrium at the
predicted velocity.  The solver still decides convergence: it iterates from the
prediction until its own residual criterion is met.

Network (channels-last, circular padding everywhere since the porous boxes
are periodic):
  encoder level l (l = 0..3, channels 16, 32, 64, 64): two 3x3x3 convs with
  leaky ReLU; between levels a stride-2 3x3x3 conv; decoder level l (2..0):
  nearest-neighbour upsampling of the coarser output, channel concatenation
  with the encoder output of level l, two 3x3x3 convs; head: 1x1x1 conv to
  3 channels (float32, no activation).
Input channels (padded to 16): solid indicator, fluid indicator, d/DMAX and
(d/DMAX)^2, with d the distance to the nearest solid voxel clamped at DMAX
(in a pore the Stokes velocity grows with the squared wall distance, which
the first convolutions cannot measure across a pore on their own).
Output: u * nu / (g * scale) — in the Stokes regime the steady velocity is
proportional to g/nu, so the network learns a geometry-only field; the
per-geometry scale (see ``kc_scale``) takes out the porosity dependence of
the permeability, which spans ~40x over the porosities trained on.
"""
from __future__ import annotations

import math
import os

import numpy as np

from . import nn

CH = (16, 32, 64, 64)
SLOPE = 0.1
CIN = 16
NFEAT = 4       # used input channels
DMAX = 12.0     # distance clamp of the distance features (lattice units)


def kc_scale(porosity: float) -> float:
    """Kozeny-Carman porosity factor phi^3 / (1 - phi)^2: the permeability
    of a packing of given grain size scales with it, so velocities divided
    by it vary little across porosities."""
    phi = min(max(float(porosity), 1e-3), 0.999)
    return phi ** 3 / (1.0 - phi) ** 2


class Conv:
    def __init__(self, name, c_in, c_out, stride=1, taps=27, act=True, c_store=None, out_f32=False):
        self.name, self.c_in, self.c_out = name, c_in, c_out
        self.stride, self.taps, self.act = stride, taps, act
        self.c_store = c_out if c_store is None else c_store
        self.out_f32 = out_f32

    def desc(self, batch, d):
        return nn.desc(batch, d, d, d, self.c_in, self.c_out, self.c_store, self.stride, self.taps,
                       self.act, SLOPE, self.out_f32)


def _layers():
    c0, c1, c2, c3 = CH
    return [
        Conv("e0a", CIN, c0), Conv("e0", c0, c0),
        Conv("d1", c0, c1, stride=2), Conv("e1a", c1, c1), Conv("e1", c1, c1),
        Conv("d2", c1, c2, stride=2), Conv("e2a", c2, c2), Conv("e2", c2, c2),
        Conv("d3", c2, c3, stride=2), Conv("e3a", c3, c3), Conv("e3", c3, c3),
        Conv("u2a", c3 + c2, c2), Conv("u2", c2, c2),
        Conv("u1a", c2 + c1, c1), Conv("u1", c1, c1),
        Conv("u0a", c1 + c0, c0), Conv("u0", c0, c0),
        Conv("head", c0, 16, taps=1, act=False, c_store=3, out_f32=True),
    ]


class UNet:
    """Parameters (float32 masters, bf16 copies, Adam moments) on the GPU."""

    def __init__(self, device=None, seed=0, u_scale=1.0):
        import torch
        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.layers = _layers()
        self.u_scale = float(u_scale)
        self.t = 0
        rng = np.random.default_rng(seed)
        self.p = {}
        # every parameter tensor, gradient, moment and bf16 copy is a view
        # into one flat buffer of its kind (tensors start 64 elements
        # apart at least, 16-byte aligned; the gaps stay zero), so one
        # element-wise Adam launch updates the whole network
        self._offsets = {}
        total = 0
        for L in self.layers:
            nw = L.taps * L.c_out * L.c_in
            self._offsets[L.name] = (total, total + -(-nw // 64) * 64)
            total += -(-nw // 64) * 64 + -(-L.c_out // 64) * 64
        d = self.device
        self.flat = {k: torch.zeros(total, dtype=torch.float32, device=d) for k in ("p", "g", "m", "v")}
        self.flat["p16"] = torch.zeros(total, dtype=torch.bfloat16, device=d)
        for L in self.layers:
            fan_in = L.taps * L.c_in
            std = math.sqrt(2.0 / fan_in) if L.act else 0.1 / math.sqrt(fan_in)
            w = rng.normal(0.0, std, size=(L.taps, L.c_out, L.c_in)).astype(np.float32)
            if L.name == "head":
                w[:, 3:, :] = 0.0           # padded output channels stay zero
            if L.name == "e0a":
                w[:, :, NFEAT:] = 0.0       # padded input channels carry zeros anyway
            self._add(L.name, w, np.zeros(L.c_out, np.float32))

    def _add(self, name, w, b):
        ow, ob = self._offsets[name]
        nw, nb = w.size, b.size
        F = self.flat
        q = {}
        for key, buf, off, n, shape in (("w", "p", ow, nw, w.shape), ("b", "p", ob, nb, b.shape),
                                        ("dw", "g", ow, nw, w.shape), ("db", "g", ob, nb, b.shape),
                                        ("mw", "m", ow, nw, w.shape), ("mb", "m", ob, nb, b.shape),
                                        ("vw", "v", ow, nw, w.shape), ("vb", "v", ob, nb, b.shape),
                                        ("w16", "p16", ow, nw, w.shape), ("b16", "p16", ob, nb, b.shape)):
            q[key] = F[buf][off:off + n].view(shape)
        q["w"].copy_(self.torch.from_numpy(w))
        q["b"].copy_(self.torch.from_numpy(b))
        self.p[name] = q
        nn.to_bf16(q["w"], q["w16"])

    # -- persistence ----------------------------------------------------------
    def state_dict(self):
        out = {"u_scale": np.array([self.u_scale], np.float64), "t": np.array([self.t], np.int64)}
        for k, v in self.p.items():
            out[k + ".w"] = v["w"].cpu().numpy()
            out[k + ".b"] = v["b"].cpu().numpy()
        return out

    def save(self, path):
        np.savez(path, **self.state_dict())

    @classmethod
    def load(cls, path, device=None):
        data = np.load(path, allow_pickle=False)
        net = cls(device=device, u_scale=float(data["u_scale"][0]))
        net.t = int(data["t"][0])
        for k in net.p:
            net.p[k]["w"].copy_(net.torch.from_numpy(data[k + ".w"]))
            net.p[k]["b"].copy_(net.torch.from_numpy(data[k + ".b"]))
            nn.to_bf16(net.p[k]["w"], net.p[k]["w16"])
        return net

    # -- buffers ----------------------------------------------------------------
    def _buffers(self, batch, n):
        key = (batch, n)
        if getattr(self, "_bkey", None) == key:
            return self._buf
        torch = self.torch
        d = self.device
        bf = torch.bfloat16
        f32 = torch.float32
        sizes = {0: n, 1: n // 2, 2: n // 4, 3: n // 8}
        vox = {l: batch * sizes[l] ** 3 for l in sizes}
        acts = {
            "x0": (0, CIN), "e0a": (0, CH[0]), "e0": (0, CH[0]), "d1": (1, CH[1]), "e1a": (1, CH[1]),
            "e1": (1, CH[1]), "d2": (2, CH[2]), "e2a": (2, CH[2]), "e2": (2, CH[2]), "d3": (3, CH[3]),
            "e3a": (3, CH[3]), "e3": (3, CH[3]), "c2": (2, CH[3] + CH[2]), "u2a": (2, CH[2]),
            "u2": (2, CH[2]), "c1": (1, CH[2] + CH[1]), "u1a": (1, CH[1]), "u1": (1, CH[1]),
            "c0": (0, CH[1] + CH[0]), "u0a": (0, CH[0]), "u0": (0, CH[0]),
        }
        b = {"a": {}, "g": {}, "sizes": sizes, "vox": vox}
        for name, (lvl, c) in acts.items():
            b["a"][name] = torch.empty(vox[lvl] * c, dtype=bf, device=d)
            if name != "x0":
                b["g"][name] = torch.empty(vox[lvl] * c, dtype=f32, device=d)
        b["out"] = torch.empty(vox[0] * 3, dtype=f32, device=d)
        b["dist"] = torch.empty(2 * vox[0], dtype=f32, device=d)
        b["dpre"] = torch.empty(vox[0] * max(CH[1] + CH[0], 16), dtype=bf, device=d)
        b["dpre_head"] = torch.empty(vox[0] * 16, dtype=bf, device=d)
        wsz = 0
        maxw = 0
        for L in self.layers:
            wsz = max(wsz, nn.wgrad_workspace(L.desc(batch, sizes[self._level_in(L.name)])))
            maxw = max(maxw, L.taps * L.c_in * L.c_out)
        b["ws"] = torch.empty(wsz // 4 + 1, dtype=f32, device=d)
        b["wt"] = torch.empty(maxw, dtype=bf, device=d)
        b["loss"] = torch.zeros(1, dtype=f32, device=d)
        b["loss_ws"] = torch.empty(4096, dtype=f32, device=d)
        # larger dpre for the biggest pre-activation (any level)
        b["dpre"] = torch.empty(max(vox[l] * c for (l, c) in acts.values()), dtype=bf, device=d)
        self._buf, self._bkey = b, key
        return b

    @staticmethod
    def _level_in(name):
        return {"e0a": 0, "e0": 0, "d1": 0, "e1a": 1, "e1": 1, "d2": 1, "e2a": 2, "e2": 2, "d3": 2,
                "e3a": 3, "e3": 3, "u2a": 2, "u2": 2, "u1a": 1, "u1": 1, "u0a": 0, "u0": 0,
                "head": 0}[name]

    def conv_flops(self, batch, n, train=False):
        """Multiply-add flops (2 per MAC) of the convolutions for one forward
        pass, or for a training step (forward, weight gradient and data
        gradient of every layer except the first, which has no input
        gradient).  Channel counts as the network defines them; the head
        counts its 3 stored outputs."""
        sizes = {0: n, 1: n // 2, 2: n // 4, 3: n // 8}
        fwd = first = 0
        for L in self.layers:
            m_out = batch * (sizes[self._level_in(L.name)] // L.stride) ** 3
            f = 2 * L.taps * L.c_in * L.c_store * m_out
            fwd += f
            if L.name == "e0a":
                first = f
        return 3 * fwd - first if train else fwd

    # -- forward ----------------------------------------------------------------
    def forward(self, mask_u8, batch, n, fuse_concat=False):
        """mask_u8: device uint8 [batch*n^3]; returns the float32 output
        [batch*n^3][3] (normalised units).  fuse_concat: the decoder's first
        layers read the up-sampled coarse tensor and the skip tensor directly
        instead of their concatenation (inference; the backward pass needs
        the concatenations, so training keeps them)."""
        assert n % 16 == 0, "grid edge must be a multiple of 16"
        b = self._buffers(batch, n)
        A = b["a"]
        S = b["sizes"]
        nn.prepare_input_dist(mask_u8, A["x0"], batch, n, CIN, DMAX, b["dist"])
        L = {l.name: l for l in self.layers}

        def conv(name, src, dst):
            lyr = L[name]
            nn.conv_fwd(lyr.desc(batch, S[self._level_in(name)]), src, self.p[name]["w16"],
                        self.p[name]["b"], dst)

        conv("e0a", A["x0"], A["e0a"]); conv("e0", A["e0a"], A["e0"])
        conv("d1", A["e0"], A["d1"]); conv("e1a", A["d1"], A["e1a"]); conv("e1", A["e1a"], A["e1"])
        conv("d2", A["e1"], A["d2"]); conv("e2a", A["d2"], A["e2a"]); conv("e2", A["e2a"], A["e2"])
        conv("d3", A["e2"], A["d3"]); conv("e3a", A["d3"], A["e3a"]); conv("e3", A["e3a"], A["e3"])
        def upcat_conv(name, coarse, c_coarse, skip, cat, lvl, c_skip):
            lyr = L[name]
            dsc = lyr.desc(batch, S[lvl])
            if fuse_concat and S[lvl] % 16 == 0:
                nn.conv_fwd_upcat(dsc, coarse, c_coarse, skip, self.p[name]["w16"], self.p[name]["b"],
                                  A[name])
            else:
                nn.up_concat(coarse, skip, cat, batch, S[lvl], S[lvl], S[lvl], c_coarse, c_skip)
                conv(name, cat, A[name])

        upcat_conv("u2a", A["e3"], CH[3], A["e2"], A["c2"], 2, CH[2]); conv("u2", A["u2a"], A["u2"])
        upcat_conv("u1a", A["u2"], CH[2], A["e1"], A["c1"], 1, CH[1]); conv("u1", A["u1a"], A["u1"])
        upcat_conv("u0a", A["u1"], CH[1], A["e0"], A["c0"], 0, CH[0]); conv("u0", A["u0a"], A["u0"])
        conv("head", A["u0"], b["out"])
        return b["out"]

    # -- backward ---------------------------------------------------------------
    def backward(self, batch, n, dpre_head):
        """Gradients of all parameters given the head's pre-activation
        gradient (bf16 [batch*n^3][16]).  Call after forward()."""
        b = self._buffers(batch, n)
        A, G, S = b["a"], b["g"], b["sizes"]
        L = {l.name: l for l in self.layers}
        dpre = b["dpre"]

        def back(name, x_in, dy, g_in, accumulate=False):
            lyr = L[name]
            dsc = lyr.desc(batch, S[self._level_in(name)])
            nn.conv_wgrad(dsc, x_in, dy, self.p[name]["dw"], self.p[name]["db"], b["ws"])
            if g_in is not None:
                nn.conv_dgrad(dsc, dy, self.p[name]["w16"], b["wt"], g_in, accumulate)

        def act_back(name, x_in, g_in, accumulate=False):
            n_el = A[name].numel()
            d = dpre[:n_el]
            nn.lrelu_bwd(G[name], A[name], d, SLOPE)
            back(name, x_in, d, g_in, accumulate)

        back("head", A["u0"], dpre_head, G["u0"])
        act_back("u0", A["u0a"], G["u0a"])
        act_back("u0a", A["c0"], G["c0"])
        nn.split_down(G["c0"], G["u1"], G["e0"], batch, S[0], S[0], S[0], CH[1], CH[0])
        act_back("u1", A["u1a"], G["u1a"])
        act_back("u1a", A["c1"], G["c1"])
        nn.split_down(G["c1"], G["u2"], G["e1"], batch, S[1], S[1], S[1], CH[2], CH[1])
        act_back("u2", A["u2a"], G["u2a"])
        act_back("u2a", A["c2"], G["c2"])
        nn.split_down(G["c2"], G["e3"], G["e2"], batch, S[2], S[2], S[2], CH[3], CH[2])
        act_back("e3", A["e3a"], G["e3a"])
        act_back("e3a", A["d3"], G["d3"])
        act_back("d3", A["e2"], G["e2"], accumulate=True)
        act_back("e2", A["e2a"], G["e2a"])
        act_back("e2a", A["d2"], G["d2"])
        act_back("d2", A["e1"], G["e1"], accumulate=True)
        act_back("e1", A["e1a"], G["e1a"])
        act_back("e1a", A["d1"], G["d1"])
        act_back("d1", A["e0"], G["e0"], accumulate=True)
        act_back("e0", A["e0a"], G["e0a"])
        act_back("e0a", A["x0"], None)

    def loss_and_grad(self, target, mask_u8, batch, n):
        b = self._buffers(batch, n)
        nn.masked_mse(b["out"], target, mask_u8, b["dpre_head"], b["loss"], b["loss_ws"])
        return b["loss"], b["dpre_head"]

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step of every parameter: a single launch over the flat
        buffers (the update is element-wise, and the zero gaps between
        tensors stay zero)."""
        self.t += 1
        F = self.flat
        nn.adam_step(F["p"], F["g"], F["m"], F["v"], F["p16"], lr, beta1, beta2, eps, self.t)

    def train_step(self, mask_u8, target, batch, n, lr=1e-3):
        self.forward(mask_u8, batch, n)
        loss, dpre_head = self.loss_and_grad(target, mask_u8, batch, n)
        self.backward(batch, n, dpre_head)
        self.adam(lr)
        return loss

    def predict_velocity(self, mask_u8, n, g_over_nu, porosity, out_u=None):
        """Velocity field [3][n^3] float64 on the device for one geometry:
        (g/nu) * kc_scale(porosity) * u_scale * network output on fluid
        voxels, 0 on solids."""
        out = self.forward(mask_u8, 1, n, fuse_concat=True)
        if out_u is None:
            out_u = self.torch.empty(3 * n ** 3, dtype=self.torch.float64, device=self.device)
        nn.velocity_out(out, mask_u8, g_over_nu * kc_scale(porosity) * self.u_scale, out_u)
        return out_u
