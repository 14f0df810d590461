"""Learned registration initialiser (not part of the paper's method): an
8-layer CNN that proposes each patch's rigid correction from the pair
(observed patch, patch simulated from the current volume at the current
motion); the paper's NCC registration then refines every proposal and keeps
the unchanged motion when the proposal scores worse.

Training pairs come from the library's own forward model: the observed patch
is simulated at a reference motion, the second patch at that motion minus a
random offset (rotation <= 10 deg, translation <= 5 mm); the target is the
offset expressed in the patch's own frame (in-plane u, v, slice normal), with
rotations scaled by the patch half-diagonal (mm of displacement).  Every arithmetic step runs in libpvr.so (include/pvr_cnn.h); torch
holds the device buffers.
"""
from __future__ import annotations

import ctypes
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import pvr

# (cin, cout, stride) of the 8 convolutions
LAYERS = [(2, 32, 1), (32, 32, 2), (32, 64, 1), (64, 64, 2),
          (64, 64, 1), (64, 64, 2), (64, 64, 1), (64, 64, 1)]
SIDE = 64


def _final_hw() -> int:
    h = SIDE
    for _, _, s in LAYERS:
        h = (h - 1) // s + 1
    return h * h


HW = _final_hw()          # positions of the last feature map (8 x 8)


def macs_per_pair() -> int:
    """Multiply-accumulates of one forward pass (convolutions and head)."""
    h, total = SIDE, 0
    for cin, cout, s in LAYERS:
        h = (h - 1) // s + 1
        total += h * h * cout * 9 * cin
    return total + HW * 64 * 6
N_FC = HW * 64 * 6        # head weights [HW][64][6]


def activation_bytes_per_pair() -> int:
    """Algorithmic memory traffic of one inference pass (BF16): the packed
    input read once, every layer's output written once and read once by the
    next layer (the last one by the head)."""
    h, total = SIDE, 2 * SIDE * SIDE * 2
    for _, cout, s in LAYERS:
        h = (h - 1) // s + 1
        total += 2 * h * h * cout * 2
    return total


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ck(st):
    pvr._check(st)


class Net:
    """Parameters, Adam state and activation buffers of the CNN."""

    def __init__(self, device="cuda", seed: int = 5005):
        import torch
        L = pvr.load()
        self.L = L
        self.dev = device
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.conv = []
        for cin, cout, s in LAYERS:
            n = cout * 9 * cin
            w = (torch.randn(n, generator=g, dtype=torch.float32) * math.sqrt(2.0 / (9 * cin)))
            layer = dict(cin=cin, cout=cout, s=s, n=n,
                         w=w.to(device), b=torch.zeros(cout, device=device),
                         mw=torch.zeros(n, device=device), vw=torch.zeros(n, device=device),
                         mb=torch.zeros(cout, device=device), vb=torch.zeros(cout, device=device),
                         wb=torch.empty(n, dtype=torch.bfloat16, device=device),
                         wt=torch.empty(n, dtype=torch.bfloat16, device=device),
                         dw=torch.zeros(n, device=device), db=torch.zeros(cout, device=device))
            _ck(L.pvr_cnn_adam(_p(layer["w"]), None, _p(layer["mw"]), _p(layer["vw"]), n,
                               0.0, 0.9, 0.999, 1e-8, 0, _p(layer["wb"]), _p(layer["wt"]),
                               cout, cin, _s()))
            self.conv.append(layer)
        self.wfc = (torch.randn(N_FC, generator=g) * math.sqrt(1.0 / (HW * 64))).to(device)
        self.bfc = torch.zeros(6, device=device)
        self.mfc = torch.zeros(N_FC, device=device)
        self.vfc = torch.zeros(N_FC, device=device)
        self.mbf = torch.zeros(6, device=device)
        self.vbf = torch.zeros(6, device=device)
        self.dwfc = torch.zeros(N_FC, device=device)
        self.dbfc = torch.zeros(6, device=device)
        self.loss_w = torch.ones(6, device=device)
        self.step_no = 0
        self._bufs: Dict[int, dict] = {}

    # -- buffers ---------------------------------------------------------------------
    def buffers(self, B: int) -> dict:
        import torch
        if B in self._bufs:
            return self._bufs[B]
        acts, grads, shapes = [], [], []
        H = W = SIDE
        for cin, cout, s in LAYERS:
            Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
            acts.append(torch.empty(B * Ho * Wo * cout, dtype=torch.bfloat16, device=self.dev))
            grads.append(torch.empty(B * Ho * Wo * cout, dtype=torch.bfloat16, device=self.dev))
            shapes.append((H, W))
            H, W = Ho, Wo
        scr = max(self.L.pvr_cnn_wgrad_scratch(B, h, w, cin, cout, s)
                  for (h, w), (cin, cout, s) in zip(shapes, LAYERS))
        b = dict(x=torch.empty(B * SIDE * SIDE * 2, dtype=torch.bfloat16, device=self.dev),
                 acts=acts, grads=grads, shapes=shapes, hw=H * W,
                 scratch=torch.empty(scr // 4 + 16, dtype=torch.float32, device=self.dev),
                 hscr=torch.empty(self.L.pvr_cnn_head_scratch(B) // 4 + 16, dtype=torch.float32,
                                  device=self.dev),
                 pred=torch.empty(B * 6, device=self.dev),
                 loss=torch.zeros(1, device=self.dev),
                 ids=torch.empty(B, dtype=torch.int32, device=self.dev))
        self._bufs[B] = b
        return b

    # -- passes ----------------------------------------------------------------------
    def forward(self, B: int, target=None):
        """Forward pass on buffers(B)['x']; with target also the loss and the
        head gradients.  Returns the prediction tensor [B*6]."""
        L, bf = self.L, self.buffers(B)
        x = bf["x"]
        for (H, W), layer, out in zip(bf["shapes"], self.conv, bf["acts"]):
            _ck(L.pvr_cnn_conv_fwd(_p(x), _p(layer["wb"]), _p(layer["b"]), _p(out), B, H, W,
                                   layer["cin"], layer["cout"], layer["s"], 1, _s()))
            x = out
        _ck(L.pvr_cnn_head(_p(x), B, bf["hw"], _p(self.wfc), _p(self.bfc), _p(target),
                           _p(self.loss_w), _p(bf["pred"]), _p(bf["loss"]),
                           _p(bf["grads"][-1]) if target is not None else None,
                           _p(self.dwfc) if target is not None else None,
                           _p(self.dbfc) if target is not None else None,
                           _p(bf["hscr"]) if target is not None else None, _s()))
        return bf["pred"]

    def backward(self, B: int):
        L, bf = self.L, self.buffers(B)
        for li in range(len(LAYERS) - 1, -1, -1):
            layer = self.conv[li]
            H, W = bf["shapes"][li]
            inp = bf["x"] if li == 0 else bf["acts"][li - 1]
            _ck(L.pvr_cnn_conv_wgrad(_p(bf["grads"][li]), _p(bf["acts"][li]), _p(inp),
                                     _p(bf["scratch"]), _p(layer["dw"]), _p(layer["db"]), B, H, W,
                                     layer["cin"], layer["cout"], layer["s"], _s()))
            if li > 0:
                _ck(L.pvr_cnn_conv_dgrad(_p(bf["grads"][li]), _p(bf["acts"][li]),
                                         _p(layer["wt"]), _p(bf["grads"][li - 1]), B, H, W,
                                         layer["cin"], layer["cout"], layer["s"], _s()))

    def adam(self, lr: float = 1e-3):
        L = self.L
        self.step_no += 1
        t = self.step_no
        for layer in self.conv:
            _ck(L.pvr_cnn_adam(_p(layer["w"]), _p(layer["dw"]), _p(layer["mw"]), _p(layer["vw"]),
                               layer["n"], lr, 0.9, 0.999, 1e-8, t, _p(layer["wb"]),
                               _p(layer["wt"]), layer["cout"], layer["cin"], _s()))
            _ck(L.pvr_cnn_adam(_p(layer["b"]), _p(layer["db"]), _p(layer["mb"]), _p(layer["vb"]),
                               layer["cout"], lr, 0.9, 0.999, 1e-8, t, None, None, 0, 0, _s()))
        _ck(L.pvr_cnn_adam(_p(self.wfc), _p(self.dwfc), _p(self.mfc), _p(self.vfc), N_FC, lr,
                           0.9, 0.999, 1e-8, t, None, None, 0, 0, _s()))
        _ck(L.pvr_cnn_adam(_p(self.bfc), _p(self.dbfc), _p(self.mbf), _p(self.vbf), 6, lr,
                           0.9, 0.999, 1e-8, t, None, None, 0, 0, _s()))

    def pack(self, plan, ids, y_obs, y_sim, B: int):
        bf = self.buffers(B)
        _ck(self.L.pvr_cnn_pack_pairs(plan.h, _p(ids), B, _p(y_obs), _p(y_sim), _p(bf["x"]),
                                      _s()))

    def predict(self, plan, y_obs, y_sim, ids, B: int):
        """Scaled 6-DoF corrections [B, 6] for the patches ids [B] (int32,
        device) of a built plan."""
        self.pack(plan, ids, y_obs, y_sim, B)
        return self.forward(B).view(B, 6)


def make_pairs(plan, X, theta_ref, offsets, noise_sd: float, seed: int):
    """Observed patches at theta_ref (plus Gaussian noise) and patches
    simulated at theta_ref - offsets; returns (y_obs, y_sim) device tensors
    and leaves the plan built at theta_ref - offsets."""
    import torch
    y_obs = torch.empty(plan.N, dtype=torch.float32, device=X.device)
    y_sim = torch.empty_like(y_obs)
    plan.build(theta_ref)
    plan.simulate(X, y_sim=y_obs)
    if noise_sd > 0:
        gen = torch.Generator(device=X.device).manual_seed(seed)
        y_obs.add_(torch.randn(plan.N, generator=gen, device=X.device) * noise_sd)
    plan.build(theta_ref - offsets)
    plan.simulate(X, y_sim=y_sim)
    return y_obs, y_sim


def train(net: Net, plan, volumes: List, n_pairs: int, batch: int = 256, lr: float = 1e-3,
          max_rot_deg: float = 10.0, max_trans: float = 5.0, seed: int = 5100,
          log=None) -> dict:
    """Train on n_pairs pairs drawn round by round from the plan's patches
    over the given volumes (device tensors [V]).  Returns timing and loss
    history."""
    import torch
    from . import synth
    dev = volumes[0].device
    M = plan.M
    rounds = max(1, int(math.ceil(n_pairs / M)))
    hist = []
    t0 = time.perf_counter()
    t_data = 0.0
    seen = 0
    rng = np.random.default_rng(seed)
    for r in range(rounds):
        td = time.perf_counter()
        X = volumes[r % len(volumes)]
        ref = torch.from_numpy(synth.random_motion_batch(M, max_rot_deg, max_trans,
                                                         seed + 2 * r).astype(np.float32)).to(dev)
        off = torch.from_numpy(synth.random_motion_batch(M, max_rot_deg, max_trans,
                                                         seed + 2 * r + 1).astype(np.float32)).to(dev)
        y_obs, y_sim = make_pairs(plan, X, ref, off, 0.01 * float(X.max()), seed + r)
        target = plan.motion_frame(off)  # the offset in each patch's own frame
        perm = torch.from_numpy(rng.permutation(M).astype(np.int32)).to(dev)
        torch.cuda.synchronize()
        t_data += time.perf_counter() - td
        for b0 in range(0, M - batch + 1, batch):
            if seen >= n_pairs:
                break
            ids = perm[b0:b0 + batch].contiguous()
            bf = net.buffers(batch)
            bf["ids"].copy_(ids)
            tgt = target[ids.long()].reshape(-1).contiguous()
            net.pack(plan, bf["ids"], y_obs, y_sim, batch)
            net.forward(batch, tgt)
            net.backward(batch)
            net.adam(lr)
            seen += batch
            if seen == batch or (seen // batch) % 50 == 0:
                hist.append((seen, float(bf["loss"].item())))
                if log:
                    log(f"[learned] pairs {seen} loss {hist[-1][1]:.4f}")
        if seen >= n_pairs:
            break
    torch.cuda.synchronize()
    return dict(seconds=time.perf_counter() - t0, data_seconds=t_data, pairs=seen, loss=hist)


def init_fn_factory(net: Net, batch: int = 1024):
    """A driver init function: predicts every patch's correction from the
    current volume and keeps, per patch, whichever of the old and the
    proposed motion has the higher NCC (the registration refines it next).
    Every build takes the cycle's active set and sample mask; the plan is
    left built at the proposal (the registration that follows computes each
    patch's geometry itself and needs only the build's mask and active set,
    and the driver rebuilds after it).  Returns the per-patch NCC before the
    prediction and at the motion kept."""
    import torch

    def init_fn(plan, X, y, theta, active=None, mask=None):
        dev = X.device
        ysim = torch.empty(plan.N, dtype=torch.float32, device=dev)
        plan.build(theta, active=active, mask=mask)
        plan.simulate(X, y_sim=ysim)
        n_old = torch.empty(plan.M, device=dev)
        plan.ncc_grad(y, ysim, None, n_old)
        delta = torch.empty(plan.M, 6, device=dev)
        ids_all = torch.arange(plan.M, dtype=torch.int32, device=dev)
        for b0 in range(0, plan.M, batch):
            B = min(batch, plan.M - b0)
            bf = net.buffers(B)
            bf["ids"].copy_(ids_all[b0:b0 + B])
            delta[b0:b0 + B] = net.predict(plan, y, ysim, bf["ids"], B)
        # proposal = theta + the predicted offset taken back from the patch frame
        prop = plan.motion_frame(delta, inverse=True, base=theta)
        plan.build(prop, active=active, mask=mask)
        plan.simulate(X, y_sim=ysim)
        n_new = torch.empty(plan.M, device=dev)
        plan.ncc_grad(y, ysim, None, n_new)
        n_before = n_old.clone()
        plan.motion_accept(prop, n_new, theta, n_old)  # keep the better of the two
        return n_before, n_old

    return init_fn
