"""Fitting loop of the training appendix, driven from the host; every step
runs in the library's kernels.

Per epoch: uniforms are drawn (random numbers are inputs), the SDF surface
sampler traces random rays against the analytic shape (or fixed surface
samples are reused), the 2:2:1 surface/near/uniform training set is built
on the device in batch-major order, and each batch takes one Eq. 4
fwd+bwd (per-LOD weights) and one fused Adam step.

Schedules (training appendix): "joint" trains every LOD from the start;
"progressive" starts with the finest LOD and adds the next coarser one
every `grow_every` epochs (LODs not yet added have loss weight 0 and their
feature levels are not updated).  `freeze_decoders` keeps the decoders
fixed and trains only the features (the "general" surface extractor of the
generalisation experiment).
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np
import torch

from . import ngl


def device_uniforms(gen: torch.Generator, device):
    """Uniform source on the device (torch's Philox generator)."""
    return lambda rows, n: torch.rand((rows, n), generator=gen, device=device, dtype=torch.float32)


class Fitter:
    def __init__(self, model: ngl.Model, shape: ngl.DeviceShape, *, points: int = 500_000, batch: int = 512,
                 lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 sigma: float = 0.01, schedule: str = "joint", grow_every: int = 100,
                 freeze_decoders: bool = False, rays: Optional[int] = None, max_steps: int = 256,
                 delta: float = 1e-5, surface: Optional[torch.Tensor] = None,
                 uniforms: Optional[Callable[[int, int], torch.Tensor]] = None, seed: int = 0):
        if schedule not in ("joint", "progressive"):
            raise ValueError("schedule is 'joint' or 'progressive'")
        if model.feat_dtype != ngl.F32 or model.w_dtype != ngl.F32:
            raise ngl.NGLError("fitting needs FP32 features and decoders")
        dev = model.b2.device
        self.model, self.shape = model, shape
        self.batch = int(batch)
        self.N = (int(points) // self.batch) * self.batch
        if self.N == 0:
            raise ValueError("points must be at least one batch")
        self.hp = dict(lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        self.sigma, self.schedule, self.grow_every = float(sigma), schedule, int(grow_every)
        self.freeze = bool(freeze_decoders)
        self.rays = int(rays) if rays is not None else self.N
        self.max_steps, self.delta = int(max_steps), float(delta)
        self.fixed_surface = surface
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(seed))
        self.uniforms = uniforms if uniforms is not None else device_uniforms(gen, dev)
        self.grads = ngl.Grads(model)
        self.ws = ngl.train_workspace(model, self.batch, dev)
        self.params = ngl.parameters(model)
        gl = [*self.grads.dfeat, *self.grads.dW1, *self.grads.db1, *self.grads.dw2, self.grads.db2]
        self.grad_of = {id(p): g for p, g in zip(self.params, gl)}
        self.m = {id(p): torch.zeros_like(p) for p in self.params}
        self.v = {id(p): torch.zeros_like(p) for p in self.params}
        self.x = torch.empty((self.N // self.batch, 3, self.batch), dtype=torch.float32, device=dev)
        self.target = torch.empty(self.N, dtype=torch.float32, device=dev)
        self.losses = torch.zeros(self.N // self.batch, dtype=torch.float32, device=dev)
        self.sampler = None
        self.step = 0
        self.epoch = 0

    # -- schedule -----------------------------------------------------------
    def active_lods(self, epoch: Optional[int] = None) -> List[int]:
        L = self.model.num_lods
        if self.schedule == "joint":
            return list(range(1, L + 1))
        e = self.epoch if epoch is None else epoch
        first = max(1, L - e // self.grow_every)
        return list(range(first, L + 1))

    def trainable(self, active: List[int]):
        """Feature levels of the active LODs, and the decoders unless frozen
        (decoders of inactive LODs get zero gradients and stay put)."""
        m = self.model
        out = [m.feats[l - 1] for l in active]
        if not self.freeze:
            out += [*m.W1, *m.b1, *m.w2, m.b2]
        return out

    # -- one epoch ----------------------------------------------------------
    def surface_samples(self):
        if self.fixed_surface is not None:
            return self.fixed_surface, self.fixed_surface.shape[1]
        u = self.uniforms(5, self.rays)
        self.sampler = ngl.sample_surface(self.shape, u, self.max_steps, self.delta, out=self.sampler)
        n = int(self.sampler["count"].item())
        if n == 0:
            raise RuntimeError("the surface sampler found no surface points")
        return self.sampler["pts"], n

    def run_epoch(self) -> float:
        """One pass over a freshly sampled training set; returns the mean
        batch loss (Eq. 4 over the active LODs)."""
        S, ns = self.surface_samples()
        uni = self.uniforms(4, self.N)
        ngl.training_points(self.shape, S, ns, uni, self.batch, self.sigma, x=self.x, target=self.target)
        active = self.active_lods()
        wts = [1.0 if L in active else 0.0 for L in range(1, self.model.num_lods + 1)]
        tensors = self.trainable(active)
        grads = [self.grad_of[id(t)] for t in tensors]
        ms = [self.m[id(t)] for t in tensors]
        vs = [self.v[id(t)] for t in tensors]
        adam = ngl.AdamGroup(tensors, grads, ms, vs)
        B = self.batch
        for b in range(self.N // B):
            ngl.train_fwd_bwd_lods(self.model, self.x[b], self.target[b * B:(b + 1) * B], wts, grads=self.grads,
                                   ws=self.ws, loss=self.losses[b:b + 1])
            self.step += 1
            adam.step(self.step, **self.hp)
        self.epoch += 1
        return float(self.losses.mean().item())
