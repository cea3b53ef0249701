"""The paper's training protocol (Sec. 4.4) driven through the C ABI.

Every step runs in the HIP library: the render (deformation MLP, lists,
blending, with the per-pixel blend state kept), the hybrid loss
lambda1 * l1 + (1 - lambda1) * (1 - SSIM) and its gradient, the hand-written
backward, anneal smoothing of the moving positions, the Adam update and the
repacking of the updated scene. This module only sequences the calls and holds
the device tensors (parameters, Adam moments); the standard normal draws of
anneal smoothing come from torch's seeded generator (the caller's random
numbers).

Schedule (Sec. 4.4, coarse-to-fine training): for the first `coarse_iters`
steps only the canonical Gaussians are fitted to the spectra, with the
deformation MLP inactive (static renders); afterwards the MLP deforms the
Gaussians for each position, both are trained, and the gradients of the
canonical positions are frozen. Hyperparameter table: Gaussian learning rate
1e-2, MLP learning rate 8e-3, lambda1 = 0.7, anneal weight gamma = 1 and
threshold tau = 10k; Adam's decays and epsilon are not given (0.9, 0.999,
1e-8 here).
"""
from __future__ import annotations

import torch

from . import binding as B

GAUSSIAN_KEYS = B.PARAMS[:7]


class Trainer:
    def __init__(self, lib: B.Context, gaussians: dict, H: int, W: int, mlp, *, n_positions: int,
                 coarse_iters: int = 0, bf16: bool = True, lambda1: float = 0.7, lr_gaussians: float = 1e-2,
                 lr_mlp: float = 8e-3, gamma: float = 1.0, tau: int = 10_000, stop_grad_positions: bool = True,
                 room=((0.0, 0.0, 0.0), (6.0, 6.0, 3.0)), seed: int = 0, flags: int = 0):
        self.lib, self.H, self.W = lib, H, W
        self.room = room
        self.sid = lib.upload_scene(gaussians, H, W, mlp=mlp, room=room)
        dev = lib.device
        self.g = {k: torch.as_tensor(gaussians[k], dtype=torch.float32).to(dev).contiguous() for k in GAUSSIAN_KEYS}
        self.Ws = [torch.as_tensor(w, dtype=torch.float32).to(dev).contiguous() for w in mlp[0]]
        self.bs = [torch.as_tensor(b, dtype=torch.float32).to(dev).contiguous() for b in mlp[1]]
        zeros = lambda t: torch.zeros_like(t)
        self.m = {id(t): zeros(t) for t in self._all()}
        self.v = {id(t): zeros(t) for t in self._all()}
        self.steps_g = 0  # Adam step numbers per group
        self.steps_m = 0
        self.it = 0
        self.n_positions = n_positions
        self.coarse_iters = coarse_iters
        self.bf16 = bf16
        self.extra_flags = flags
        self.lambda1, self.lr_g, self.lr_m = lambda1, lr_gaussians, lr_mlp
        self.gamma, self.tau = gamma, tau
        self.stop_grad_positions = stop_grad_positions
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)

    def _all(self):
        return list(self.g.values()) + self.Ws + self.bs

    @property
    def fine(self) -> bool:
        return self.it >= self.coarse_iters

    def render(self, tx, flags_extra: int = 0):
        """Spectra of the current model for positions tx (batch, 3) without smoothing (evaluation)."""
        if self.fine:
            flags = (B.MLP_BF16 if self.bf16 else B.MLP_FP32) | self.extra_flags | flags_extra
            return self.lib.render(self.sid, tx, flags=flags)
        return self.lib.render(self.sid, None, flags=B.NO_DEFORM | self.extra_flags | flags_extra,
                               batch=tx.shape[0])

    def step(self, tx, target):
        """One training step on positions tx (batch, 3) and target spectra (batch, H, W); returns the loss tensor
        (3,) = (total, l1, ssim) of the forward pass, on the device."""
        lib = self.lib
        nb = tx.shape[0]
        fine = self.fine
        if fine:
            noise = torch.randn(tx.shape, generator=self.gen, device=tx.device, dtype=torch.float32)
            txs = lib.anneal_tx(tx, noise, self.it - self.coarse_iters, self.n_positions, gamma=self.gamma,
                                tau=self.tau, room=self.room)
            flags = (B.MLP_BF16 if self.bf16 else B.MLP_FP32) | self.extra_flags
            out, aux = lib.render(self.sid, txs, flags=flags | B.KEEP_AUX)
        else:
            txs = None
            flags = B.NO_DEFORM | self.extra_flags
            out, aux = lib.render(self.sid, None, flags=flags | B.KEEP_AUX, batch=nb)
        loss, grad = lib.hybrid_loss(out, target, self.lambda1)
        freeze = fine and self.stop_grad_positions
        gg = {k: (None if (freeze and k in ("mean_x", "mean_y")) else torch.zeros_like(t))
              for k, t in self.g.items()}
        grads = dict(gg)
        if fine:
            grads["weight"] = [torch.zeros_like(w) for w in self.Ws]
            grads["bias"] = [torch.zeros_like(b) for b in self.bs]
        lib.render_backward(self.sid, txs, flags, grad, aux, grads)
        # Adam: the Gaussians (the canonical positions only while not frozen), then the MLP in the fine stage
        ps = [self.g[k] for k in GAUSSIAN_KEYS if gg[k] is not None]
        gs = [gg[k] for k in GAUSSIAN_KEYS if gg[k] is not None]
        self.steps_g += 1
        lrs = [self.lr_g] * len(ps)
        if fine:
            self.steps_m += 1
            mp = self.Ws + self.bs
            mg = grads["weight"] + grads["bias"]
            # one launch per group: each group keeps its own bias-correction step count
            lib.adam_step(mp, mg, [self.m[id(t)] for t in mp], [self.v[id(t)] for t in mp], [self.lr_m] * len(mp),
                          self.steps_m)
        lib.adam_step(ps, gs, [self.m[id(t)] for t in ps], [self.v[id(t)] for t in ps], lrs, self.steps_g)
        lib.update_scene(self.sid, gaussians=self.g, mlp=(self.Ws, self.bs) if fine else None)
        self.it += 1
        return loss
