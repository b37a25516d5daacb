"""Learned warm start of the iteration-0 LCP: collect training rows from the
solver's own runs, fit the per-contact MLP on the GPU with the library's
forward/backward/Adam kernels, install it in a context.  The network
corrects the previous-step multiplier of the pair (zero output = the plain
previous-step start).

The paper leaves the start of the projected-gradient LCP open (Eq. cqpp
converges from any nonnegative start); the model only moves the start, so
results stay those of the plain method.  Targets are the multipliers of the
iteration-0 rows after the step's last recursion.  Everything numeric runs
in librelcp (through `relcp`); this module only batches and schedules.
"""
from __future__ import annotations

import math

import numpy as np

from . import relcp as R

H = 128
F = R.MLP_NFEAT


def init_params(seed: int) -> np.ndarray:
    """He-normal hidden layers, zero biases and a zero output layer, so that
    the untrained network gives the previous-step start (flat float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.normal(0.0, math.sqrt(2.0 / F), (H, F)).ravel(), np.zeros(H),
             rng.normal(0.0, math.sqrt(2.0 / H), (H, H)).ravel(), np.zeros(H),
             np.zeros(H), np.zeros(1)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == R.MLP_NPARAM
    return out


def normalisation(feat, gamma) -> np.ndarray:
    """mean (8), std (8) of the features and the correction scale (std of
    target minus previous-step multiplier) of a training set (torch or
    numpy arrays)."""
    f = np.asarray(feat.cpu() if hasattr(feat, "cpu") else feat, dtype=np.float64)
    g = np.asarray(gamma.cpu() if hasattr(gamma, "cpu") else gamma, dtype=np.float64)
    mean = f.mean(axis=0)
    std = f.std(axis=0)
    std = np.where(std > 1e-6 * np.maximum(1.0, np.abs(mean)), std, 1.0)
    d = g - f[:, 2]
    scale = d.std() if d.size and d.std() > 0 else 1.0
    return np.concatenate([mean, std, [scale]]).astype(np.float32)


class ContactLog:
    """Rows of A_0 (features, final multipliers) of accepted steps, kept on
    the GPU."""

    def __init__(self):
        self.feat, self.gamma = [], []

    def record(self, sim):
        f, g, _, _ = sim.log_contacts()
        if f.shape[0]:
            self.feat.append(f.clone())
            self.gamma.append(g.clone())

    def tensors(self):
        import torch
        return torch.cat(self.feat), torch.cat(self.gamma)

    def __len__(self):
        return sum(int(f.shape[0]) for f in self.feat)


class Trainer:
    """Adam on minibatches, every update on the GPU (relcp_mlp_grad,
    relcp_mlp_adam); batches are index lists into the resident data."""

    def __init__(self, norm, seed=0, device="cuda:0", batch=8192, params=None):
        import torch
        self.dev = torch.device(device)
        self.norm = np.asarray(norm, dtype=np.float32)
        p0 = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.tensor(p0, device=self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.empty_like(self.params)
        self.batch = batch
        self.work = R.mlp_workspace(batch, self.dev)
        self.t = 0
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)

    def epoch(self, feat, gamma, lr):
        """One pass over the data in shuffled minibatches; mean batch loss."""
        import torch
        n = feat.shape[0]
        perm = torch.randperm(n, generator=self.gen, device=self.dev).to(torch.int32)
        losses = torch.zeros(max(1, (n + self.batch - 1) // self.batch), dtype=torch.float32, device=self.dev)
        for k, s in enumerate(range(0, n, self.batch)):
            idx = perm[s:s + self.batch]
            R.mlp_grad(self.params, self.norm, feat, gamma, idx=idx, grad=self.grad, loss=losses[k:k + 1],
                       work=self.work)
            self.t += 1
            R.mlp_adam(self.params, self.grad, self.m, self.v, self.t, lr)
        return float(losses.mean().item())

    def fit(self, feat, gamma, epochs=20, lr=2e-3, lr_end=2e-4):
        hist = []
        for e in range(epochs):
            f = e / max(1, epochs - 1)
            hist.append(self.epoch(feat, gamma, lr * (lr_end / lr) ** f))
        return hist

    def predict(self, feat):
        return R.mlp_forward(self.params, self.norm, feat)[:feat.shape[0]]

    def start_error(self, feat, gamma):
        """rms and largest |start - target| (length units) of the learned
        start and of the previous-step start over a data set."""
        pred = self.predict(feat)
        out = {}
        for name, e in (("learned", pred - gamma), ("previous", feat[:, 2] - gamma)):
            out[name] = (float((e ** 2).mean().sqrt().item()), float(e.abs().max().item()))
        return out

    def weights(self) -> np.ndarray:
        return self.params.cpu().numpy().copy()
