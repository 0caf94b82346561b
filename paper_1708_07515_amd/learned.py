"""Learned decimation filter: parameters, AdamW state and one training step.

The network (two 5 x 5 convolutions over angle x column, 16 channels, added to
the plan's decimation of Sec. 2.1: the triangle, or the windowed sinc) and
every step of its training run in the
library's kernels; this module only owns the device buffers and sequences the
calls:

    learned_decompose   Y = T + R                       (forward)
    reconstruct         f = backprojection of Y         (eq. (6))
    sq_residual         r = 2 (f - target), loss = sum (f - target)^2
    reconstruct_adjoint dY = backprojection^T r
    learned_backward    g = dL / dweights
    adamw_step          master weights, moments, BF16 copy

Parameter order: W1 [16][5][5], b1 [16], W2 [16][5][5], b2 (817 values).
"""

import numpy as np
import torch

from ._lib import LEARNED_PARAMS, adamw_step, sq_residual, sq_residual_weighted

CH, TAPS = 16, 5
OFF_W1, OFF_B1, OFF_W2, OFF_B2 = 0, 400, 416, 816


class LearnedDecimation:
    """FP32 master weights on the device, their BF16 copy and AdamW moments.

    A new instance has W1 ~ N(0, (scale / 5)^2) (seeded), b1 = 0 and a zero
    second layer, so it computes the plan's plain decimation until trained."""

    def __init__(self, device="cuda:0", seed=0, scale=0.1, lr=2e-3, betas=(0.9, 0.999), eps=1e-8,
                 weight_decay=0.0):
        gen = torch.Generator().manual_seed(seed)
        master = torch.zeros(LEARNED_PARAMS, dtype=torch.float32)
        master[OFF_W1:OFF_B1] = torch.randn(CH * TAPS * TAPS, generator=gen) * (scale / TAPS)
        self.device = torch.device(device)
        self.master = master.to(self.device)
        self.weights = self.master.to(torch.bfloat16)
        self.m1 = torch.zeros_like(self.master)
        self.m2 = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.step_count = 0
        self.lr, self.betas, self.eps, self.weight_decay = lr, betas, eps, weight_decay

    def load(self, master):
        """Set the master weights (817 floats, any device) and the BF16 copy."""
        self.master.copy_(torch.as_tensor(master, dtype=torch.float32).reshape(-1))
        self.weights.copy_(self.master.to(torch.bfloat16))

    def state(self):
        return self.master.detach().cpu().clone()

    def save_checkpoint(self, path):
        """Write the training state (master weights, both AdamW moments, the
        step count and the hyper-parameters) to ``path`` (numpy .npz, no
        pickled objects)."""
        hyper = np.array([self.step_count, self.lr, self.betas[0], self.betas[1], self.eps, self.weight_decay],
                         dtype=np.float64)
        with open(path, "wb") as f:
            np.savez(f, master=self.master.detach().cpu().numpy(), m1=self.m1.detach().cpu().numpy(),
                     m2=self.m2.detach().cpu().numpy(), hyper=hyper)

    def load_checkpoint(self, path):
        """Restore a state written by save_checkpoint: the next apply() takes
        the step an uninterrupted run would have taken."""
        with np.load(path, allow_pickle=False) as z:
            master, m1, m2, hyper = z["master"], z["m1"], z["m2"], z["hyper"]
        if master.shape != (LEARNED_PARAMS,) or m1.shape != master.shape or m2.shape != master.shape \
                or hyper.shape != (6,):
            raise ValueError(f"{path}: not a learned decimation checkpoint")
        self.load(master)
        self.m1.copy_(torch.from_numpy(m1))
        self.m2.copy_(torch.from_numpy(m2))
        self.step_count = int(hyper[0])
        self.lr, self.betas = float(hyper[1]), (float(hyper[2]), float(hyper[3]))
        self.eps, self.weight_decay = float(hyper[4]), float(hyper[5])

    def as_arrays(self):
        """The master weights as a dict of float64 numpy arrays."""
        w = self.master.detach().double().cpu().numpy()
        return dict(w1=w[OFF_W1:OFF_B1].reshape(CH, TAPS, TAPS), b1=w[OFF_B1:OFF_W2].copy(),
                    w2=w[OFF_W2:OFF_B2].reshape(CH, TAPS, TAPS), b2=w[OFF_B2:].copy())

    def forward(self, plan, filt, ws, vol, stream=None):
        plan.learned_decompose(filt, ws, self.weights, stream)
        plan.reconstruct(filt, ws, vol, stream)

    def gradient(self, plan, filt, ws, vol, target, resid, dws, stream=None):
        """Forward, loss and gradient (into self.grad) for one volume."""
        self.forward(plan, filt, ws, vol, stream)
        sq_residual(vol, target, resid, self.loss, stream)
        plan.reconstruct_adjoint(resid, dws, stream)
        plan.learned_backward(filt, dws, self.weights, self.grad, stream)

    def apply(self, stream=None):
        self.step_count += 1
        adamw_step(self.master, self.m1, self.m2, self.grad, self.weights, self.step_count, self.lr,
                   self.betas[0], self.betas[1], self.eps, self.weight_decay, stream)

    def train_step(self, plan, filt, ws, vol, target, resid, dws, stream=None):
        """One AdamW step on one volume; returns the loss tensor (device)."""
        self.gradient(plan, filt, ws, vol, target, resid, dws, stream)
        self.apply(stream)
        return self.loss

    def forward_slab(self, plan, filt_band, v0, ws_band, z0, vol_slab, stream=None):
        """The learned FDK-OD reconstruction of slices [z0, z0 + nzs) from the
        band of detector rows starting at v0 (the slab mode's band)."""
        plan.learned_decompose_band(filt_band, v0, ws_band, self.weights, stream)
        plan.reconstruct_slab(filt_band, ws_band, v0, filt_band.shape[1], z0, vol_slab, stream)

    def train_step_slab(self, plan, filt_band, v0, ws_band, z0, vol_slab, target_slab, resid, dws_band,
                        weight=1.0, stream=None):
        """One AdamW step on one slab: the loss is the squared error of the
        slab's reconstruction, times ``weight`` (e.g. the inverse of the
        target's energy, so that every slab counts by its relative error);
        its gradient reaches the weights through the transpose of the slab's
        backprojection."""
        nrows = filt_band.shape[1]
        self.forward_slab(plan, filt_band, v0, ws_band, z0, vol_slab, stream)
        sq_residual_weighted(vol_slab, target_slab, resid, self.loss, weight, stream)
        plan.reconstruct_adjoint_slab(resid, v0, nrows, z0, dws_band, stream)
        plan.learned_backward_band(filt_band, v0, dws_band, self.weights, self.grad, stream)
        self.apply(stream)
        return self.loss
