"""Differentiation pattern: the snapshot energy as a torch.autograd.Function whose backward is
the library's hand-written reverse pass, a fitter that runs whole training steps (forward,
loss, backward, Adam) inside the library, and the cluster-expansion label source.

Every computation runs in libsmc's kernels; this module only marshals tensors.
"""
from __future__ import annotations

import numpy as np

from ._lib import smc_ce_energy, smc_ce_triangles, smc_energy_bwd, smc_energy_fwd, smc_fit_step


def _torch():
    import torch
    return torch


def _check_snaps(snaps, cells_per_axis):
    torch = _torch()
    if snaps.dtype != torch.uint8 or snaps.dim() != 2 or not snaps.is_contiguous():
        raise ValueError("snapshots must be a contiguous uint8 tensor [batch, 2 L^3]")
    if snaps.shape[1] != 2 * cells_per_axis ** 3:
        raise ValueError(f"snapshots have {snaps.shape[1]} sites, L = {cells_per_axis} implies {2 * cells_per_axis ** 3}")


class SnapshotEnergy(_torch().autograd.Function):
    """S_b(params) = sum of local MLP energies of snapshot b (Eqs. (4)-(6)); backward gives
    dL/dparams = sum_b dL/dS_b dS_b/dparams through smc_energy_bwd."""

    @staticmethod
    def forward(ctx, params, mc, snaps, cells_per_axis):
        torch = _torch()
        _check_snaps(snaps, cells_per_axis)
        params = params.contiguous()
        S = torch.empty(snaps.shape[0], dtype=torch.float64, device=snaps.device)
        smc_energy_fwd(mc.ctx, snaps.data_ptr(), snaps.shape[0], cells_per_axis, params.data_ptr(), S.data_ptr())
        ctx.save_for_backward(params, snaps)
        ctx.mc = mc
        ctx.L = cells_per_axis
        return S

    @staticmethod
    def backward(ctx, grad_S):
        torch = _torch()
        params, snaps = ctx.saved_tensors
        g = grad_S.to(torch.float64).contiguous()
        grad = torch.empty_like(params)
        smc_energy_bwd(ctx.mc.ctx, snaps.data_ptr(), snaps.shape[0], ctx.L, params.data_ptr(), g.data_ptr(),
                       grad.data_ptr())
        return grad, None, None, None


def snapshot_energy(mc, params, snaps, cells_per_axis):
    return SnapshotEnergy.apply(params, mc, snaps, cells_per_axis)


class Fitter:
    """Adam fit of the FP32 master parameters to per-snapshot labels; each step is one
    smc_fit_step call (forward, per-atom MSE loss, hand-written backward, Adam)."""

    def __init__(self, mc, params, lr=1e-3):
        torch = _torch()
        self.mc = mc
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.lr = float(lr)
        self.step_count = 0

    def step(self, snaps, labels, cells_per_axis, want_loss=True):
        torch = _torch()
        _check_snaps(snaps, cells_per_axis)
        labels = labels.to(torch.float64).contiguous()
        self.step_count += 1
        return smc_fit_step(self.mc.ctx, snaps.data_ptr(), snaps.shape[0], cells_per_axis, labels.data_ptr(),
                            self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.lr, self.step_count,
                            want_loss)


def ce_energy(mc, ce: dict, snaps, cells_per_axis):
    """Cluster-expansion energies (double [batch]) of the snapshots."""
    torch = _torch()
    _check_snaps(snaps, cells_per_axis)
    out = torch.empty(snaps.shape[0], dtype=torch.float64, device=snaps.device)
    smc_ce_energy(mc.ctx, ce, snaps.data_ptr(), snaps.shape[0], cells_per_axis, out.data_ptr())
    return out


def ce_triangles() -> np.ndarray:
    return smc_ce_triangles()
