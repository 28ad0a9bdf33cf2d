"""Differentiation pattern: the snapshot energy as a torch.autograd.Function whose backward is
the library's hand-written reverse pass, a fitter that runs whole training steps (forward,
loss, backward, Adam) inside the library, the cluster-expansion label source, and training
snapshots drawn by the library's own swap-MC sweeps.

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


# Coordination numbers of BCC shells 1..3.
BCC_SHELL_SIZES = (8, 6, 12)


def ce_pair_qsro(pair) -> np.ndarray:
    """qSRO blob (Eq. (2): V[3][5][5], W[3][5], lambda, C) whose swap energy changes equal those
    of the pair part of a cluster expansion, pair[m][p][q] per shell m = 1..3.

    Every site has z_m shell-m neighbours, so the pair energy sum over site pairs of
    pair_m(s_i, s_j) equals the same sum of V'_m(s_i, s_j) = pair_m(s_i, s_j) -
    (pair_m(s_i, s_i) + pair_m(s_j, s_j)) / 2 plus a function of the composition alone, which
    species swaps keep.  V' vanishes on like pairs; the qSRO term V_m^{pq} n_m^{pq}(j) / z_m
    summed over sites j counts each unlike pair twice, hence V_m^{pq} = z_m V'_m(p, q) / 2.
    W, lambda and C are zero."""
    pair = np.asarray(pair, dtype=np.float64)
    S = pair.shape[1]
    if pair.shape != (3, S, S) or S > 5:
        raise ValueError("pair must be [3][S][S] with S <= 5")
    V = np.zeros((3, 5, 5))
    for m in range(3):
        d = np.diag(pair[m])
        V[m, :S, :S] = BCC_SHELL_SIZES[m] * (pair[m] - 0.5 * (d[:, None] + d[None, :])) / 2.0
    return np.concatenate([V.ravel(), np.zeros(15), [0.0, 0.0]]).astype(np.float32)


def sample_snapshots(start, cells_per_axis, temperatures, pair, burn_in=200, n_per_chain=1, gap=10, seed=0,
                     precision="fp32"):
    """Training snapshots drawn by swap MC: one chain per row of `start` (uint8 [chains][2 L^3],
    species 0..S-1) at its own temperature, driven by the pair part of a cluster expansion
    (`pair` [3][S][S], carried exactly by ce_pair_qsro); all chains are replicas of one context,
    so each sweep is one launch per colour over every chain.  After `burn_in` sweeps, takes
    `n_per_chain` snapshots `gap` sweeps apart.  Returns a uint8 device tensor
    [n_per_chain * chains][2 L^3], snapshot k of chain b at row k * chains + b."""
    from . import SwapMC
    torch = _torch()
    start = np.ascontiguousarray(np.asarray(start, dtype=np.uint8))
    B, N = start.shape
    L = int(cells_per_axis)
    if N != 2 * L ** 3:
        raise ValueError(f"snapshots have {N} sites, L = {L} implies {2 * L ** 3}")
    temps = [float(t) for t in np.asarray(temperatures, dtype=np.float64).reshape(-1)]
    if len(temps) != B:
        raise ValueError("one temperature per chain")
    S = int(np.asarray(pair).shape[1])
    mc = SwapMC([(L, L, L)] * B, temps, start.reshape(-1), ce_pair_qsro(pair), n_species=S, feature=2, hidden=0,
                precision=precision, seed=seed)
    try:
        out = torch.empty((n_per_chain, B, N), dtype=torch.uint8, device=mc.occ.device)
        mc.sweep(burn_in)
        for k in range(n_per_chain):
            if k:
                mc.sweep(gap)
            out[k].copy_(mc.occ.view(B, N))
    finally:
        mc.close()
    return out.view(n_per_chain * B, N)
