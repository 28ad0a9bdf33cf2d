"""Swap Monte Carlo on periodic BCC and FCC alloys with local MLP or qSRO energies, for MI355X (gfx950).

The compute path is the HIP library ``libsmc.so`` behind the C ABI of ``include/smc.h``;
this package only marshals arguments.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import numpy as np

from ._lib import (PRECISIONS, SMC_BF16, SMC_BF16X3, SMC_FEAT_COUNTS_S12, SMC_FEAT_ONEHOT_S123,
                   SMC_FEAT_QSRO_S123, SMC_FEAT_MLPNET_S12, SMC_LATTICE_BCC, SMC_LATTICE_FCC, LATTICES, BASIS,
                   smc_lattice_shells, SMC_FP8_E4M3, SMC_FP32, SMC_FP64, SMCError, lib, smc_autotune, smc_counters,
                   smc_delta_e64, smc_destroy, smc_energy, smc_get_sweep, smc_get_variant, smc_init,
                   smc_kernel_times, smc_n_colours, smc_n_sites, smc_profile, smc_refresh,
                   smc_set_params, smc_set_sweep, smc_set_variant, smc_site_energies, smc_sweep,
                   smc_use_graph, smc_set_strategy, smc_get_strategy, STRATEGIES, smc_set_temperatures,
                   smc_warren_cowley)

__all__ = ["SwapMC", "SMCError", "PRECISIONS", "lib"]


def _torch():
    import torch
    return torch


class SwapMC:
    """One libsmc context over caller-owned torch tensors (occupancy, parameters, cache)."""

    def __init__(self, cells, temperatures, occ, params, *, n_species, feature, hidden,
                 precision="fp32", seed=0, guard_eV=-1.0, device="cuda:0", stream=None, lattice="bcc"):
        torch = _torch()
        cells = np.asarray(cells, dtype=np.int32).reshape(-1, 3)
        self.cells = cells
        self.temperatures = np.asarray(temperatures, dtype=np.float64).reshape(-1)
        self.n_replicas = len(self.temperatures)
        self.device = torch.device(device)
        self.occ = torch.as_tensor(np.asarray(occ, dtype=np.uint8)).to(self.device).contiguous()
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.device).contiguous()
        self.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
        n_total = int(sum(BASIS[self.lattice] * int(np.prod(c)) for c in cells))
        if self.occ.numel() != n_total:
            raise ValueError(f"occupancy has {self.occ.numel()} sites, cells imply {n_total}")
        self.ecache = torch.empty(n_total, dtype=torch.float32, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.n_sites = n_total
        self.n_species = int(n_species)
        self.ctx = None
        self.ctx = smc_init(cells, self.temperatures, n_species, feature, hidden, self.precision,
                            seed, guard_eV, self.occ.data_ptr(), self.params.data_ptr(),
                            self.ecache.data_ptr(), self.stream.cuda_stream, self.lattice)

    def sweep(self, n=1, stats=False, trace=False):
        torch = _torch()
        if not stats and not trace:
            smc_sweep(self.ctx, n)
            return None
        R = self.n_replicas
        cnt = {k: np.zeros(R, dtype=np.uint64) for k in ("attempts", "diff_species", "accepts", "rechecks")}
        tr = {}
        if trace:
            tr["dE"] = torch.zeros(self.n_sites, dtype=torch.float64, device=self.device)
            tr["dE_fast"] = torch.zeros(self.n_sites, dtype=torch.float64, device=self.device)
            tr["flags"] = torch.zeros(self.n_sites, dtype=torch.uint8, device=self.device)
        smc_sweep(self.ctx, n, cnt["attempts"], cnt["diff_species"], cnt["accepts"], cnt["rechecks"],
                  tr["dE"].data_ptr() if trace else 0, tr["dE_fast"].data_ptr() if trace else 0,
                  tr["flags"].data_ptr() if trace else 0, with_stats=True)
        out = dict(cnt)
        out.update(tr)
        return out

    def counters(self, reset=False):
        """Cumulative [attempts, diff_species, accepts, rechecks] x replicas (synchronises)."""
        return smc_counters(self.ctx, self.n_replicas, reset)

    def energy(self):
        return smc_energy(self.ctx, self.n_replicas)

    def profile(self, enable=True):
        """Record HIP events around every colour / re-decision kernel launch."""
        smc_profile(self.ctx, enable)

    def kernel_times(self):
        """(colour-kernel ms, re-decision-kernel ms, colour launches) since profile(True)."""
        return smc_kernel_times(self.ctx)

    def delta_e64(self, sites, sweep=None, replica=0):
        """FP64 dE of the swaps the given trial sites propose at `sweep` (default: the next
        sweep), on the current lattice; returns (partners, dE)."""
        return smc_delta_e64(self.ctx, replica, self.sweep_index if sweep is None else sweep, sites)

    def site_energies(self, precision=None):
        torch = _torch()
        p = self.precision if precision is None else (PRECISIONS[precision] if isinstance(precision, str) else precision)
        dt = torch.float64 if p == SMC_FP64 else torch.float32
        out = torch.empty(self.n_sites, dtype=dt, device=self.device)
        smc_site_energies(self.ctx, p, out.data_ptr())
        return out

    def set_params(self, params):
        torch = _torch()
        self.params.copy_(torch.as_tensor(np.asarray(params, dtype=np.float32)))
        smc_set_params(self.ctx, self.params.data_ptr())

    def refresh(self):
        smc_refresh(self.ctx)

    @property
    def sweep_index(self):
        return smc_get_sweep(self.ctx)

    @sweep_index.setter
    def sweep_index(self, v):
        smc_set_sweep(self.ctx, int(v))

    def set_temperatures(self, temperatures):
        """Temperatures (K) of every replica for the following sweeps (scalar: all replicas)."""
        t = np.broadcast_to(np.asarray(temperatures, dtype=np.float64), (self.n_replicas,)).copy()
        smc_set_temperatures(self.ctx, t)
        self.temperatures = t

    def anneal(self, schedule, sweeps_per_temperature):
        """Run sweeps_per_temperature sweeps at each temperature of the schedule (K)."""
        for T in schedule:
            self.set_temperatures(T)
            self.sweep(sweeps_per_temperature)

    def warren_cowley(self, replica=0):
        """Warren-Cowley alpha[shell][p][q] of the replica's current occupancy."""
        return smc_warren_cowley(self.ctx, replica, self.n_species)

    @property
    def strategy(self):
        """'zone' (default) or 'double_lattice' (Algorithm 1 with sigma0/sigma1 and all-site
        energies; same trajectory, about 10x the evaluations)."""
        v = smc_get_strategy(self.ctx)
        return {b: a for a, b in STRATEGIES.items()}[v]

    @strategy.setter
    def strategy(self, name):
        smc_set_strategy(self.ctx, STRATEGIES[name] if isinstance(name, str) else int(name))

    def use_graph(self, enable=True):
        """Replay plain sweeps from a captured hipGraph (default on); results are identical."""
        smc_use_graph(self.ctx, enable)

    @property
    def variant(self):
        return smc_get_variant(self.ctx)

    @variant.setter
    def variant(self, v):
        smc_set_variant(self.ctx, v)

    def autotune(self, cache_path=None):
        """Time every colour-kernel variant on one sweep of the current state (restored
        afterwards), keep the fastest; returns (variant, ms per variant)."""
        return smc_autotune(self.ctx, cache_path)

    def n_colours(self, replica=0):
        return smc_n_colours(self.ctx, replica)

    def close(self):
        if self.ctx:
            smc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
