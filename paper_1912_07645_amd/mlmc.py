"""Multilevel Monte Carlo on one GPU (Section 2.2 of the paper): levels of uneven resolution
evolved together, then level-difference statistics and the telescoping estimate.

The estimator is sum_{l=1..L} (1/M_l) sum_k (G(u^l_k) - G(u^{l-1}_k)) with u^0 := 0. Level
l >= 2 uses M_l coupled samples: the same random input evolved on grid n_l and on grid
n_{l-1}. So each distinct grid n_l holds one batch (a "group") with the M_l fine samples of
level l followed by the M_{l+1} coarse partners of level l+1. All groups step through the
same launches (fv_evolve_multi), each sample with its own time step; the level statistics
(fv_stats_accumulate / fv_stats_accumulate_diff) and the combination on the finest grid
(fv_mlmc_combine) run on the device.
"""
from __future__ import annotations

import time

import torch

from .solver import Solver, Stats, evolve_multi, mlmc_combine


class MultilevelRun:
    """Grids ns[0] < ns[1] < ... (coarse to fine, each dividing the next) with Ms[l] samples
    on level l; scheme keyword arguments as for Solver (dim, eq, flux, recon, integrator, ...)."""

    def __init__(self, ns, Ms, dim=2, device=None, **scheme):
        if len(ns) != len(Ms) or len(ns) < 1:
            raise ValueError("one sample count per level")
        self.ns, self.Ms, self.dim = list(ns), list(Ms), dim
        self.solvers = [Solver(dim=dim, n=(n,) * dim, device=device, **scheme) for n in self.ns]
        self.device = self.solvers[0].device

    def group_batch(self, l: int) -> int:
        """Samples on grid l: level l's fine samples, then level l+1's coarse partners."""
        return self.Ms[l] + (self.Ms[l + 1] if l + 1 < len(self.Ms) else 0)

    def tune(self, states, cfl, steps=4, reps=3) -> int:
        """Pick the tile variant (shared by every grid: one launch covers them all) by timing
        `steps` multi-grid steps of copies of `states` per variant; returns the variant."""
        best, best_t = 0, None
        # untimed steps first, so that the clocks have left their idle state before the first
        # variant is timed
        for s in self.solvers:
            s.set_variant(0)
        warm = 0.0
        while warm < 0.05:
            G = [U.clone() for U in states]
            torch.cuda.synchronize(self.device)
            t0 = time.perf_counter()
            self.evolve(G, 1e30, cfl, max_steps=steps)
            torch.cuda.synchronize(self.device)
            warm += time.perf_counter() - t0
        for v in range(self.solvers[0].num_variants()):
            for s in self.solvers:
                s.set_variant(v)
            ts = []
            for _ in range(reps + 1):
                G = [U.clone() for U in states]
                torch.cuda.synchronize(self.device)
                t0 = time.perf_counter()
                self.evolve(G, 1e30, cfl, max_steps=steps)
                torch.cuda.synchronize(self.device)
                ts.append(time.perf_counter() - t0)
            t = min(ts[1:])
            if best_t is None or t < best_t:
                best, best_t = v, t
        for s in self.solvers:
            s.set_variant(best)
        return best

    def evolve(self, states, t_end, cfl, max_steps=10**9):
        """Evolve every group (list of device tensors, one per grid) from t = 0 to t_end."""
        ts = [torch.zeros(U.shape[0], dtype=torch.float64, device=self.device) for U in states]
        ks = [torch.zeros(U.shape[0], dtype=torch.int64, device=self.device) for U in states]
        errs = [torch.zeros(U.shape[0], dtype=torch.int32, device=self.device) for U in states]
        st = evolve_multi(self.solvers, states, ts, t_end, cfl, max_steps, ks, errs)
        self.last_steps = ks
        return st, ts, errs

    def statistics(self, states):
        """Level statistics and the multilevel estimate on the finest grid."""
        levels = []
        for l, U in enumerate(states):
            lv = Stats(self.solvers[l])
            fine = U[:self.Ms[l]]
            if l == 0:
                lv.accumulate(fine)
            else:
                coarse = states[l - 1][self.Ms[l - 1]:self.Ms[l - 1] + self.Ms[l]]
                lv.accumulate_diff(fine, self.solvers[l - 1], coarse)
            levels.append(lv)
        return mlmc_combine(levels), levels
