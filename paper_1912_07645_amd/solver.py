"""Solver and Stats: an object wrapper over the C names in ``fv.py``.

PyTorch supplies device memory (the state, time and status tensors, and the library
workspace) and the stream; every numerical step runs in libfv's HIP kernels.
"""
from __future__ import annotations

import torch

from . import fv


def _require_gpu_tensor(x, name, dtype):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Solver:
    """One grid, equation and scheme (Section 2.1 of the paper): an fv_solver handle."""

    def __init__(self, dim, n, eq="euler", flux="rusanov", recon="first_order",
                 integrator="forward_euler", bc="periodic", gamma=1.4, velocity=(0.0, 0.0, 0.0),
                 lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), device=None, gravity=9.81):
        self.device = torch.device(device if device is not None else "cuda")
        self.dim = dim
        self.n = tuple(list(n) + [1] * (3 - len(n)))
        self.grid = fv.make_grid(dim, n, bc, lo, hi)
        self.eq = fv.make_equation(eq, gamma, velocity, gravity)
        self.names = dict(eq=eq, flux=flux, recon=recon, integrator=integrator)
        with torch.cuda.device(self.device):
            self.handle = fv.fv_create(self.grid, self.eq, fv.FLUX[flux], fv.RECON[recon],
                                       fv.INTEGRATOR[integrator])
        self.nf = fv.fv_num_fields(self.handle)
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                fv.fv_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def state_shape(self):
        return (self.nf, self.n[2], self.n[1], self.n[0])

    def _prepare(self, batch):
        fv.fv_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)
        need = fv.fv_workspace_size(self.handle, batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            fv.fv_set_workspace(self.handle, aligned, need)

    def _check_state(self, U):
        _require_gpu_tensor(U, "state", torch.float64)
        if tuple(U.shape[1:]) != self.state_shape:
            raise ValueError(f"state shape {tuple(U.shape)} != [batch]+{self.state_shape}")
        return U.shape[0]

    def evolve(self, U, t, t_end, cfl, max_steps=10**9, steps=None, err=None) -> int:
        B = self._check_state(U)
        _require_gpu_tensor(t, "t", torch.float64)
        self._prepare(B)
        return fv.fv_evolve(self.handle, U, B, t, t_end, cfl, max_steps, steps, err)

    def advance(self, U, t, t_end, cfl, nsteps, steps=None, err=None) -> int:
        B = self._check_state(U)
        _require_gpu_tensor(t, "t", torch.float64)
        self._prepare(B)
        return fv.fv_advance(self.handle, U, B, t, t_end, cfl, nsteps, steps, err)

    def advance_noalloc(self, U, t, t_end, cfl, nsteps, steps=None, err=None) -> int:
        """fv_advance in the library's fixed per-device workspace: no allocation, no workspace
        argument (FV_ENOMEM beyond fv.fv_noalloc_capacity() bytes of workspace)."""
        B = self._check_state(U)
        _require_gpu_tensor(t, "t", torch.float64)
        fv.fv_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)
        return fv.fv_advance_noalloc(self.handle, U, B, t, t_end, cfl, nsteps, steps, err)

    def evolve_fixed_dt(self, U, dt, nsteps, cfl_bound=1.0, err=None) -> int:
        B = self._check_state(U)
        self._prepare(B)
        return fv.fv_evolve_fixed_dt(self.handle, U, B, dt, nsteps, cfl_bound, err)

    @property
    def num_quantities(self) -> int:
        return self.nf if self.names["eq"] in ("euler", "swe", "mhd") else 1

    def point_pdf(self, U, quantity, points, lo, hi, nbins, counts=None):
        """Histograms over the samples of U of `quantity` at each cell of `points` (flat cell
        indices): int64 [len(points)][nbins + 2] (bins, below lo, not below hi), added to
        `counts` if given."""
        B = self._check_state(U)
        if counts is None:
            counts = torch.zeros((len(points), nbins + 2), dtype=torch.int64, device=self.device)
        fv.fv_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)
        fv.fv_point_pdf(self.handle, U, B, quantity, points, lo, hi, nbins, counts)
        return counts

    def joint_pdf(self, U, quantity_a, quantity_b, pairs, lo_a, hi_a, lo_b, hi_b, nbins, counts=None):
        """Histograms over samples of (quantity_a at x, quantity_b at y) for each pair (x, y):
        int64 [len(pairs)][nbins * nbins + 1] (bins, then outside), added to `counts` if given."""
        B = self._check_state(U)
        if counts is None:
            counts = torch.zeros((len(pairs), nbins * nbins + 1), dtype=torch.int64, device=self.device)
        fv.fv_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)
        fv.fv_joint_pdf(self.handle, U, B, quantity_a, quantity_b, pairs, lo_a, hi_a, lo_b, hi_b,
                        nbins, counts)
        return counts

    def structure_shell(self, U, max_h, order=2, ball=False):
        """Per-sample structure functions over cube (or ball) shells:
        float64 [batch][quantities][max_h], entry h - 1 for radius h."""
        B = self._check_state(U)
        out = torch.empty((B, self.num_quantities, max_h), dtype=torch.float64, device=self.device)
        fv.fv_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)
        fv.fv_structure_shell(self.handle, U, B, max_h, order, ball, out)
        return out

    def num_variants(self) -> int:
        return fv.fv_num_variants(self.handle)

    def set_variant(self, v: int) -> None:
        fv.fv_set_variant(self.handle, v)

    def tile(self):
        return fv.fv_get_tile(self.handle)

    def tune(self, U, reps=3) -> int:
        B = self._check_state(U)
        self._prepare(B)
        return fv.fv_tune(self.handle, U, B, reps)


def mlmc_combine(levels) -> "torch.Tensor":
    """sum_l P_{l->L} mean_l on the finest (last) level's grid (levels ordered coarse to fine)."""
    fin = levels[-1].solver
    out = torch.empty((fin.nf,) + fin.state_shape[1:], dtype=torch.float64, device=fin.device)
    fv.fv_mlmc_combine([lv.handle for lv in levels], out)
    return out


def evolve_multi(solvers, states, ts, t_end, cfl, max_steps=10**9, steps=None, errs=None) -> int:
    """Evolve several grids (e.g. multilevel Monte Carlo levels) in shared launches."""
    for s, U in zip(solvers, states):
        s._prepare(s._check_state(U))
    return fv.fv_evolve_multi([s.handle for s in solvers], states, [U.shape[0] for U in states],
                              ts, t_end, cfl, max_steps, steps, errs)


class Stats:
    """Running on-device Monte Carlo statistics (Section 2.2) for a solver's grid."""

    def __init__(self, solver: Solver, max_h: int = 0):
        self.solver = solver
        self.max_h = int(max_h)
        self.handle = fv.fv_stats_create(solver.handle, self.max_h)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                fv.fv_stats_destroy(h)
            except Exception:
                pass
            self.handle = None

    def accumulate(self, U) -> None:
        B = self.solver._check_state(U)
        fv.fv_set_stream(self.solver.handle, torch.cuda.current_stream(self.solver.device).cuda_stream)
        fv.fv_stats_accumulate(self.handle, U, B)

    def accumulate_diff(self, U_fine, coarse: Solver, U_coarse) -> None:
        """Multilevel level difference: moments of q(u_fine) - P q(u_coarse)."""
        B = self.solver._check_state(U_fine)
        if coarse._check_state(U_coarse) != B:
            raise ValueError("fine and coarse batches differ")
        fv.fv_set_stream(self.solver.handle, torch.cuda.current_stream(self.solver.device).cuda_stream)
        fv.fv_stats_accumulate_diff(self.handle, U_fine, coarse.handle, U_coarse, B)

    def reset(self) -> None:
        fv.fv_stats_reset(self.handle)

    def read(self):
        s = self.solver
        nq = s.nf
        dev = s.device
        mean = torch.empty((nq,) + s.state_shape[1:], dtype=torch.float64, device=dev)
        var = torch.empty_like(mean)
        s2m = torch.empty((nq, max(self.max_h, 1)), dtype=torch.float64, device=dev)
        s2v = torch.empty_like(s2m)
        n = fv.fv_stats_read(self.handle, mean, var, s2m if self.max_h else None,
                             s2v if self.max_h else None)
        return dict(count=n, mean=mean, var=var, s2_mean=s2m[:, :self.max_h],
                    s2_var=s2v[:, :self.max_h])
