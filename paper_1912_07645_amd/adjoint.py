"""Discrete adjoint (gradients of a quantity of interest with respect to the parameters of
the initial data) on top of libfv's adjoint entry points, and a torch.autograd.Function.

Every numerical step runs in libfv's kernels: the fixed-step forward run with checkpoints
(fv_adjoint_forward), the reverse sweep (fv_adjoint_backward), the kinetic-energy quantity
of interest and its gradient (fv_qoi_kinetic_energy) and the chain rule through initial data
that depends on theta through one scalar per line along y (fv_line_vjp). PyTorch provides
device memory and the autograd plumbing.
"""
from __future__ import annotations

import math

import torch

from . import fv
from .solver import Solver


class Adjoint:
    """Forward run with checkpoints and reverse sweep for a batch on a solver's grid.

    Checkpoints every `every` steps (default ceil(sqrt(nsteps))), or, with `snapshots` given,
    the binomial schedule with that many checkpoint slots besides the initial state."""

    def __init__(self, solver: Solver, batch: int, nsteps: int, dt: float, every: int = 0,
                 cfl_bound: float = 1.0, snapshots: int | None = None):
        self.solver = solver
        self.batch, self.nsteps, self.dt = int(batch), int(nsteps), float(dt)
        self.snapshots = None if snapshots is None else int(snapshots)
        if self.snapshots is None:
            self.every = int(every) if every > 0 else int(math.ceil(math.sqrt(nsteps)))
            self.handle = fv.fv_adjoint_create(solver.handle, batch, nsteps, dt, self.every,
                                               cfl_bound)
        else:
            self.every = None
            self.handle = fv.fv_adjoint_create_binomial(solver.handle, batch, nsteps, dt,
                                                        self.snapshots, cfl_bound)
        # forward runs so far: the checkpoints (and the backward sweep) belong to the last one
        self.generation = 0

    def recomputed_steps(self) -> int:
        """Forward steps the last reverse sweep ran to recompute states."""
        return fv.fv_adjoint_recomputed_steps(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                fv.fv_adjoint_destroy(h)
            except Exception:
                pass
            self.handle = None

    def _stream(self):
        fv.fv_set_stream(self.solver.handle,
                         torch.cuda.current_stream(self.solver.device).cuda_stream)

    def forward(self, U0):
        self.solver._check_state(U0)
        self._stream()
        UT = torch.empty_like(U0)
        fv.fv_adjoint_forward(self.handle, U0, UT)
        self.generation += 1
        return UT

    def backward(self, dQ_dUT):
        self.solver._check_state(dQ_dUT)
        self._stream()
        g0 = torch.empty_like(dQ_dUT)
        fv.fv_adjoint_backward(self.handle, dQ_dUT.contiguous(), g0)
        return g0

    def branch_signature(self, U0):
        """(sig, U_T): the signature of the branches the forward run from U0 takes
        (fv_adjoint_set_signature; int64 [batch], the bits of the uint64 sums) and the run's
        final state. Runs the forward pass and one reverse sweep."""
        B = self.solver._check_state(U0)
        sig = torch.zeros(B, dtype=torch.int64, device=U0.device)
        UT = self.forward(U0)
        fv.fv_adjoint_set_signature(self.handle, sig)
        try:
            self.backward(torch.zeros_like(U0))
        finally:
            fv.fv_adjoint_set_signature(self.handle, None)
        return sig, UT


def band_rows(n: int, centre: float = 0.5, half_width: float = 0.1):
    """Rows j with |y_j - centre| < half_width on the unit interval (cell centres)."""
    rows = [j for j in range(n) if abs((j + 0.5) / n - centre) < half_width]
    return rows[0], rows[-1] + 1


def kinetic_energy(solver: Solver, U, j0, j1, seed=None):
    """Q[b] and, if seed is given, seed[b] dQ[b]/dU."""
    B = solver._check_state(U)
    Q = torch.empty(B, dtype=torch.float64, device=U.device)
    grad = torch.empty_like(U) if seed is not None else None
    fv.fv_set_stream(solver.handle, torch.cuda.current_stream(solver.device).cuda_stream)
    fv.fv_qoi_kinetic_energy(solver.handle, U, B, j0, j1, seed, Q, grad)
    return Q, grad


def line_vjp(solver: Solver, lam0, D, E):
    """sum over lines of (sum_line lam0 . D) * E -> [batch][ntheta]."""
    B = solver._check_state(lam0)
    ntheta = E.shape[-1]
    out = torch.empty((B, ntheta), dtype=torch.float64, device=lam0.device)
    fv.fv_set_stream(solver.handle, torch.cuda.current_stream(solver.device).cuda_stream)
    fv.fv_line_vjp(solver.handle, lam0, D.contiguous(), E.contiguous(), ntheta, B, out)
    return out


class LineInitialDataQoI(torch.autograd.Function):
    """Q(theta): band kinetic energy after nsteps fixed steps from initial data U0(theta) that
    depends on theta through one scalar per line along y.

    forward(theta, U0, D, E, adjoint, j0, j1): theta [B][K] (for autograd), U0 the initial
    state built from theta by the caller, D = dU0/d(line scalar) (state-shaped), E = d(line
    scalar)/d theta [B][lines][K]. Returns Q [B]. backward gives dQ/dtheta."""

    @staticmethod
    def forward(ctx, theta, U0, D, E, adjoint: Adjoint, j0: int, j1: int):
        UT = adjoint.forward(U0)
        Q, _ = kinetic_energy(adjoint.solver, UT, j0, j1)
        ctx.adjoint, ctx.j0, ctx.j1 = adjoint, j0, j1
        ctx.generation = adjoint.generation
        ctx.save_for_backward(UT, D, E)
        return Q

    @staticmethod
    def backward(ctx, gQ):
        UT, D, E = ctx.saved_tensors
        adj = ctx.adjoint
        if adj.generation != ctx.generation:
            raise RuntimeError("the Adjoint handle ran another forward pass after this graph was "
                               "built: its checkpoints belong to that run; use one Adjoint per "
                               "pending backward")
        _, dQ_dUT = kinetic_energy(adj.solver, UT, ctx.j0, ctx.j1, seed=gQ.contiguous())
        lam0 = adj.backward(dQ_dUT)
        g = line_vjp(adj.solver, lam0, D, E)
        return g, None, None, None, None, None, None
