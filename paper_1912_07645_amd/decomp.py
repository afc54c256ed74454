"""Split-buffer domain decomposition (fv_decomp_*): one grid cut into subdomains with their own
arrays on one device, advanced with a halo exchange every Runge--Kutta stage, optionally
overlapped with the interior update. Argument marshalling only; the packing, copies, unpacking
and stage updates run in libfv."""
from __future__ import annotations

import torch

from . import fv
from .solver import Solver, _require_gpu_tensor


class Decomposition:
    def __init__(self, solver: Solver, parts, batch: int):
        self.solver = solver
        self.parts = tuple(list(parts) + [1] * (3 - len(parts)))
        self.batch = int(batch)
        self.handle = fv.fv_decomp_create(solver.handle, self.parts, self.batch)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                fv.fv_decomp_destroy(h)
            except Exception:
                pass
            self.handle = None

    def _stream(self):
        fv.fv_set_stream(self.solver.handle,
                         torch.cuda.current_stream(self.solver.device).cuda_stream)

    def _check(self, U):
        if self.solver._check_state(U) != self.batch:
            raise ValueError(f"state batch {U.shape[0]} != decomposition batch {self.batch}")

    def scatter(self, U):
        self._check(U)
        self._stream()
        fv.fv_decomp_scatter(self.handle, U)

    def gather(self, U):
        self._check(U)
        self._stream()
        fv.fv_decomp_gather(self.handle, U)

    def advance(self, t, t_end, cfl, nsteps, steps=None, err=None, overlap=True,
                dma=False) -> int:
        _require_gpu_tensor(t, "t", torch.float64)
        if t.numel() != self.batch:
            raise ValueError("t must have one entry per sample")
        self._stream()
        return fv.fv_decomp_advance(self.handle, t, t_end, cfl, nsteps, steps, err, overlap, dma)

    def profile(self, on: bool):
        fv.fv_decomp_profile_enable(self.handle, on)

    def profile_read(self):
        """(step_ms, copy_ms, steps) accumulated while profiling."""
        return fv.fv_decomp_profile_read(self.handle)

    def info(self) -> dict:
        return fv.fv_decomp_info(self.handle)
