"""Helpers for the GPU tests: run the HIP path through the C-ABI binding and compare with
the oracle."""
import sys

import numpy as np

import oracle as O


def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def note(*msg):
    print("[gpu-case]", *msg, flush=True)
    sys.stdout.flush()


def solver_for(p: O.Problem, variant=None):
    from paper_1912_07645_amd import Solver
    s = Solver(dim=p.dim, n=p.n[:p.dim], eq=p.eq, flux=p.flux, recon=p.recon,
               integrator=p.integrator, bc=p.bc[:3], gamma=p.gamma, velocity=p.vel,
               lo=p.lo, hi=p.hi, gravity=p.gravity)
    if variant is not None:
        s.set_variant(variant)
    return s


def gpu_evolve(p: O.Problem, U0, t_end, cfl, max_steps=10**9, variant=None, mode="evolve",
               solver=None, t0=0.0):
    torch = torch_gpu()
    s = solver if solver is not None else solver_for(p, variant)
    U = torch.from_numpy(np.ascontiguousarray(U0)).to("cuda")
    B = U.shape[0]
    t = torch.full((B,), float(t0), dtype=torch.float64, device="cuda")
    steps = torch.zeros(B, dtype=torch.int64, device="cuda")
    err = torch.zeros(B, dtype=torch.int32, device="cuda")
    if mode == "evolve":
        st = s.evolve(U, t, t_end, cfl, max_steps, steps, err)
    else:
        st = s.advance(U, t, t_end, cfl, max_steps, steps, err)
    torch.cuda.synchronize()
    return (U.cpu().numpy(), t.cpu().numpy(), steps.cpu().numpy(), err.cpu().numpy(), st)


def rel_l1(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return np.abs(a - b).sum() / (den if den > 0 else 1.0)


def assert_parity(gpu, ref, tol=1e-12, bitwise=True, what=""):
    """The parity bar: relative L1 <= tol (the arithmetic contract makes the two sides agree
    bit for bit, which is checked too unless bitwise=False)."""
    r = rel_l1(gpu, ref)
    assert r <= tol, f"{what}: relative L1 {r:.3e} > {tol:g}"
    if bitwise:
        diff = np.argwhere(~(np.asarray(gpu) == np.asarray(ref)))
        assert diff.size == 0, f"{what}: {len(diff)} values differ, first at {diff[:3].tolist()}"
