"""Benchmark of the finite-volume hot path on one MI355X.

Default workload: 2D compressible Euler, Kelvin--Helmholtz shear layer on the periodic unit
square at 1024^2 cells, FP64, WENO3 reconstruction, HLLC flux, SSP-RK3, CFL 0.4 (seed 1912,
sample 0). One "step" is one full time step of the whole path: the CFL wave-speed reduction,
three fused Runge--Kutta stage launches (ghost fill, reconstruction, flux, divergence, stage
combination) and the device-side step control.

Prints ONE JSON line: cell-updates/s (cells x steps / wall time of the timed region, the
state already resident in HBM), the roofline of the dominant kernel (the stage kernel,
timed with HIP events on the library's stream over its own launches) and the CPU oracle's
rate on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload kh2d|kh2d_roe|kh2d_godunov|kh2d_ec4|kh3d|mc|sod|swe2d|mhd2d|mlmc|adjoint|halo|stats]
    python bench.py --copy-calibration     # plain copy of known size, for rocprof counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, 8 TB/s
# FP64 issue peak: 256 CUs x 64 FP64 lanes per clock x 2.4 GHz = 39.3e12 lane-ops/s. The
# published 78.6 TFLOP/s counts an FMA as 2 flops; here every FP64 operation, an FMA
# included, is one lane-op, since the stage kernel is bound by issuing them.
FP64_LANE_OPS_PEAK = 256 * 64 * 2.4e9

# FP64 lane-operations the arithmetic contract needs, with each face counted once: every
# + - x, fused multiply-add and comparison/select counts 1, a correctly rounded division 10
# and a square root 14 (the lengths of their gfx950 expansions). Derivation in the design
# notes.
WENO3_PER_COMPONENT = 43        # both face values of one component (shared indicator)
EULER_PRIM = {1: 31, 2: 34, 3: 37}            # primitives of one face state
EULER_FLUX = {1: 4, 2: 5, 3: 6}                # physical flux of one face state
HLLC = {1: 76, 2: 85, 3: 94}                   # wave speeds, contact, star state, selects
ROE = {1: 193, 2: 222, 3: 251}                 # Roe averages, strengths, entropy fix, dissipation
DIVERGENCE_RK = {1: 3 + 5, 2: 6 + 5, 3: 9 + 5}  # per component: flux difference sum, stage
CFL_CELL = {1: 45, 2: 47, 3: 55}              # per cell, last stage only


# Flops per cell-stage of the same contract (an FMA counts two flops, divisions and square roots
# by their expansions): the lane-op figure with every fused multiply-add unfused.
FLOPS_PER_CELL_STAGE = {("hllc", 2): 797.7, ("hllc", 3): 1399.3}
FP64_FLOPS_PEAK = 78.6e12   # MI355X FP64 vector, published (an FMA as two flops)


def lane_ops_per_cell_stage(dim: int, integrator: str, flux: str = "hllc") -> float:
    """WENO3 + HLLC (or Roe) Euler: algorithmic FP64 lane-ops per cell per Runge--Kutta stage."""
    nf = dim + 2
    riemann = HLLC[dim] if flux == "hllc" else ROE[dim]
    face = nf * WENO3_PER_COMPONENT + 2 * (EULER_PRIM[dim] + EULER_FLUX[dim]) + riemann
    stages = {"forward_euler": 1, "ssprk2": 2, "ssprk3": 3}[integrator]
    return dim * face + nf * DIVERGENCE_RK[dim] + CFL_CELL[dim] / stages

# Algorithmic HBM bytes per cell per full step (streaming minimum: each stage reads its
# input state once, stages >= 2 re-read U^n, every stage writes its output once; halos and
# faces never leave the chip).
def algorithmic_bytes_per_cell_step(nf: int, integrator: str) -> int:
    per = 8 * nf
    if integrator == "forward_euler":
        return 2 * per
    if integrator == "ssprk2":
        return 2 * per + 3 * per
    return 2 * per + 3 * per + 3 * per


WORKLOADS = {
    "kh2d": dict(name="kh2d_1024x1024_weno3_hllc_ssprk3", dim=2, n=1024, flux="hllc",
                 recon="weno3", integrator="ssprk3", cfl=0.4, batch=1, seed=1912,
                 steps=2000, warmup=100, cpu_steps=96),
    "kh3d": dict(name="kh3d_512^3_weno3_hllc_ssprk3", dim=3, n=512, flux="hllc",
                 recon="weno3", integrator="ssprk3", cfl=0.4, batch=1, seed=1914,
                 steps=20, warmup=2, cpu_steps=1),
    "kh2d_roe": dict(name="kh2d_1024x1024_weno3_roe_ssprk3", dim=2, n=1024, flux="roe",
                     recon="weno3", integrator="ssprk3", cfl=0.4, batch=1, seed=1912,
                     steps=1000, warmup=50, cpu_steps=4),
    "kh2d_godunov": dict(name="kh2d_1024x1024_weno3_godunov_ssprk3", dim=2, n=1024,
                         flux="godunov", recon="weno3", integrator="ssprk3", cfl=0.4, batch=1,
                         seed=1912, steps=200, warmup=20, cpu_steps=1),
    "kh2d_ec4": dict(name="kh2d_1024x1024_fourth_order_entropy_conservative_ssprk3", dim=2,
                     n=1024, flux="ec4", recon="first_order", integrator="ssprk3", cfl=0.4,
                     batch=1, seed=1912, steps=400, warmup=20, cpu_steps=2),
    "mhd2d": dict(name="mhd_orszag_tang_1024x1024_muscl_rusanov_ssprk2", eq="mhd", dim=2, n=1024,
                  flux="rusanov", recon="muscl_minmod", integrator="ssprk2", cfl=0.4, batch=1,
                  seed=0, gamma=5.0 / 3.0, steps=1000, warmup=50, cpu_steps=4),
    "swe2d": dict(name="swe_circular_dam_break_1024x1024_muscl_hll_ssprk2", eq="swe", dim=2,
                  n=1024, flux="hll", recon="muscl_minmod", integrator="ssprk2", cfl=0.4,
                  batch=1, seed=0, steps=2000, warmup=100, cpu_steps=8),
    "mc": dict(name="kh2d_256x256_x1024_samples_weno3_hllc_ssprk3", dim=2, n=256, flux="hllc",
               recon="weno3", integrator="ssprk3", cfl=0.4, batch=1024, seed=1912,
               steps=50, warmup=5, cpu_steps=2),
    "mlmc": dict(name="mlmc_kh2d_64-512_4096-64_samples_muscl_hll_ssprk2", dim=2, n=512,
                 flux="hll", recon="muscl_minmod", integrator="ssprk2", cfl=0.4, batch=64,
                 seed=1913, steps=1, warmup=1, cpu_steps=2, t_end=1.0,
                 ns=(64, 128, 256, 512), Ms=(4096, 1024, 256, 64)),
    "adjoint": dict(name="adjoint_kh2d_256x256_x64_samples_muscl_rusanov_ssprk3_500_steps", dim=2,
                    n=256, flux="rusanov", recon="muscl_minmod", integrator="ssprk3", cfl=0.4,
                    batch=64, seed=1915, steps=1, warmup=1, cpu_steps=2, nsteps=500),
    "sod": dict(name="sod_1024_first_order_rusanov_forward_euler", dim=1, n=1024,
                flux="rusanov", recon="first_order", integrator="forward_euler", cfl=0.45,
                batch=1, seed=0, steps=1000, warmup=100, cpu_steps=1000),
}


# rocprofv3 summaries of the stage kernel (commands, counters, traffic) per workload
PROFILE_SUMMARY = {"kh2d": "stage_kernel_kh2d_1024.md", "kh3d": "stage_kernel_kh3d_512.md",
                   "kh2d_roe": "stage_kernel_kh2d_roe_1024.md", "swe2d": "stage_kernel_swe2d_1024.md",
                   "kh2d_godunov": "stage_kernel_kh2d_godunov_1024.md",
                   "kh2d_ec4": "stage_kernel_kh2d_ec4_1024.md",
                   "mhd2d": "stage_kernel_mhd2d_1024.md"}


def initial_state(w):
    import numpy as np
    import fv_inputs as fi
    if w.get("eq") == "swe":
        return fi.swe_circular_dam_break(w["n"], batch=w["batch"])
    if w.get("eq") == "mhd":
        return fi.orszag_tang_state(w["n"], gamma=w["gamma"])
    if w["dim"] == 1:
        return fi.sod_state(w["n"])
    if w["dim"] == 2:
        c, phi = fi.kh_coefficients(w["seed"], np.arange(w["batch"]))
        return fi.kh2d_state(w["n"], c, phi)
    cx, px, cz, pz = fi.kh3d_coefficients(w["seed"], np.arange(w["batch"]))
    return fi.kh3d_state(w["n"], cx, px, cz, pz)


# The sources that define the stage kernel of each benchmarked workload: the headers every
# stage kernel compiles from, plus the instantiation unit that builds the workload's kernel. A
# change to any of them invalidates that workload's committed traffic counters.
STAGE_KERNEL_COMMON = ("fv_common.h", "fv_physics.h", "fv_registry.h", "fv_stage.h", "fv_stage_z.h")
STAGE_KERNEL_UNIT = {"kh2d": "inst_euler2d_hot.hip", "kh3d": "inst_euler3d_hot.hip",
                     "kh2d_roe": "inst_more2d.hip", "swe2d": "inst_swe.hip",
                     "kh2d_godunov": "inst_godunov.hip", "kh2d_ec4": "inst_ec.hip",
                     "mhd2d": "inst_mhd.hip"}


def stage_kernel_sources(workload: str):
    return STAGE_KERNEL_COMMON + (STAGE_KERNEL_UNIT[workload],)


def kernel_sources_hash(workload: str) -> str:
    return sources_hash(stage_kernel_sources(workload))


# The statistics pass: the sources of its kernels and the summary holding its counters.
STATS_KERNEL_SOURCES = ("fv_common.h", "fv_stats.h", "fv_stats.hip")
STATS_SUMMARY = "stats_mc_256x1024.md"


def sources_hash(names) -> str:
    h = hashlib.sha256()
    for name in names:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1912_07645_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_stats_traffic():
    """HBM bytes of one whole-batch Welford launch from the committed counter summary, if it was
    taken on the current sources of the statistics kernels (else None)."""
    path = os.path.join(ROOT, "profiles", STATS_SUMMARY)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"sources_sha256:\s*([0-9a-f]+)", text)
    m_val = re.search(r"traffic_bytes_per_call:\s*([0-9.e+]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != sources_hash(STATS_KERNEL_SOURCES):
        return None
    return float(m_val.group(1))


def measured_traffic(workload: str, variant: int):
    """HBM bytes per stage launch of tuner variant `variant` from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources and on that variant (else
    None). The summary names its variant (`traffic_variant: N` before the figure, or the form
    `traffic_bytes_per_launch[variant N]: X`)."""
    path = os.path.join(ROOT, "profiles", PROFILE_SUMMARY.get(workload, "-"))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"sources_sha256:\s*([0-9a-f]+)", text)
    if not m_hash or workload not in STAGE_KERNEL_UNIT \
            or m_hash.group(1) != kernel_sources_hash(workload):
        return None
    by_variant = {}
    m_var = re.search(r"traffic_variant:\s*(\d+)", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.e+]+)", text)
    if m_var and m_val:
        by_variant[int(m_var.group(1))] = float(m_val.group(1))
    for v, x in re.findall(r"traffic_bytes_per_launch\[variant (\d+)\]:\s*([0-9.e+]+)", text):
        by_variant[int(v)] = float(x)
    return by_variant.get(int(variant))


def cpu_baseline(w, U0, steps):
    """The oracle as it stands, on all the host's cores over a bounded prefix of the run, and
    on one core over a shorter prefix."""
    import oracle as O
    cores = O.set_threads(0)
    one = _cpu_rate(O, w, U0, max(1, steps // 8), threads=1)
    O.set_threads(cores)
    out = _cpu_rate(O, w, U0, steps, threads=cores)
    out["one_core"] = one
    return out


def _cpu_rate(O, w, U0, steps, threads):
    O.set_threads(threads)
    p = O.Problem(dim=w["dim"], n=(w["n"],) * w["dim"], eq=w.get("eq", "euler"), flux=w["flux"],
                  recon=w["recon"], integrator=w["integrator"],
                  bc=("transmissive",) if w["dim"] == 1 else ("periodic",) * 3,
                  gamma=w.get("gamma", 1.4))
    samples = min(U0.shape[0], 2)
    U = U0[:samples]
    t0 = time.perf_counter()
    _, _, k, _ = O.evolve(p, U, 1e9, w["cfl"], max_steps=steps)
    el = time.perf_counter() - t0
    cells = w["n"] ** w["dim"]
    return {"value": cells * int(k.sum()) / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {steps} steps of {samples} sample(s) of the same workload "
                      f"({cells} cells each), {el:.1f} s"}


def copy_calibration():
    """A plain device copy of 1 GiB, ten times (for FETCH_SIZE / WRITE_SIZE scaling)."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 10}))


def run_mlmc(a, w):
    """The mixed multilevel batch: every level's groups evolved together to T = 1 in shared
    launches, then level statistics and the estimate on the finest grid. One "step" here is one
    whole multilevel run (the state is reloaded before each run, outside the timed region)."""
    import numpy as np
    import torch
    import fv_inputs as fi
    from paper_1912_07645_amd.mlmc import MultilevelRun

    ns, Ms = w["ns"], w["Ms"]
    groups = fi.mlmc_inputs(ns, Ms, seed=w["seed"])
    run = MultilevelRun(ns, Ms, dim=2, eq="euler", flux=w["flux"], recon=w["recon"],
                        integrator=w["integrator"], device="cuda:0")
    K = a.steps if a.steps is not None else w["steps"]
    W = a.warmup if a.warmup is not None else w["warmup"]
    dev_groups = [torch.from_numpy(g).to("cuda:0") for g in groups]
    tuned = run.tune(dev_groups, w["cfl"]) if a.variant is None else a.variant
    for s in run.solvers:
        s.set_variant(tuned)
    times, cell_updates = [], 0
    steps_per_grid = None
    for r in range(W + K):
        G = [g.clone() for g in dev_groups]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, ts, errs = run.evolve(G, w["t_end"], w["cfl"])
        est, levels = run.statistics(G)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert st == 0
        if r >= W:
            times.append(el)
        steps_per_grid = [int(k.sum()) for k in run.last_steps]
    for l, n in enumerate(ns):
        cell_updates += n * n * steps_per_grid[l]
    el = sum(times) / len(times)
    out = {
        "metric": "FP64 cell-updates/s", "value": cell_updates / el, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": el * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["name"], "grids": list(ns), "samples_per_level": list(Ms),
                   "samples_per_grid": [int(g.shape[0]) for g in groups],
                   "sample_steps_per_grid": steps_per_grid, "t_end": w["t_end"],
                   "cfl": w["cfl"], "seed": w["seed"],
                   "step": "one whole multilevel run (all levels to T, statistics, estimate)",
                   "tile": list(run.solvers[0].tile()[0]), "tuned_variant": tuned},
        "mlmc_runs_per_s": 1.0 / el,
        "roofline": None,
    }
    print(json.dumps(out))


def run_adjoint(a, w):
    """Gradient of the band kinetic energy with respect to the 20 perturbation coefficients of
    each of 64 samples (256^2, 500 fixed steps): the plain forward run, then the forward run
    with sqrt(N) checkpoints plus the reverse sweep; reports the adjoint/forward cost ratio."""
    import numpy as np
    import torch
    import fv_inputs as fi
    from paper_1912_07645_amd import Solver
    from paper_1912_07645_amd.adjoint import Adjoint, LineInitialDataQoI, band_rows

    n, B, N = w["n"], w["batch"], w["nsteps"]
    c, phi = fi.kh_coefficients(w["seed"], np.arange(B))
    U0, D, E = fi.kh2d_state_and_jacobian(n, c, phi)
    s = Solver(dim=2, n=(n, n), eq="euler", flux=w["flux"], recon=w["recon"],
               integrator=w["integrator"], device="cuda:0")
    dev = torch.device("cuda:0")
    U0d, Dd, Ed = (torch.from_numpy(x).to(dev) for x in (U0, D, E))
    outer = (0.5 + (1.4 * 2.5 / 1.0) ** 0.5) * n       # max speed of the unperturbed outer state
    Ut = U0d[:1].clone()
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    k = torch.zeros(1, dtype=torch.int64, device=dev)
    s.advance(Ut, t, 1e9, 1e-9, 1, k)   # dt of the first step = 1e-9 / M0: read M0 back
    M0 = 1e-9 / float(t[0])
    dt = w["cfl"] / M0
    j0, j1 = band_rows(n)
    K = a.steps if a.steps is not None else w["steps"]
    W = a.warmup if a.warmup is not None else w["warmup"]
    tuned = s.tune(U0d) if a.variant is None else a.variant   # the forward stage's tile
    s.set_variant(tuned)
    adj = Adjoint(s, B, N, dt, cfl_bound=0.6)
    fwd, grad = [], []
    for r in range(W + K):
        U = U0d.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.evolve_fixed_dt(U, dt, N, 0.6)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        theta = torch.tensor(np.concatenate([c, phi], axis=1), device=dev, requires_grad=True)
        Q = LineInitialDataQoI.apply(theta, U0d, Dd, Ed, adj, j0, j1)
        Q.sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r >= W:
            fwd.append(t1 - t0)
            grad.append(t2 - t1)
    tf, tg = sum(fwd) / len(fwd), sum(grad) / len(grad)
    # the same gradient with binomial checkpointing: less memory, more recomputation
    snaps = w.get("binomial_snapshots", 10)
    adjb = Adjoint(s, B, N, dt, cfl_bound=0.6, snapshots=snaps)
    tb = []
    for r in range(2):
        theta = torch.tensor(np.concatenate([c, phi], axis=1), device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Q = LineInitialDataQoI.apply(theta, U0d, Dd, Ed, adjb, j0, j1)
        Q.sum().backward()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t1)
    nst = {"forward_euler": 1, "ssprk2": 2, "ssprk3": 3}[w["integrator"]]
    binomial = {"snapshots": snaps, "gradient_ms": tb[-1] * 1e3,
                "recomputed_steps": adjb.recomputed_steps(),
                "state_copies": snaps + nst + 5,
                "segment_state_copies": -(-N // adj.every) + adj.every * nst + 4}
    del adjb
    cells = n * n * B * N
    out = {
        "metric": "FP64 cell-updates/s", "value": cells / tg, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": tg * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["name"], "grid": [n, n], "samples": B, "time_steps": N,
                   "dt": dt, "checkpoint_every": adj.every, "outer_state_speed_check": outer,
                   "step": "one gradient evaluation (forward with checkpoints + reverse sweep)",
                   "forward_tile": list(s.tile()[0]), "tuned_variant": tuned},
        "forward_ms": tf * 1e3, "gradient_ms": tg * 1e3, "adjoint_over_forward_cost": tg / tf,
        "binomial_checkpointing": binomial,
        "roofline": None,
    }
    return out


# LDS roof of the shell structure functions: every (cell, offset) term reads one double from
# LDS (plus 3 FP64 operations, whose issue ceiling, 13.1e12 terms/s, lies above): 256 CUs x
# 128 B per clock x 2.4 GHz / 8 B.
SHELL_TERMS_PEAK = 256 * 128 * 2.4e9 / 8


def functionals(s, U, cells, B):
    """Point PDFs (1024 cells x 4 quantities, 64 bins), joint PDFs (256 pairs of neighbouring
    cells, 32 x 32 bins) and cube-shell structure functions (order 2, radius 1..8) of the
    batch, each timed once after an untimed call."""
    import torch
    N = cells
    points = list(range(0, N, max(1, N // 1024)))[:1024]
    pairs = [(c, (c + 1) % N) for c in points[:256]]
    ranges = ((0.9, 2.1), (-0.6, 0.6), (-0.05, 0.05), (2.4, 3.6))
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    out["point_pdf_ms"] = timed(lambda: [s.point_pdf(U, q, points, lo, hi, 64)
                                         for q, (lo, hi) in enumerate(ranges)])
    out["joint_pdf_ms"] = timed(lambda: s.joint_pdf(U, 0, 3, pairs, *ranges[0], *ranges[3], 32))
    H = 8
    ms = timed(lambda: s.structure_shell(U, H, 2, False))
    terms = N * B * s.num_quantities * sum(8 * h for h in range(1, H + 1))   # 2D cube shells
    out["shell_cube_h8_ms"] = ms
    out["shell_terms_per_s"] = terms / (ms * 1e-3)
    out["shell_lds_roof_frac"] = terms / (ms * 1e-3) / SHELL_TERMS_PEAK
    return out


def run_halo(a):
    """Split-buffer halo exchange (one GPU emulating the subdomains of several): the 1024^2
    Kelvin--Helmholtz run split along x, along y and both ways, and the 512^3 run split along
    z. Per split: the step time with the interior updated while the halo copies run
    (overlap), with the exchange before the whole update (serial), the unsplit step time on
    the same tile kernel, and the copies' own device time per step (events on the copy stream,
    serial mode), from which the fraction of copy time the overlap hides follows."""
    import numpy as np
    import torch
    import fv_inputs as fi
    from paper_1912_07645_amd import Solver
    from paper_1912_07645_amd.decomp import Decomposition

    dev = torch.device("cuda:0")
    out = {"metric": "split-buffer step time (ms) and hidden fraction of halo-copy time",
           "n_gpus": 1, "data": "synthetic", "dtype": "f64", "cases": []}

    def timed(fn, reps=3):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        return best

    for dim, n, splits, K in ((2, 1024, ((2, 1), (1, 2), (2, 2)), 320), (3, 512, ((1, 1, 2),), 16)):
        if dim == 2:
            c, phi = fi.kh_coefficients(1912, [0])
            U0 = fi.kh2d_state(n, c, phi)
        else:
            cx, px, cz, pz = fi.kh3d_coefficients(1914, [0])
            U0 = fi.kh3d_state(n, cx, px, cz, pz)
        s = Solver(dim=dim, n=(n,) * dim, eq="euler", flux="hllc", recon="weno3",
                   integrator="ssprk3", device=dev)
        want = (16, 15, 1) if dim == 2 else (8, 8, 4)     # the tile of the split-run kernel
        for v in range(s.num_variants()):
            s.set_variant(v)
            if tuple(s.tile()[0]) == want:
                break
        U = torch.from_numpy(U0).to(dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        s.advance(U, t, 1e9, 0.4, 2)
        unsplit = timed(lambda: s.advance(U, t, 1e9, 0.4, K)) / K
        for parts in splits:
            d = Decomposition(s, parts, 1)
            d.scatter(U)
            td = torch.zeros(1, dtype=torch.float64, device=dev)
            info = d.info()
            case = {"workload": f"kh{dim}d_{n}^{dim}_weno3_hllc_ssprk3", "parts": list(parts),
                    "messages_per_stage": info["messages"],
                    "halo_bytes_per_stage": info["halo_bytes_per_stage"],
                    "interior_tiles": info["interior_tiles"], "shell_tiles": info["shell_tiles"],
                    "unsplit_ms_per_step": unsplit * 1e3}
            for dma in (False, True):
                key = "dma" if dma else "copy_kernels"
                d.advance(td, 1e9, 0.4, 16, overlap=True, dma=dma)
                ov = timed(lambda: d.advance(td, 1e9, 0.4, K, overlap=True, dma=dma)) / K
                d.advance(td, 1e9, 0.4, 16, overlap=False, dma=dma)
                se = timed(lambda: d.advance(td, 1e9, 0.4, K, overlap=False, dma=dma)) / K
                d.profile(True)
                d.advance(td, 1e9, 0.4, 8, overlap=False, dma=dma)
                step_ms, copy_ms, nprof = d.profile_read()
                d.profile(False)
                copy = copy_ms / nprof * 1e-3
                case[key] = {"overlap_ms_per_step": ov * 1e3, "serial_ms_per_step": se * 1e3,
                             "copy_ms_per_step": copy * 1e3,
                             "hidden_copy_fraction": max(0.0, min(1.0, (se - ov) / copy)) if copy > 0 else None,
                             "overlap_over_unsplit": ov / unsplit}
            out["cases"].append(case)
            del d
            torch.cuda.empty_cache()
        del s, U
        torch.cuda.empty_cache()
    print(json.dumps(out))


def run_stats(a):
    """On-device Monte Carlo statistics of a batch of 1024 Kelvin--Helmholtz samples of 256^2
    (WENO3 + HLLC + SSP-RK3, 20 steps from the seed-1912 initial data): the per-cell Welford
    pass alone (max_h = 0) against the HBM roof (the state read once: 32 B per cell and sample,
    plus the running moments read and written once per call), and the pass with the structure
    functions S_q(h), h = 1..32, whose sums (a difference and a fused multiply-add per (cell,
    axis, lag, quantity) term) are priced against the FP64 issue ceiling. Device time of each
    call from HIP events on the caller's stream (the library's stream is ordered between them);
    median of the timed calls after one untimed call."""
    import numpy as np
    import torch
    import fv_inputs as fi
    from paper_1912_07645_amd import Solver, Stats

    B, n, H = 1024, 256, 32
    K = a.steps if a.steps is not None else 5
    dev = torch.device("cuda:0")
    c, phi = fi.kh_coefficients(1912, np.arange(B))
    s = Solver(dim=2, n=(n, n), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3",
               device=dev)
    U = torch.from_numpy(fi.kh2d_state(n, c, phi)).to(dev)
    t = torch.zeros(B, dtype=torch.float64, device=dev)
    s.advance(U, t, 1e9, 0.4, 20)
    cells = n * n
    nq = s.num_quantities

    def device_ms(st):
        st.reset()
        st.accumulate(U)
        times = []
        for _ in range(K):
            st.reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            st.accumulate(U)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times))

    welford_ms = device_ms(Stats(s, max_h=0))
    full_ms = device_ms(Stats(s, max_h=H))
    bytes_welford = B * cells * nq * 8 + 2 * 2 * cells * nq * 8
    terms = B * cells * 2 * H * nq
    welford_gbs = bytes_welford / (welford_ms * 1e-3) / 1e9
    sf_ms = full_ms - welford_ms
    out = {
        "metric": "MC statistics of a 1024 x 256^2 batch: device ms per batch", "value": full_ms,
        "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": K, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "stats_kh2d_256x256_x1024_samples_lag32", "samples": B,
                   "grid": [n, n], "quantities": nq, "max_h": H},
        "welford_ms": welford_ms, "full_ms": full_ms,
        "roofline": {"bound": "hbm", "kernel": "welford (max_h = 0)", "achieved": welford_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": welford_gbs / HBM_PEAK_GBS,
                     "traffic": measured_stats_traffic(),
                     "algorithmic_bytes_per_call": bytes_welford},
        "structure_functions": {"bound": "alu", "ms": sf_ms, "terms": terms,
                                "lane_ops_per_term": 2,
                                "achieved": 2 * terms / (sf_ms * 1e-3) / 1e12,
                                "peak": FP64_LANE_OPS_PEAK / 1e12, "unit": "T lane-ops/s",
                                "frac": 2 * terms / (sf_ms * 1e-3) / FP64_LANE_OPS_PEAK},
    }
    print(json.dumps(out))


def per_sample_rate(s, U, cfl, K, B1):
    """The same kernels with one sample per launch (the unbatched way), over B1 samples."""
    import torch
    t = torch.zeros(1, dtype=torch.float64, device=U.device)
    k = torch.zeros(1, dtype=torch.int64, device=U.device)
    Us = [U[b:b + 1].clone() for b in range(B1)]
    s.advance(Us[0], t, 1e9, cfl, 2, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(B1):
        t.zero_()
        s.advance(Us[b], t, 1e9, cfl, K, k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return B1 * K / el, Us


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="kh2d", choices=sorted(WORKLOADS) + ["halo", "stats"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="kh2d only: skip the short batched-MC and adjoint measurements")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--variant", type=int, default=None, help="tile variant (default: tuned)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file remembering the tuned variant per workload")
    a = ap.parse_args()

    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or ws != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(several GPUs would each hold a subdomain of the grid, with a halo exchange "
              "between them every stage)",
              file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    if a.workload == "mlmc":
        run_mlmc(a, WORKLOADS["mlmc"])
        return
    if a.workload == "adjoint":
        print(json.dumps(run_adjoint(a, WORKLOADS["adjoint"])))
        return
    if a.workload == "halo":
        run_halo(a)
        return
    if a.workload == "stats":
        run_stats(a)
        return

    out = measure(a, dict(WORKLOADS[a.workload]))
    print(json.dumps(out))


def measure(a, w, steps=None, warmup=None):
    """Time K full steps of workload w; returns the JSON record."""
    import numpy as np
    import torch
    from paper_1912_07645_amd import Solver, fv

    K = a.steps if a.steps is not None else (steps if steps is not None else w["steps"])
    W = a.warmup if a.warmup is not None else (warmup if warmup is not None else w["warmup"])
    dev = torch.device("cuda:0")
    U0 = initial_state(w)
    bc = "transmissive" if w["dim"] == 1 else "periodic"
    s = Solver(dim=w["dim"], n=(w["n"],) * w["dim"], eq=w.get("eq", "euler"), flux=w["flux"],
               recon=w["recon"], integrator=w["integrator"], bc=bc, gamma=w.get("gamma", 1.4),
               device=dev)
    U = torch.from_numpy(U0).to(dev)
    B = U.shape[0]
    t = torch.zeros(B, dtype=torch.float64, device=dev)
    steps_t = torch.zeros(B, dtype=torch.int64, device=dev)
    err = torch.zeros(B, dtype=torch.int32, device=dev)
    cache = {}
    if a.tune_cache and os.path.exists(a.tune_cache):
        cache = json.load(open(a.tune_cache))
    if a.variant is not None:
        s.set_variant(a.variant)
        tuned = a.variant
    elif w["name"] in cache:
        tuned = int(cache[w["name"]])
        s.set_variant(tuned)
    else:
        tuned = s.tune(U, reps=3) if s.num_variants() > 1 else 0
        if a.tune_cache:
            cache[w["name"]] = tuned
            json.dump(cache, open(a.tune_cache, "w"))
    tile, _ = s.tile()

    t_end = 1e9
    s.advance(U, t, t_end, w["cfl"], W, steps_t, err)
    torch.cuda.synchronize()
    # timed region: K full steps, state resident in HBM. HIP events on the caller's stream
    # (the library's stream is ordered after it on entry and before it on exit) bracket the
    # region on the device as well.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    st = s.advance(U, t, t_end, w["cfl"], K, steps_t, err)
    ev1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert st == 0 and int(steps_t.min()) == K, (st, steps_t.min())
    cells = w["n"] ** w["dim"]
    value = cells * B * K / el

    # mean stage-launch duration: the device time of the timed region over its stage launches
    # (K steps x stages). It includes the per-step control kernel and the launch gaps, so it
    # bounds the stage kernel's own duration from above.
    nstages = {"forward_euler": 1, "ssprk2": 2, "ssprk3": 3}[w["integrator"]]
    launches = K * nstages
    nf = s.nf
    bytes_step = algorithmic_bytes_per_cell_step(nf, w["integrator"]) * cells * B
    avg_launch_s = ev0.elapsed_time(ev1) * 1e-3 / launches
    bytes_per_launch = bytes_step / nstages
    achieved = bytes_per_launch / avg_launch_s / 1e9
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_per_launch,
           "traffic": measured_traffic(a.workload, tuned)}
    if w.get("eq", "euler") == "euler" and w["recon"] == "weno3" and w["flux"] in ("hllc", "roe"):
        ops_launch = lane_ops_per_cell_stage(w["dim"], w["integrator"], w["flux"]) * cells * B
        alu_tops = ops_launch / avg_launch_s / 1e12
        # FP64 issue: every operation (an FMA included) is one lane-op; peak 256 CUs x 64 FP64
        # lanes x 2.4 GHz. The flop figure beside it counts an FMA as two, against the
        # published 78.6 TFLOP/s.
        roof = {"bound": "alu", "achieved": alu_tops, "peak": FP64_LANE_OPS_PEAK / 1e12,
                "unit": "T lane-ops/s", "frac": alu_tops * 1e12 / FP64_LANE_OPS_PEAK,
                "traffic": hbm["traffic"], "kernel": "stage_kernel",
                "avg_launch_us": avg_launch_s * 1e6,
                "algorithmic_fp64_lane_ops_per_launch": ops_launch,
                "fp64_lane_ops_per_cell_stage": lane_ops_per_cell_stage(w["dim"], w["integrator"], w["flux"]),
                "hbm": hbm}
        fl = FLOPS_PER_CELL_STAGE.get((w["flux"], w["dim"]))
        if fl is not None:
            tf = fl * cells * B / avg_launch_s
            roof["flops"] = {"per_cell_stage": fl, "achieved_tflops": tf / 1e12,
                             "peak_tflops": FP64_FLOPS_PEAK / 1e12, "frac": tf / FP64_FLOPS_PEAK}
    else:
        # a 1D run on the single-workgroup variant (tile = the whole grid) has no stage
        # launches: its "launch" figure is then the device time per stage of the one kernel
        small = w["dim"] == 1 and tile[0] == w["n"]
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None if small else hbm["traffic"],
                "kernel": "small1d_kernel" if small else "stage_kernel",
                "avg_launch_us": avg_launch_s * 1e6,
                "algorithmic_bytes_per_launch": bytes_per_launch}

    out = {
        "metric": "FP64 cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": [w["n"]] * w["dim"], "samples": B,
                   "cells_per_sample": cells, "cfl": w["cfl"], "seed": w["seed"],
                   "tile": list(tile), "tuned_variant": tuned},
        "roofline": roof,
        "hbm_frac_whole_step": bytes_step * K / el / 1e9 / HBM_PEAK_GBS,
    }
    if a.workload == "kh2d" and not a.no_extras:
        # the other two headline figures, measured briefly on their own configurations
        ea = argparse.Namespace(steps=None, warmup=None, no_cpu=True, tune_cache=a.tune_cache,
                                variant=None, workload="mc", no_extras=True)
        mc = measure(ea, dict(WORKLOADS["mc"]), steps=20, warmup=2)
        out["batched_mc"] = {k: mc[k] for k in (
            "mc_sample_steps_per_s", "per_sample_launch_sample_steps_per_s",
            "batched_speedup_over_per_sample_launches", "stats_ms_for_batch", "stats_ms_timing",
            "functionals")}
        out["batched_mc"]["config"] = mc["config"]["workload"]
        adj = run_adjoint(argparse.Namespace(steps=1, warmup=1, variant=None), WORKLOADS["adjoint"])
        out["adjoint"] = {k: adj[k] for k in ("forward_ms", "gradient_ms",
                                               "adjoint_over_forward_cost",
                                               "binomial_checkpointing")}
        out["adjoint"]["config"] = adj["config"]["workload"]
    if w["name"].startswith("sod"):
        # the latency-bound configuration: time to solution (T = 0.2) on the tiled path and
        # on the single-workgroup time loop
        tts = {}
        variants = [("tiled", 0)]
        s.set_variant(s.num_variants() - 1)
        if s.num_variants() > 1 and s.tile()[0][0] == w["n"]:
            variants.append(("single_workgroup", s.num_variants() - 1))
        for name, v in variants:
            s.set_variant(v)
            for r in range(2):
                U2 = torch.from_numpy(U0).to(dev)
                t2 = torch.zeros(B, dtype=torch.float64, device=dev)
                k2 = torch.zeros(B, dtype=torch.int64, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.evolve(U2, t2, 0.2, w["cfl"], 10**6, k2, err)
                torch.cuda.synchronize()
                el2 = time.perf_counter() - t0
            tts[name] = {"ms": el2 * 1e3, "steps": int(k2[0])}
        out["time_to_solution_T0.2"] = tts
    if w["name"].startswith("kh2d_256x256_x1024"):
        from paper_1912_07645_amd import Stats
        out["mc_sample_steps_per_s"] = B * K / el
        # batched against per-sample launches of the same kernels, on the first 32 samples
        U2 = torch.from_numpy(U0).to(dev)
        t2 = torch.zeros(B, dtype=torch.float64, device=dev)
        s.advance(U2[:32], t2[:32], 1e9, w["cfl"], 2)
        single, Us = per_sample_rate(s, torch.from_numpy(U0[:32]).to(dev), w["cfl"], K, 32)
        out["per_sample_launch_sample_steps_per_s"] = single
        out["batched_speedup_over_per_sample_launches"] = (B * K / el) / single
        # on-device statistics of the batch: Welford mean/variance of (rho, u, v, E) and S2(h),
        # h = 1..32
        st = Stats(s, max_h=32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.accumulate(U)
        res = st.read()
        torch.cuda.synchronize()
        out["stats_ms_for_batch"] = (time.perf_counter() - t0) * 1e3
        out["stats_ms_timing"] = ("host clock around one accumulate and read of the batch; "
                                  "bench.py --workload stats gives device-timed medians")
        out["functionals"] = functionals(s, U, cells, B)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, U0, w["cpu_steps"])
    return out


if __name__ == "__main__":
    main()
