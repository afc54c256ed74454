"""Thin ctypes binding of libfv (include/fv.h), with the C names.

Argument marshalling only: every step of the finite-volume path runs in the HIP kernels of
libfv.so. Device arrays are torch tensors on a gfx950 GPU (PyTorch provides device memory
and streams); pointers are passed as integers. If libfv.so is missing, importing this
module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfv.so")

FV_OK, FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE, FV_ENONPHYS, FV_EMAXSTEPS, FV_ECFL = range(8)
STATUS_NAMES = {0: "FV_OK", 1: "FV_EINVAL", 2: "FV_ENOTSUP", 3: "FV_ENOMEM", 4: "FV_EDEVICE",
                5: "FV_ENONPHYS", 6: "FV_EMAXSTEPS", 7: "FV_ECFL"}
BC = {"periodic": 0, "transmissive": 1}
EQ = {"advection": 0, "burgers": 1, "euler": 2, "swe": 3, "mhd": 4}
FLUX = {"rusanov": 0, "hll": 1, "hllc": 2, "roe": 3, "ec": 4, "godunov": 5, "ec4": 6}
RECON = {"first_order": 0, "muscl_minmod": 1, "weno3": 2, "eno2": 3}
INTEGRATOR = {"forward_euler": 0, "ssprk2": 1, "ssprk3": 2}


class fv_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("bc", C.c_int32 * 3), ("n", C.c_int64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class fv_equation(C.Structure):
    _fields_ = [("kind", C.c_int32), ("gamma", C.c_double), ("velocity", C.c_double * 3),
                ("gravity", C.c_double)]


class FVError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libfv.so not found at {LIB_PATH}; build it with "
            "`python -m paper_1912_07645_amd.build` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "fv_create": (i32, [C.POINTER(fv_grid), C.POINTER(fv_equation), i32, i32, i32, C.POINTER(vp)]),
        "fv_destroy": (i32, [vp]),
        "fv_set_stream": (i32, [vp, vp]),
        "fv_num_fields": (i32, [vp]),
        "fv_workspace_size": (i32, [vp, i64, C.POINTER(C.c_size_t)]),
        "fv_set_workspace": (i32, [vp, vp, C.c_size_t]),
        "fv_evolve": (i32, [vp, vp, i64, vp, dbl, dbl, i64, vp, vp]),
        "fv_advance": (i32, [vp, vp, i64, vp, dbl, dbl, i64, vp, vp]),
        "fv_advance_noalloc": (i32, [vp, vp, i64, vp, dbl, dbl, i64, vp, vp]),
        "fv_noalloc_capacity": (C.c_size_t, []),
        "fv_evolve_fixed_dt": (i32, [vp, vp, i64, dbl, i64, dbl, vp]),
        "fv_evolve_multi": (i32, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64), C.POINTER(vp),
                                  dbl, dbl, i64, C.POINTER(vp), C.POINTER(vp)]),
        "fv_num_variants": (i32, [vp]),
        "fv_set_variant": (i32, [vp, i32]),
        "fv_get_tile": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "fv_tune": (i32, [vp, vp, i64, i32, C.POINTER(i32)]),
        "fv_stats_create": (i32, [vp, i32, C.POINTER(vp)]),
        "fv_stats_accumulate": (i32, [vp, vp, i64]),
        "fv_stats_read": (i32, [vp, vp, vp, vp, vp, C.POINTER(i64)]),
        "fv_stats_reset": (i32, [vp]),
        "fv_stats_accumulate_diff": (i32, [vp, vp, vp, vp, i64]),
        "fv_mlmc_combine": (i32, [i32, C.POINTER(vp), vp]),
        "fv_stats_destroy": (i32, [vp]),
        "fv_check_arith": (i32, [vp, vp, vp, vp, i64]),
        "fv_point_pdf": (i32, [vp, vp, i64, i32, i64, C.POINTER(i64), dbl, dbl, i32, vp]),
        "fv_joint_pdf": (i32, [vp, vp, i64, i32, i32, i64, C.POINTER(i64), dbl, dbl, dbl, dbl,
                               i32, vp]),
        "fv_structure_shell": (i32, [vp, vp, i64, i32, i32, i32, vp]),
        "fv_adjoint_create": (i32, [vp, i64, i64, dbl, i64, dbl, C.POINTER(vp)]),
        "fv_adjoint_create_binomial": (i32, [vp, i64, i64, dbl, i64, dbl, C.POINTER(vp)]),
        "fv_adjoint_recomputed_steps": (i32, [vp, C.POINTER(i64)]),
        "fv_adjoint_forward": (i32, [vp, vp, vp]),
        "fv_adjoint_backward": (i32, [vp, vp, vp]),
        "fv_adjoint_destroy": (i32, [vp]),
        "fv_adjoint_set_signature": (i32, [vp, vp]),
        "fv_qoi_kinetic_energy": (i32, [vp, vp, i64, i64, i64, vp, vp, vp]),
        "fv_line_vjp": (i32, [vp, vp, vp, vp, i32, i64, vp]),
        "fv_profile_enable": (i32, [vp, i32]),
        "fv_profile_read": (i32, [vp, C.POINTER(dbl), C.POINTER(i64)]),
        "fv_decomp_create": (i32, [vp, C.POINTER(i32), i64, C.POINTER(vp)]),
        "fv_decomp_scatter": (i32, [vp, vp]),
        "fv_decomp_gather": (i32, [vp, vp]),
        "fv_decomp_advance": (i32, [vp, vp, dbl, dbl, i64, vp, vp, i32]),
        "fv_decomp_profile_enable": (i32, [vp, i32]),
        "fv_decomp_profile_read": (i32, [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(i64)]),
        "fv_decomp_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64),
                                 C.POINTER(i32), C.POINTER(i32)]),
        "fv_decomp_destroy": (i32, [vp]),
        "fv_last_error": (C.c_char_p, []),
        "fv_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def last_error() -> str:
    return lib.fv_last_error().decode()


def check(status: int, where: str) -> int:
    if status != FV_OK:
        raise FVError(status, where, last_error())
    return status


def ptr(t) -> int | None:
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    return t.data_ptr()


def make_grid(dim, n, bc="periodic", lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> fv_grid:
    g = fv_grid()
    g.dim = dim
    n = list(n) + [1] * (3 - len(n))
    bcs = [bc] * 3 if isinstance(bc, str) else list(bc) + ["periodic"] * (3 - len(bc))
    for k in range(3):
        g.n[k] = int(n[k])
        g.bc[k] = BC[bcs[k]] if isinstance(bcs[k], str) else int(bcs[k])
        g.lo[k] = float(lo[k]) if k < len(lo) else 0.0
        g.hi[k] = float(hi[k]) if k < len(hi) else 1.0
    return g


def make_equation(kind="euler", gamma=1.4, velocity=(0.0, 0.0, 0.0), gravity=9.81) -> fv_equation:
    e = fv_equation()
    e.kind = EQ[kind] if isinstance(kind, str) else int(kind)
    e.gamma = float(gamma)
    e.gravity = float(gravity)
    for k in range(3):
        e.velocity[k] = float(velocity[k]) if k < len(velocity) else 0.0
    return e


# ----------------------------------------------------------------- C names


def fv_create(grid: fv_grid, eq: fv_equation, flux: int, recon: int, integrator: int) -> int:
    h = C.c_void_p()
    check(lib.fv_create(C.byref(grid), C.byref(eq), int(flux), int(recon), int(integrator),
                        C.byref(h)), "fv_create")
    return h.value


def fv_destroy(solver: int) -> None:
    check(lib.fv_destroy(solver), "fv_destroy")


def fv_set_stream(solver: int, stream: int | None) -> None:
    check(lib.fv_set_stream(solver, stream), "fv_set_stream")


def fv_num_fields(solver: int) -> int:
    return lib.fv_num_fields(solver)


def fv_workspace_size(solver: int, batch: int) -> int:
    n = C.c_size_t()
    check(lib.fv_workspace_size(solver, int(batch), C.byref(n)), "fv_workspace_size")
    return n.value


def fv_set_workspace(solver: int, dev_ptr: int | None, nbytes: int) -> None:
    check(lib.fv_set_workspace(solver, dev_ptr, int(nbytes)), "fv_set_workspace")


def fv_evolve(solver, state, batch, t, t_end, cfl, max_steps, steps=None, err=None) -> int:
    """Returns the status (FV_OK or the first failing sample's status); raises on argument or
    device errors."""
    st = lib.fv_evolve(solver, ptr(state), int(batch), ptr(t), float(t_end), float(cfl),
                       int(max_steps), ptr(steps), ptr(err))
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_evolve")
    return st


def fv_advance(solver, state, batch, t, t_end, cfl, nsteps, steps=None, err=None) -> int:
    st = lib.fv_advance(solver, ptr(state), int(batch), ptr(t), float(t_end), float(cfl),
                        int(nsteps), ptr(steps), ptr(err))
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_advance")
    return st


def fv_advance_noalloc(solver, state, batch, t, t_end, cfl, nsteps, steps=None, err=None) -> int:
    st = lib.fv_advance_noalloc(solver, ptr(state), int(batch), ptr(t), float(t_end), float(cfl),
                                int(nsteps), ptr(steps), ptr(err))
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_advance_noalloc")
    return st


def fv_noalloc_capacity() -> int:
    return lib.fv_noalloc_capacity()


def fv_evolve_fixed_dt(solver, state, batch, dt, nsteps, cfl_bound, err=None) -> int:
    st = lib.fv_evolve_fixed_dt(solver, ptr(state), int(batch), float(dt), int(nsteps),
                                float(cfl_bound), ptr(err))
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_evolve_fixed_dt")
    return st


def fv_evolve_multi(solvers, states, batches, ts, t_end, cfl, max_steps, steps=None,
                    errs=None) -> int:
    n = len(solvers)
    A = C.c_void_p * n
    errs = errs if errs is not None else [None] * n
    steps = steps if steps is not None else [None] * n
    st = lib.fv_evolve_multi(n, A(*solvers), A(*[ptr(s) for s in states]),
                             (C.c_int64 * n)(*[int(b) for b in batches]), A(*[ptr(t) for t in ts]),
                             float(t_end), float(cfl), int(max_steps),
                             A(*[ptr(k) for k in steps]), A(*[ptr(e) for e in errs]))
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_evolve_multi")
    return st


def fv_num_variants(solver) -> int:
    return lib.fv_num_variants(solver)


def fv_set_variant(solver, variant: int) -> None:
    check(lib.fv_set_variant(solver, int(variant)), "fv_set_variant")


def fv_get_tile(solver):
    bx, by, bz, v = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    check(lib.fv_get_tile(solver, C.byref(bx), C.byref(by), C.byref(bz), C.byref(v)), "fv_get_tile")
    return (bx.value, by.value, bz.value), v.value


def fv_tune(solver, state, batch, reps=3) -> int:
    ch = C.c_int32()
    check(lib.fv_tune(solver, ptr(state), int(batch), int(reps), C.byref(ch)), "fv_tune")
    return ch.value


def fv_stats_create(solver, max_h: int) -> int:
    h = C.c_void_p()
    check(lib.fv_stats_create(solver, int(max_h), C.byref(h)), "fv_stats_create")
    return h.value


def fv_stats_accumulate(stats, state, batch) -> None:
    check(lib.fv_stats_accumulate(stats, ptr(state), int(batch)), "fv_stats_accumulate")


def fv_stats_read(stats, mean=None, var=None, s2_mean=None, s2_var=None) -> int:
    n = C.c_int64()
    check(lib.fv_stats_read(stats, ptr(mean), ptr(var), ptr(s2_mean), ptr(s2_var), C.byref(n)),
          "fv_stats_read")
    return n.value


def fv_stats_accumulate_diff(stats, fine, coarse_solver, coarse_state, batch) -> None:
    check(lib.fv_stats_accumulate_diff(stats, ptr(fine), coarse_solver, ptr(coarse_state), int(batch)),
          "fv_stats_accumulate_diff")


def fv_mlmc_combine(levels, out) -> None:
    n = len(levels)
    check(lib.fv_mlmc_combine(n, (C.c_void_p * n)(*levels), ptr(out)), "fv_mlmc_combine")


def fv_stats_reset(stats) -> None:
    check(lib.fv_stats_reset(stats), "fv_stats_reset")


def fv_stats_destroy(stats) -> None:
    check(lib.fv_stats_destroy(stats), "fv_stats_destroy")


def _host_i64(cells):
    arr = (C.c_int64 * len(cells))(*[int(c) for c in cells])
    return arr


def fv_point_pdf(solver, state, batch, quantity, points, lo, hi, nbins, counts) -> None:
    pts = [int(p) for p in points]
    check(lib.fv_point_pdf(solver, ptr(state), int(batch), int(quantity), len(pts), _host_i64(pts),
                           float(lo), float(hi), int(nbins), ptr(counts)), "fv_point_pdf")


def fv_joint_pdf(solver, state, batch, quantity_a, quantity_b, pairs, lo_a, hi_a, lo_b, hi_b,
                 nbins, counts) -> None:
    flat = [int(c) for pr in pairs for c in pr]
    check(lib.fv_joint_pdf(solver, ptr(state), int(batch), int(quantity_a), int(quantity_b),
                           len(flat) // 2, _host_i64(flat), float(lo_a), float(hi_a), float(lo_b),
                           float(hi_b), int(nbins), ptr(counts)), "fv_joint_pdf")


def fv_structure_shell(solver, state, batch, max_h, order, ball, out) -> None:
    check(lib.fv_structure_shell(solver, ptr(state), int(batch), int(max_h), int(order),
                                 int(bool(ball)), ptr(out)), "fv_structure_shell")


def fv_check_arith(a, b, quot, root) -> None:
    check(lib.fv_check_arith(ptr(a), ptr(b), ptr(quot), ptr(root), a.numel()), "fv_check_arith")


def fv_adjoint_create(solver, batch, nsteps, dt, every=0, cfl_bound=1.0) -> int:
    h = C.c_void_p()
    check(lib.fv_adjoint_create(solver, int(batch), int(nsteps), float(dt), int(every),
                                float(cfl_bound), C.byref(h)), "fv_adjoint_create")
    return h.value


def fv_adjoint_create_binomial(solver, batch, nsteps, dt, snapshots, cfl_bound=1.0) -> int:
    h = C.c_void_p()
    check(lib.fv_adjoint_create_binomial(solver, int(batch), int(nsteps), float(dt), int(snapshots),
                                         float(cfl_bound), C.byref(h)), "fv_adjoint_create_binomial")
    return h.value


def fv_adjoint_recomputed_steps(adj) -> int:
    n = C.c_int64()
    check(lib.fv_adjoint_recomputed_steps(adj, C.byref(n)), "fv_adjoint_recomputed_steps")
    return n.value


def fv_adjoint_forward(adj, state0, stateT) -> None:
    check(lib.fv_adjoint_forward(adj, ptr(state0), ptr(stateT)), "fv_adjoint_forward")


def fv_adjoint_backward(adj, dQ_dUT, dQ_dU0) -> None:
    check(lib.fv_adjoint_backward(adj, ptr(dQ_dUT), ptr(dQ_dU0)), "fv_adjoint_backward")


def fv_adjoint_set_signature(adj, sig) -> None:
    check(lib.fv_adjoint_set_signature(adj, ptr(sig)), "fv_adjoint_set_signature")


def fv_adjoint_destroy(adj) -> None:
    check(lib.fv_adjoint_destroy(adj), "fv_adjoint_destroy")


def fv_qoi_kinetic_energy(solver, state, batch, j0, j1, seed=None, Q=None, dQ_dU=None) -> None:
    check(lib.fv_qoi_kinetic_energy(solver, ptr(state), int(batch), int(j0), int(j1), ptr(seed),
                                    ptr(Q), ptr(dQ_dU)), "fv_qoi_kinetic_energy")


def fv_line_vjp(solver, lambda0, dU_dline, dline_dtheta, ntheta, batch, out) -> None:
    check(lib.fv_line_vjp(solver, ptr(lambda0), ptr(dU_dline), ptr(dline_dtheta), int(ntheta),
                          int(batch), ptr(out)), "fv_line_vjp")


def fv_profile_enable(solver, on: bool) -> None:
    check(lib.fv_profile_enable(solver, 1 if on else 0), "fv_profile_enable")


def fv_profile_read(solver):
    ms = C.c_double()
    n = C.c_int64()
    check(lib.fv_profile_read(solver, C.byref(ms), C.byref(n)), "fv_profile_read")
    return ms.value, n.value


def fv_decomp_create(solver, parts, batch) -> int:
    h = C.c_void_p()
    p = (C.c_int32 * 3)(*[int(x) for x in (list(parts) + [1, 1, 1])[:3]])
    check(lib.fv_decomp_create(solver, p, int(batch), C.byref(h)), "fv_decomp_create")
    return h.value


def fv_decomp_scatter(d, state) -> None:
    check(lib.fv_decomp_scatter(d, ptr(state)), "fv_decomp_scatter")


def fv_decomp_gather(d, state) -> None:
    check(lib.fv_decomp_gather(d, ptr(state)), "fv_decomp_gather")


FV_DECOMP_OVERLAP, FV_DECOMP_DMA = 1, 2


def fv_decomp_advance(d, t, t_end, cfl, nsteps, steps=None, err=None, overlap=True,
                      dma=False) -> int:
    mode = (FV_DECOMP_OVERLAP if overlap else 0) | (FV_DECOMP_DMA if dma else 0)
    st = lib.fv_decomp_advance(d, ptr(t), float(t_end), float(cfl), int(nsteps), ptr(steps),
                               ptr(err), mode)
    if st in (FV_EINVAL, FV_ENOTSUP, FV_ENOMEM, FV_EDEVICE):
        check(st, "fv_decomp_advance")
    return st


def fv_decomp_profile_enable(d, on: bool) -> None:
    check(lib.fv_decomp_profile_enable(d, 1 if on else 0), "fv_decomp_profile_enable")


def fv_decomp_profile_read(d):
    a, b, n = C.c_double(), C.c_double(), C.c_int64()
    check(lib.fv_decomp_profile_read(d, C.byref(a), C.byref(b), C.byref(n)), "fv_decomp_profile_read")
    return a.value, b.value, n.value


def fv_decomp_info(d):
    ns, nm, ni, nsh = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    hb = C.c_int64()
    check(lib.fv_decomp_info(d, C.byref(ns), C.byref(nm), C.byref(hb), C.byref(ni), C.byref(nsh)),
          "fv_decomp_info")
    return dict(subdomains=ns.value, messages=nm.value, halo_bytes_per_stage=hb.value,
                interior_tiles=ni.value, shell_tiles=nsh.value)


def fv_decomp_destroy(d) -> None:
    check(lib.fv_decomp_destroy(d), "fv_decomp_destroy")


def fv_version() -> str:
    return lib.fv_version().decode()
