"""Python access to the plain FP64 CPU oracle (``fv_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark use this package to check and time the GPU library. The GPU library never imports
it, and it never imports the GPU library.

``build()`` compiles ``fv_oracle.c`` with gcc (``-O2 -ffp-contract=off``, no fast-math, with
OpenMP) into ``oracle/_build/liboracle.so``; ``lib()`` loads it, building it first if it is
missing or older than the source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fv_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "liboracle.so")

EQ = {"advection": 0, "burgers": 1, "euler": 2, "swe": 3, "mhd": 4}
FLUX = {"rusanov": 0, "hll": 1, "hllc": 2, "roe": 3, "ec": 4, "godunov": 5, "ec4": 6}
RECON = {"first_order": 0, "muscl_minmod": 1, "weno3": 2, "eno2": 3}
INTEGRATOR = {"forward_euler": 0, "ssprk2": 1, "ssprk3": 2}
BC = {"periodic": 0, "transmissive": 1}
STATUS = {0: "ok", 1: "einval", 2: "enotsup", 3: "enomem", 5: "enonphys", 6: "emaxsteps",
          7: "ecfl"}


class OcProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("eq", C.c_int32), ("flux", C.c_int32), ("recon", C.c_int32),
        ("integrator", C.c_int32), ("bc", C.c_int32 * 3), ("n", C.c_int64 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("gamma", C.c_double),
        ("vel", C.c_double * 3), ("grav", C.c_double),
    ]


def build(force: bool = False) -> str:
    os.makedirs(_BUILD, exist_ok=True)
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER(OcProblem)
        dp = C.POINTER(C.c_double)
        L.oc_num_fields.argtypes = [P]
        L.oc_validate.argtypes = [P]
        L.oc_rhs.argtypes = [P, dp, dp]
        L.oc_step.argtypes = [P, dp, C.c_double]
        L.oc_evolve.argtypes = [P, dp, C.c_int64, dp, C.c_double, C.c_double, C.c_int64,
                                C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.oc_evolve_fixed_dt.argtypes = [P, dp, C.c_int64, C.c_double, C.c_int64, C.c_double,
                                         C.POINTER(C.c_int32)]
        L.oc_max_speed.argtypes = [P, dp, dp, C.POINTER(C.c_int)]
        L.oc_numerical_flux.argtypes = [P, C.c_int, dp, dp, dp]
        L.oc_weno3.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oc_weno3.restype = C.c_double
        L.oc_quantities.argtypes = [P, dp, dp]
        L.oc_structure_function.argtypes = [P, dp, C.c_int64]
        L.oc_structure_function.restype = C.c_double
        L.oc_stats_accumulate.argtypes = [P, dp, C.c_int64, C.c_int32, dp, dp, dp, dp,
                                          C.POINTER(C.c_int64)]
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_stats_accumulate_diff.argtypes = [P, P, dp, dp, C.c_int64, dp, dp,
                                               C.POINTER(C.c_int64)]
        L.oc_mlmc_combine.argtypes = [C.c_int32, P, C.POINTER(dp), dp]
        L.oc_reconstruct.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        ip = C.POINTER(C.c_int64)
        L.oc_point_pdf.argtypes = [P, dp, C.c_int64, C.c_int32, C.c_int64, ip, C.c_double,
                                   C.c_double, C.c_int32, ip]
        L.oc_joint_pdf.argtypes = [P, dp, C.c_int64, C.c_int32, C.c_int32, C.c_int64, ip,
                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, ip]
        L.oc_structure_shell.argtypes = [P, dp, C.c_int64, C.c_int32, C.c_int32]
        L.oc_structure_shell.restype = C.c_double
        L.oc_structure_shell_batch.argtypes = [P, dp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, dp]
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (n <= 0 leaves it); returns the count in use."""
    return lib().oc_set_threads(int(n))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Problem:
    """Grid, equation and scheme of one finite-volume problem (names as in the C oracle)."""
    dim: int
    n: tuple
    eq: str = "euler"
    flux: str = "rusanov"
    recon: str = "first_order"
    integrator: str = "forward_euler"
    bc: tuple = ("periodic", "periodic", "periodic")
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    gamma: float = 1.4
    vel: tuple = (0.0, 0.0, 0.0)
    gravity: float = 9.81
    _c: OcProblem = field(default=None, init=False, repr=False)

    def __post_init__(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        self.n = tuple(int(v) for v in n)
        bc = list(self.bc) if not isinstance(self.bc, str) else [self.bc] * 3
        bc = bc + ["periodic"] * (3 - len(bc))
        self.bc = tuple(bc)
        c = OcProblem()
        c.dim, c.eq = self.dim, EQ[self.eq]
        c.flux, c.recon, c.integrator = FLUX[self.flux], RECON[self.recon], INTEGRATOR[self.integrator]
        for k in range(3):
            c.bc[k] = BC[self.bc[k]]
            c.n[k] = self.n[k]
            c.lo[k] = float(self.lo[k]) if k < len(self.lo) else 0.0
            c.hi[k] = float(self.hi[k]) if k < len(self.hi) else 1.0
            c.vel[k] = float(self.vel[k]) if k < len(self.vel) else 0.0
        c.gamma = float(self.gamma)
        c.grav = float(self.gravity)
        self._c = c

    @property
    def c(self):
        return C.byref(self._c)

    @property
    def nfields(self) -> int:
        return {"euler": self.dim + 2, "swe": self.dim + 1, "mhd": 8}.get(self.eq, 1)

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def state_shape(self):
        return (self.nfields, self.n[2], self.n[1], self.n[0])


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(rc, what)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


def validate(p: Problem) -> int:
    return lib().oc_validate(p.c)


def rhs(p: Problem, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(p.state_shape)
    R = np.empty_like(U)
    _check(lib().oc_rhs(p.c, _dp(U), _dp(R)), "oc_rhs")
    return R


def step(p: Problem, U: np.ndarray, dt: float) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(p.state_shape).copy()
    _check(lib().oc_step(p.c, _dp(U), float(dt)), "oc_step")
    return U


def max_speed(p: Problem, U: np.ndarray):
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(p.state_shape)
    M = C.c_double()
    bad = C.c_int()
    lib().oc_max_speed(p.c, _dp(U), C.byref(M), C.byref(bad))
    return M.value, bool(bad.value)


def evolve(p: Problem, U: np.ndarray, t_end: float, cfl: float, t0=0.0, max_steps: int = 10**9):
    """Evolve a batch U[batch][fields][nz][ny][nx] to t_end. Returns (U, t, steps, err)."""
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    B = U.shape[0]
    assert U.shape[1:] == p.state_shape, (U.shape, p.state_shape)
    t = np.full(B, t0, dtype=np.float64) if np.isscalar(t0) else np.array(t0, dtype=np.float64)
    steps = np.zeros(B, dtype=np.int64)
    err = np.zeros(B, dtype=np.int32)
    rc = lib().oc_evolve(p.c, _dp(U), B, _dp(t), float(t_end), float(cfl), int(max_steps),
                         steps.ctypes.data_as(C.POINTER(C.c_int64)),
                         err.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc in (1, 2, 3):
        _check(rc, "oc_evolve")
    return U, t, steps, err


def evolve_fixed_dt(p: Problem, U: np.ndarray, dt: float, nsteps: int, cfl_bound: float = 1.0):
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    B = U.shape[0]
    err = np.zeros(B, dtype=np.int32)
    rc = lib().oc_evolve_fixed_dt(p.c, _dp(U), B, float(dt), int(nsteps), float(cfl_bound),
                                  err.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc in (1, 2, 3):
        _check(rc, "oc_evolve_fixed_dt")
    return U, err


def numerical_flux(p: Problem, nd: int, UL, UR) -> np.ndarray:
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.empty(p.nfields, dtype=np.float64)
    lib().oc_numerical_flux(p.c, int(nd), _dp(UL), _dp(UR), _dp(F))
    return F


def weno3(a: float, b: float, c: float) -> float:
    return lib().oc_weno3(float(a), float(b), float(c))


def reconstruct(recon: str, um: float, u0: float, up: float):
    """Face values (at i - 1/2, at i + 1/2) of the cell u0 between um and up."""
    lo, hi = C.c_double(), C.c_double()
    lib().oc_reconstruct(RECON[recon], float(um), float(u0), float(up), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def quantities(p: Problem, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(p.state_shape)
    q = np.empty_like(U)
    lib().oc_quantities(p.c, _dp(U), _dp(q))
    return q


def structure_function(p: Problem, q: np.ndarray, h: int) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.size == p.cells
    return lib().oc_structure_function(p.c, _dp(q), int(h))


def _ip(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def point_pdf(p: Problem, U: np.ndarray, quantity: int, points, lo: float, hi: float,
              nbins: int) -> np.ndarray:
    """Histogram over the samples U[batch] of `quantity` at each cell of `points`:
    int64 [npoints][nbins + 2] (bins, below lo, not below hi)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    counts = np.zeros((pts.size, nbins + 2), dtype=np.int64)
    _check(lib().oc_point_pdf(p.c, _dp(U), U.shape[0], int(quantity), pts.size, _ip(pts),
                              float(lo), float(hi), int(nbins), _ip(counts)), "oc_point_pdf")
    return counts


def joint_pdf(p: Problem, U: np.ndarray, quantity_a: int, quantity_b: int, pairs, lo_a: float,
              hi_a: float, lo_b: float, hi_b: float, nbins: int) -> np.ndarray:
    """Histogram over samples of (q_a(x), q_b(y)) for each pair (x, y) of cells:
    int64 [npairs][nbins * nbins + 1] (bin ka * nbins + kb, then outside)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    counts = np.zeros((pr.shape[0], nbins * nbins + 1), dtype=np.int64)
    _check(lib().oc_joint_pdf(p.c, _dp(U), U.shape[0], int(quantity_a), int(quantity_b),
                              pr.shape[0], _ip(pr), float(lo_a), float(hi_a), float(lo_b),
                              float(hi_b), int(nbins), _ip(counts)), "oc_joint_pdf")
    return counts


def structure_shell(p: Problem, q: np.ndarray, h: int, order: int = 2, ball: bool = False) -> float:
    """S_order(h) of one periodic field q over the cube (or ball) shell of radius h."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.size == p.cells
    return lib().oc_structure_shell(p.c, _dp(q), int(h), int(order), int(bool(ball)))


def structure_shell_batch(p: Problem, U: np.ndarray, max_h: int, order: int = 2,
                          ball: bool = False) -> np.ndarray:
    """Shell structure functions of every quantity of every sample: [batch][quantities][max_h]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros((U.shape[0], p.nfields, max_h), dtype=np.float64)
    _check(lib().oc_structure_shell_batch(p.c, _dp(U), U.shape[0], int(max_h), int(order),
                                          int(bool(ball)), _dp(out)), "oc_structure_shell_batch")
    return out


class LevelStats:
    """Per-cell moments over coupled samples of q(u_fine) - P q(u_coarse) (one MLMC level);
    with coarse=None, plain moments of q(u_fine) (the first level, u^0 = 0)."""

    def __init__(self, fine: Problem, coarse: "Problem | None" = None):
        self.fine, self.coarse = fine, coarse
        self.mean = np.zeros((fine.nfields,) + fine.state_shape[1:], dtype=np.float64)
        self.m2 = np.zeros_like(self.mean)
        self.count = C.c_int64(0)
        self._plain = Stats(fine, 0) if coarse is None else None

    def accumulate(self, Uf: np.ndarray, Uc: np.ndarray | None = None):
        if self._plain is not None:
            self._plain.accumulate(Uf)
            self.mean, self.m2, self.count = self._plain.mean, self._plain.m2, self._plain.count
            return
        Uf = np.ascontiguousarray(Uf, dtype=np.float64)
        Uc = np.ascontiguousarray(Uc, dtype=np.float64)
        assert Uf.shape[0] == Uc.shape[0]
        rc = lib().oc_stats_accumulate_diff(self.fine.c, self.coarse.c, _dp(Uf), _dp(Uc),
                                            Uf.shape[0], _dp(self.mean), _dp(self.m2),
                                            C.byref(self.count))
        _check(rc, "oc_stats_accumulate_diff")

    @property
    def n(self) -> int:
        return self.count.value

    def variance(self, ddof: int = 0):
        return self.m2 / (self.n - ddof)


def mlmc_combine(levels) -> np.ndarray:
    """sum_l P_{l -> L} mean_l on the finest (last) level's grid."""
    L = len(levels)
    arr = (OcProblem * L)(*[lv.fine._c for lv in levels])
    means = [np.ascontiguousarray(lv.mean) for lv in levels]
    ptrs = (C.POINTER(C.c_double) * L)(*[_dp(m) for m in means])
    out = np.empty_like(means[-1])
    _check(lib().oc_mlmc_combine(L, arr, ptrs, _dp(out)), "oc_mlmc_combine")
    return out


class Stats:
    """Running Monte Carlo statistics over samples added in index order."""

    def __init__(self, p: Problem, max_h: int = 0):
        self.p = p
        self.max_h = int(max_h)
        nq = p.nfields
        self.mean = np.zeros((nq,) + p.state_shape[1:], dtype=np.float64)
        self.m2 = np.zeros_like(self.mean)
        self.s2mean = np.zeros((nq, max(self.max_h, 1)), dtype=np.float64)
        self.s2m2 = np.zeros_like(self.s2mean)
        self.count = C.c_int64(0)

    def accumulate(self, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        rc = lib().oc_stats_accumulate(self.p.c, _dp(U), U.shape[0], self.max_h,
                                       _dp(self.mean), _dp(self.m2), _dp(self.s2mean),
                                       _dp(self.s2m2), C.byref(self.count))
        _check(rc, "oc_stats_accumulate")

    @property
    def n(self) -> int:
        return self.count.value

    def variance(self, ddof: int = 0):
        return self.m2 / (self.n - ddof)

    def s2(self):
        return self.s2mean[:, :self.max_h]

    def s2_variance(self, ddof: int = 0):
        return self.s2m2[:, :self.max_h] / (self.n - ddof)
