"""Pins of the oracle's Godunov flux (Section 2.1 names it among the numerical fluxes; the
reading, the flux of the exact Riemann solution at x/t = 0, is stated in the oracle's header).
What fixes it independently of the code: an exact Riemann solver written separately on the
test side (bracketing root finder instead of Newton's method, its own wave sampling), the
Burgers entropy solution, upwinding for advection, consistency, the exact preservation of a
stationary contact and of a stationary shock, mirror symmetry, and convergence to the exact
Sod solution."""
import math

import numpy as np
import pytest

import exact_riemann as ER
import fv_inputs as fi
import oracle as O

GAMMA = 1.4


def conserved(rho, u, p, dim=1):
    u = list(u) + [0.0] * (dim - len(u))
    return np.array([rho] + [rho * v for v in u[:dim]]
                    + [p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in u[:dim])])


def phys_flux(rho, u, p, nd):
    """Euler flux along axis nd of the state (rho, velocity vector u, p)."""
    dim = len(u)
    E = p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in u)
    F = np.zeros(dim + 2)
    F[0] = rho * u[nd]
    for k in range(dim):
        F[1 + k] = rho * u[k] * u[nd] + (p if k == nd else 0.0)
    F[dim + 1] = (E + p) * u[nd]
    return F


def godunov(dim, nd, UL, UR, eq="euler", vel=(0.0, 0.0, 0.0)):
    p = O.Problem(dim=dim, n=(4,) * dim, eq=eq, flux="godunov", vel=vel)
    return O.numerical_flux(p, nd, np.atleast_1d(np.asarray(UL, float)),
                            np.atleast_1d(np.asarray(UR, float)))


# (rho, u, p) pairs: Sod, Lax, the 123 problem (two strong rarefactions), a strong blast, two
# colliding shocks, supersonic flow either way, transonic rarefactions either way, a stationary
# contact, plus random pairs below
RIEMANN_CASES = [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
    ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571)),
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),
    ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)),
    ((5.99924, 19.5975, 460.894), (5.99242, -6.19633, 46.0950)),
    ((1.0, 3.0, 1.0), (0.5, 2.5, 0.8)),
    ((0.5, -3.0, 0.8), (1.0, -2.6, 1.0)),
    ((1.0, 0.75, 1.0), (0.125, 0.0, 0.1)),
    ((0.125, 0.0, 0.1), (1.0, -0.75, 1.0)),
    ((1.0, 0.0, 1.0), (0.2, 0.0, 1.0)),
]


def _random_cases(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = (0.1 + 2 * rng.random(), rng.normal(), 0.1 + 2 * rng.random())
        R = (0.1 + 2 * rng.random(), rng.normal(), 0.1 + 2 * rng.random())
        cL, cR = math.sqrt(GAMMA * L[2] / L[0]), math.sqrt(GAMMA * R[2] / R[0])
        if 2.0 / (GAMMA - 1.0) * (cL + cR) <= 1.2 * (R[1] - L[1]):
            continue                        # keep clear of vacuum generation
        out.append((L, R))
    return out


@pytest.mark.parametrize("case", RIEMANN_CASES + _random_cases(60, 5))
def test_euler_flux_is_the_exact_solution_at_the_interface(case):
    L, R = case
    r, u, p = (float(v[0]) for v in ER.euler_sample(L, R, np.array([0.0])))
    want = phys_flux(r, [u], p, 0)
    got = godunov(1, 0, conserved(*L[:1], [L[1]], L[2]), conserved(*R[:1], [R[1]], R[2]))
    scale = max(np.abs(want).max(), 1e-300)
    assert np.abs(got - want).max() <= 1e-11 * scale, (L, R, got, want)


@pytest.mark.parametrize("dim", [2, 3])
def test_euler_multid_tangential_velocity_from_the_contact_side(dim):
    rng = np.random.default_rng(40 + dim)
    for (L, R) in RIEMANN_CASES + _random_cases(20, 6 + dim):
        for nd in range(dim):
            tL, tR = rng.normal(size=dim), rng.normal(size=dim)
            uL, uR = tL.copy(), tR.copy()
            uL[nd], uR[nd] = L[1], R[1]
            r, un, p = (float(v[0]) for v in ER.euler_sample(L, R, np.array([0.0])))
            _, us, _, _ = ER.euler_star(L, R)
            u = (uL if us >= 0.0 else uR).copy()
            u[nd] = un
            want = phys_flux(r, list(u), p, nd)
            got = godunov(dim, nd, conserved(L[0], uL, L[2], dim), conserved(R[0], uR, R[2], dim))
            assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), (dim, nd, L, R)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_consistency(dim):
    rng = np.random.default_rng(dim)
    for _ in range(30):
        rho, u, p = 0.3 + rng.random(), rng.normal(size=dim) * 2.0, 0.3 + rng.random()
        U = conserved(rho, u, p, dim)
        for nd in range(dim):
            assert np.allclose(godunov(dim, nd, U, U), phys_flux(rho, list(u), p, nd),
                               rtol=1e-14, atol=1e-14)


def test_stationary_contact_and_stationary_shock_are_kept_exactly():
    """Godunov's flux of a pair joined by a wave at rest is the flux of either state, so the
    scheme keeps such a profile unchanged."""
    N = 64
    # contact at rest: equal pressure and zero velocity, density jump
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="godunov", bc=("transmissive",))
    U0 = np.zeros((1,) + p.state_shape)
    U0[0, 0, 0, 0] = np.where(np.arange(N) < N // 2, 1.0, 0.25)
    U0[0, 2, 0, 0] = 1.0 / (GAMMA - 1.0)
    U, *_ = O.evolve_fixed_dt(p, U0, 1e-3, 50)
    assert np.abs(U - U0).max() <= 1e-13
    # shock at rest: Rankine--Hugoniot states for Mach 3 in the shock frame
    M, rL, pL = 3.0, 1.0, 1.0
    cL = math.sqrt(GAMMA * pL / rL)
    uL = M * cL
    rR = rL * (GAMMA + 1) * M * M / ((GAMMA - 1) * M * M + 2)
    pR = pL * (2 * GAMMA * M * M - (GAMMA - 1)) / (GAMMA + 1)
    uR = rL * uL / rR
    FL = phys_flux(rL, [uL], pL, 0)
    FR = phys_flux(rR, [uR], pR, 0)
    assert np.allclose(FL, FR, rtol=1e-14)
    UL, UR = conserved(rL, [uL], pL), conserved(rR, [uR], pR)
    assert np.allclose(godunov(1, 0, UL, UR), FL, rtol=1e-13)
    U0 = np.stack([np.where(np.arange(N) < N // 2, UL[q], UR[q]) for q in range(3)])[None, :, None, None, :]
    U, *_ = O.evolve_fixed_dt(p, U0.copy(), 1e-3, 50)
    assert np.abs(U - U0).max() <= 1e-12 * np.abs(U0).max()


def test_mirror_symmetry():
    N = 200
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="godunov", recon="muscl_minmod",
                  integrator="ssprk2", bc=("transmissive",))
    U0 = fi.sod_state(N)
    M0 = U0[:, :, :, :, ::-1].copy()
    M0[:, 1] = -M0[:, 1]
    U, *_ = O.evolve(p, U0, 0.1, 0.45)
    V, *_ = O.evolve(p, M0, 0.1, 0.45)
    V = V[:, :, :, :, ::-1].copy()
    V[:, 1] = -V[:, 1]
    assert np.abs(U - V).max() <= 1e-13 * np.abs(U).max()


def test_sod_against_exact_solution_and_order():
    errs = []
    for N in (256, 512, 1024, 2048):
        p = O.Problem(dim=1, n=(N,), eq="euler", flux="godunov", bc=("transmissive",))
        U, t, k, err = O.evolve(p, fi.sod_state(N), 0.2, 0.45)
        assert err[0] == 0
        x = fi.cell_centres(N)
        r, _, _ = ER.euler_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 0.5) / 0.2)
        errs.append(np.abs(U[0, 0, 0, 0] - r).mean())
    assert errs[2] < 1e-2
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(0.5 <= o <= 1.0 for o in orders), orders


def test_burgers_flux_is_the_entropy_solution_at_the_interface():
    rng = np.random.default_rng(3)
    pairs = [(1.0, -1.0), (-1.0, 1.0), (2.0, 1.0), (-1.0, -2.0), (1.0, -3.0), (3.0, -1.0),
             (-0.5, 0.5), (0.0, 0.0), (0.0, 1.0), (-1.0, 0.0)] + [tuple(rng.normal(size=2)) for _ in range(200)]
    for uL, uR in pairs:
        u0 = float(ER.burgers_sample(uL, uR, np.array([0.0]))[0])
        # at a shock standing exactly at x = 0 either side carries the same flux
        assert godunov(1, 0, [uL], [uR], eq="burgers")[0] == pytest.approx(0.5 * u0 * u0, rel=1e-15, abs=0.0), (uL, uR)
    assert godunov(1, 0, [-0.5], [0.5], eq="burgers")[0] == 0.0          # transonic rarefaction: f(0) = 0


def test_advection_is_upwinding():
    for a in (0.7, -0.4):
        F = godunov(2, 0, [2.0], [5.0], eq="advection", vel=(a, 0.3, 0.0))
        assert F[0] == (a * 2.0 if a > 0 else a * 5.0)
        F = godunov(2, 1, [2.0], [5.0], eq="advection", vel=(a, 0.3, 0.0))
        assert F[0] == 0.3 * 2.0


def test_shallow_water_godunov_is_not_offered():
    p = O.Problem(dim=1, n=(8,), eq="swe", flux="godunov")
    assert O.validate(p) != 0
