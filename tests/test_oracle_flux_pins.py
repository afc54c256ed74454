"""Pins of the oracle's Roe flux (Euler and scalar, with Harten's entropy fix), Tadmor's
entropy-conservative Burgers flux and the second-order ENO reconstruction (Section 2.1 names
them; the readings are stated in the oracle's header). What fixes them independently of the
code: Roe's matrix carries any jump whose waves all move one way onto the upwind flux
(supersonic pairs, a Rankine--Hugoniot shock), a stationary contact stays put, a Burgers
transonic rarefaction gets the Godunov flux f(0) = 0, the EC flux satisfies Tadmor's identity
and conserves the discrete entropy, ENO2 is exact on linear data and picks the smoother side;
plus convergence to exact solutions (Sod, characteristics, entropy wave)."""
import math

import numpy as np
import pytest

import exact_riemann as ER
import fv_inputs as fi
import oracle as O

GAMMA = 1.4


def conserved(rho, u, p, dim=1):
    """Conserved state (rho, m_1..m_dim, E) from density, velocity vector and pressure."""
    u = list(u) + [0.0] * (dim - len(u))
    return np.array([rho] + [rho * v for v in u[:dim]] + [p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in u[:dim])])


def phys_flux(U, dim, nd):
    rho, m, E = U[0], U[1:1 + dim], U[dim + 1]
    u = m / rho
    p = (GAMMA - 1.0) * (E - 0.5 * float(np.dot(m, u)))
    F = np.zeros(dim + 2)
    F[0] = m[nd]
    F[1:1 + dim] = m * u[nd]
    F[1 + nd] += p
    F[dim + 1] = (E + p) * u[nd]
    return F


def roe(dim, nd, UL, UR):
    p = O.Problem(dim=dim, n=(4,) * dim, eq="euler", flux="roe")
    return O.numerical_flux(p, nd, UL, UR)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_roe_consistency(dim):
    rng = np.random.default_rng(dim)
    for _ in range(20):
        U = conserved(0.5 + rng.random(), rng.normal(size=dim), 0.5 + rng.random(), dim)
        for nd in range(dim):
            F = roe(dim, nd, U, U)
            assert np.allclose(F, phys_flux(U, dim, nd), rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_roe_supersonic_pairs_are_upwind(dim):
    """All Roe speeds of one sign: (1/2) sum |l| alpha K = (1/2) A~ dU = (1/2)(F_R - F_L), so
    the flux is F_L (or F_R): Roe averages, wave strengths and eigenvectors all enter."""
    rng = np.random.default_rng(10 + dim)
    for sign in (1.0, -1.0):
        for _ in range(20):
            nd = int(rng.integers(dim))
            uL = rng.normal(scale=0.3, size=dim)
            uR = uL + rng.normal(scale=0.05, size=dim)
            uL[nd] += 4.0 * sign
            uR[nd] += 4.0 * sign
            UL = conserved(1.0 + 0.1 * rng.random(), uL, 1.0 + 0.1 * rng.random(), dim)
            UR = conserved(1.0 + 0.1 * rng.random(), uR, 1.0 + 0.1 * rng.random(), dim)
            want = phys_flux(UL if sign > 0 else UR, dim, nd)
            assert np.allclose(roe(dim, nd, UL, UR), want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("Ms", [1.2, 2.0, 5.0])
def test_roe_single_shock_is_upwind(Ms):
    """A right-moving shock into still gas (normal-shock relations): Roe's average speed of
    the 3-wave is the shock speed, so the flux equals the post-shock physical flux."""
    rR, pR = 1.0, 1.0
    cR = math.sqrt(GAMMA * pR / rR)
    s = Ms * cR
    rL = rR * (GAMMA + 1) * Ms * Ms / ((GAMMA - 1) * Ms * Ms + 2)
    pL = pR * (2 * GAMMA * Ms * Ms - (GAMMA - 1)) / (GAMMA + 1)
    uL = s * (1.0 - rR / rL)
    UL, UR = conserved(rL, [uL], pL), conserved(rR, [0.0], pR)
    # Rankine--Hugoniot holds for the constructed pair
    assert np.allclose(phys_flux(UR, 1, 0) - phys_flux(UL, 1, 0), s * (UR - UL), rtol=1e-13)
    assert np.allclose(roe(1, 0, UL, UR), phys_flux(UL, 1, 0), rtol=1e-12)


def test_roe_keeps_stationary_contact_exactly():
    N = 64
    U0 = fi.riemann_state_1d(N, (1.0, 0.0, 1.0), (0.5, 0.0, 1.0))
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="roe", bc=("transmissive",))
    U, *_ = O.evolve(p, U0, 0.1, 0.45)
    assert np.array_equal(U, U0)


def test_roe_sod_against_exact_solution_and_order():
    errs = []
    for N in (256, 512, 1024, 2048):
        p = O.Problem(dim=1, n=(N,), eq="euler", flux="roe", bc=("transmissive",))
        U, t, k, err = O.evolve(p, fi.sod_state(N), 0.2, 0.45)
        assert err[0] == 0
        x = fi.cell_centres(N)
        r, _, _ = ER.euler_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 0.5) / 0.2)
        errs.append(np.abs(U[0, 0, 0, 0] - r).mean())
    assert errs[2] < 1e-2
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(0.5 <= o <= 1.0 for o in orders), orders


def test_roe_mirror_symmetry():
    N = 200
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="roe", recon="muscl_minmod", integrator="ssprk2",
                  bc=("transmissive",))
    U0 = fi.sod_state(N)
    M0 = U0[:, :, :, :, ::-1].copy()
    M0[:, 1] = -M0[:, 1]
    U, *_ = O.evolve(p, U0, 0.1, 0.45)
    V, *_ = O.evolve(p, M0, 0.1, 0.45)
    V = V[:, :, :, :, ::-1].copy()
    V[:, 1] = -V[:, 1]
    assert np.abs(U - V).max() <= 1e-13 * np.abs(U).max()


def test_roe_burgers_and_advection():
    pb = O.Problem(dim=1, n=(4,), eq="burgers", flux="roe")
    # transonic rarefaction: Harten's fix over the fan gives the Godunov flux f(0) = 0
    for uL, uR in ((-1.0, 1.0), (-0.3, 0.7), (-2.0, 0.5)):
        assert abs(O.numerical_flux(pb, 0, [uL], [uR])[0]) <= 1e-15
    # shocks and one-signed pairs: the upwind flux
    for uL, uR in ((1.0, 0.0), (2.0, -1.0), (0.5, 0.7), (-0.5, -0.7), (0.0, -1.0)):
        a = 0.5 * (uL + uR)
        want = 0.5 * (uL * uL if a > 0 else uR * uR)
        assert O.numerical_flux(pb, 0, [uL], [uR])[0] == pytest.approx(want, rel=1e-15, abs=1e-16)
    pa = O.Problem(dim=2, n=(4, 4), eq="advection", flux="roe", vel=(0.7, -1.3, 0.0))
    assert O.numerical_flux(pa, 0, [2.0], [5.0])[0] == pytest.approx(0.7 * 2.0, rel=1e-15)
    assert O.numerical_flux(pa, 1, [2.0], [5.0])[0] == pytest.approx(-1.3 * 5.0, rel=1e-15)


def test_roe_advection_cfl1_is_exact_shift():
    n = 16
    U0 = np.random.default_rng(4).integers(-8, 9, size=(1, 1, 1, 1, n)).astype(np.float64)
    p = O.Problem(dim=1, n=(n,), eq="advection", flux="roe", vel=(1.0, 0, 0))
    U, t, k, err = O.evolve(p, U0, 5 / n, 1.0)
    assert k[0] == 5 and np.array_equal(U, np.roll(U0, 5, axis=4))


def test_burgers_riemann_roe_and_ec_totals():
    N = 400
    x = fi.cell_centres(N)
    for uL, uR in ((1.0, 0.0), (-1.0, 1.0)):
        U0 = np.where(x < 0.5, uL, uR)[None, None, None, None, :].astype(np.float64)
        p = O.Problem(dim=1, n=(N,), eq="burgers", flux="roe", bc=("transmissive",))
        U, *_ = O.evolve(p, U0, 0.2, 0.5)
        exact = ER.burgers_sample(uL, uR, (x - 0.5) / 0.2)
        assert np.abs(U[0, 0, 0, 0] - exact).mean() < 0.02


def test_ec_flux_identity_and_entropy_conservation():
    pe = O.Problem(dim=1, n=(4,), eq="burgers", flux="ec")
    rng = np.random.default_rng(2)
    for _ in range(50):
        uL, uR = rng.normal(size=2)
        F = O.numerical_flux(pe, 0, [uL], [uR])[0]
        # Tadmor's identity for the entropy u^2/2, entropy variable u, potential u^3/6
        assert (uR - uL) * F == pytest.approx((uR ** 3 - uL ** 3) / 6.0, rel=1e-13, abs=1e-15)
    for u in (0.0, 1.0, -3.5, 1e-3):
        assert O.numerical_flux(pe, 0, [u], [u])[0] == pytest.approx(0.5 * u * u, rel=2e-16)
    # semi-discrete entropy balance on a periodic grid: sum_i u_i rhs_i = 0 for the EC flux
    # (first order), < 0 for Rusanov
    N = 64
    u = rng.normal(size=(1, 1, 1, N))
    pec = O.Problem(dim=1, n=(N,), eq="burgers", flux="ec")
    prs = O.Problem(dim=1, n=(N,), eq="burgers", flux="rusanov")
    e_ec = float(np.sum(u * O.rhs(pec, u)))
    e_rs = float(np.sum(u * O.rhs(prs, u)))
    scale = float(np.sum(np.abs(u) * np.abs(O.rhs(pec, u))))
    assert abs(e_ec) <= 1e-13 * scale
    assert e_rs < -1e-3 * scale
    with pytest.raises(O.OracleError):                   # EC fluxes: Burgers and Euler only
        O.evolve(O.Problem(dim=1, n=(8,), eq="advection", flux="ec"), np.ones((1, 1, 1, 1, 8)), 0.1, 0.4)


def test_eno2_hand_values():
    assert O.reconstruct("eno2", 1.0, 2.0, 3.0) == (1.5, 2.5)        # linear: exact (tie: left)
    assert O.reconstruct("eno2", 0.0, 1.0, 3.0) == (0.5, 1.5)        # smaller slope on the left
    assert O.reconstruct("eno2", 0.0, 1.0, 0.5) == (1.25, 0.75)      # minmod would clip to 0
    assert O.reconstruct("muscl_minmod", 0.0, 1.0, 0.5) == (1.0, 1.0)
    assert O.reconstruct("eno2", 0.0, 1.0, 0.0) == (0.5, 1.5)        # opposite signs, tie: left
    assert O.reconstruct("eno2", 5.0, 1.0, 0.0) == (1.5, 0.5)        # smaller slope on the right
    rng = np.random.default_rng(9)
    for _ in range(50):
        a, b = rng.normal(size=2)
        lo, hi = O.reconstruct("eno2", a - b, a, a + b)              # any linear triple
        assert lo == pytest.approx(a - 0.5 * b, abs=1e-15) and hi == pytest.approx(a + 0.5 * b, abs=1e-15)


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_eno2_smooth_convergence(flux):
    errs = []
    for N in (32, 64, 128, 256):
        p = O.Problem(dim=1, n=(N,), eq="advection", flux=flux, recon="eno2",
                      integrator="ssprk2", vel=(1.0, 0, 0))
        U0 = fi.sine_state_scalar(N)
        U, *_ = O.evolve(p, U0, 1.0, 0.5)
        errs.append(np.abs(U - U0).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert orders[-1] >= 1.8, orders


@pytest.mark.parametrize("dim", [1, 2])
def test_roe_weno3_entropy_wave_convergence(dim):
    vel = (1.0, 0.5)[:dim]
    errs = []
    T = 0.25
    for N in (32, 64, 128):
        x = fi.cell_centres(N)
        grids = np.meshgrid(*([x] * dim), indexing="ij")
        def wave(shift):
            arg = sum(g - v * shift for g, v in zip(grids, vel))
            r = (1.0 + 0.2 * np.sin(2 * np.pi * arg)).transpose()
            return r.reshape((1,) * (3 - dim) + r.shape)
        r0 = wave(0.0)
        U0 = np.stack([r0] + [r0 * v for v in vel] + [1.0 / (GAMMA - 1.0) + 0.5 * r0 * sum(v * v for v in vel)])[None]
        p = O.Problem(dim=dim, n=(N,) * dim, eq="euler", flux="roe", recon="weno3", integrator="ssprk3")
        U, *_ = O.evolve(p, U0, T, 0.4)
        errs.append(np.abs(U[0, 0] - wave(T)).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] >= 2.5, (orders, errs)
