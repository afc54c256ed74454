"""Pins for the CPU oracle: every check compares it with something other than itself.

Sources of truth used here: exact Riemann solutions (Toro, Ch. 4), exact translation of
linear advection, exact solutions of smooth problems via characteristics, convergence
orders of the schemes, invariants (constant states, discrete conservation, mirror and
transposition symmetry, 1D-in-2D/3D reduction) and closed forms of the statistics.
"""
import itertools
import math

import numpy as np
import pytest

import exact_riemann as ER
import fv_inputs as fi
import oracle as O

SOD_L = (1.0, 0.0, 1.0)
SOD_R = (0.125, 0.0, 0.1)


def sod_problem(n, flux="rusanov", recon="first_order", integrator="forward_euler"):
    return O.Problem(dim=1, n=(n,), eq="euler", flux=flux, recon=recon, integrator=integrator,
                     bc=("transmissive",))


def same(a, b):
    """Bitwise equality up to the sign of zero."""
    return np.array_equal(np.asarray(a), np.asarray(b))


# --------------------------------------------------------------------------- exact solver

def test_exact_riemann_sod_star_state_matches_toro_table():
    # Toro (2009) Table 4.3, test 1: p* = 0.30313, u* = 0.92745, rho*L = 0.42632,
    # rho*R = 0.26557.
    ps, us, rl, rr = ER.euler_star(SOD_L, SOD_R)
    assert abs(ps - 0.30313) < 5e-6
    assert abs(us - 0.92745) < 5e-6
    assert abs(rl - 0.42632) < 5e-6
    assert abs(rr - 0.26557) < 5e-6


# --------------------------------------------------------------------------- Sod (1D Euler)

def test_sod_first_order_rusanov_against_exact_solution():
    """The 1D Sod configuration: first order, Rusanov, forward Euler, CFL 0.45, T = 0.2."""
    N = 1024
    U, t, steps, err = O.evolve(sod_problem(N), fi.sod_state(N), 0.2, 0.45)
    assert err[0] == 0 and t[0] == 0.2
    assert 900 < steps[0] < 1100
    x = fi.cell_centres(N)
    r, u, p = ER.euler_sample(SOD_L, SOD_R, (x - 0.5) / 0.2)
    rho = U[0, 0, 0, 0]
    assert np.abs(rho - r).mean() < 1e-2
    vel = U[0, 1, 0, 0] / rho
    assert np.abs(vel - u).mean() < 2e-2
    # far-field states are untouched by the waves
    assert rho[0] == 1.0 and rho[-1] == 0.125


@pytest.mark.parametrize("flux", ["rusanov", "hll", "hllc"])
def test_sod_convergence_order(flux):
    errs = []
    for N in (256, 512, 1024, 2048):
        U, *_ = O.evolve(sod_problem(N, flux), fi.sod_state(N), 0.2, 0.45)
        x = fi.cell_centres(N)
        r, _, _ = ER.euler_sample(SOD_L, SOD_R, (x - 0.5) / 0.2)
        errs.append(np.abs(U[0, 0, 0, 0] - r).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(0.5 <= o <= 1.0 for o in orders), orders


def test_sod_closed_form_totals():
    """While the edge cells keep their initial states, int rho and int E are conserved and
    int m grows by (p_L - p_R) T through the boundary pressure flux."""
    N = 1024
    U0 = fi.sod_state(N)
    U, t, *_ = O.evolve(sod_problem(N), U0, 0.2, 0.45)
    dx = 1.0 / N
    assert abs(math.fsum(U[0, 0].ravel()) * dx - 0.5625) < 1e-13
    assert abs(math.fsum(U[0, 2].ravel()) - math.fsum(U0[0, 2].ravel())) * dx < 1e-13
    gm1 = 1.4 - 1.0
    p_left = gm1 * U0[0, 2, 0, 0, 0]
    p_right = gm1 * U0[0, 2, 0, 0, -1]
    assert abs(math.fsum(U[0, 1].ravel()) * dx - (p_left - p_right) * 0.2) < 1e-13


@pytest.mark.parametrize("flux,recon", list(itertools.product(
    ["rusanov", "hll", "hllc"], ["first_order", "muscl_minmod", "weno3"])))
def test_sod_mirror_symmetry(flux, recon):
    """x -> 1 - x with m -> -m maps solutions onto solutions; Rusanov, HLL and the three
    reconstructions are mirror-exact in the contract's arithmetic, HLLC up to roundoff."""
    N = 200
    integ = "ssprk2" if recon != "first_order" else "forward_euler"
    p = sod_problem(N, flux, recon, integ)
    U0 = fi.sod_state(N)
    M0 = U0[:, :, :, :, ::-1].copy()
    M0[:, 1] = -M0[:, 1]
    U, *_ = O.evolve(p, U0, 0.1, 0.45)
    V, *_ = O.evolve(p, M0, 0.1, 0.45)
    V = V[:, :, :, :, ::-1].copy()
    V[:, 1] = -V[:, 1]
    if flux == "hllc":
        assert np.abs(U - V).max() <= 1e-13 * np.abs(U).max()
    else:
        assert same(U, V)


def test_hllc_keeps_stationary_contact_exactly():
    """An isolated stationary contact (u = 0, equal p, rho jump) is a fixed point of HLLC
    (Toro Sec. 10.4); HLL and Rusanov smear it."""
    N = 64
    U0 = fi.riemann_state_1d(N, (1.0, 0.0, 1.0), (0.5, 0.0, 1.0))
    for flux in ("hllc", "hll", "rusanov"):
        U, t, steps, err = O.evolve(sod_problem(N, flux), U0, 0.1, 0.45)
        if flux == "hllc":
            assert same(U, U0)
        else:
            assert not same(U, U0)


# --------------------------------------------------------------------------- advection

@pytest.mark.parametrize("flux", ["rusanov", "hll"])
@pytest.mark.parametrize("dim,axis", [(1, 0), (2, 0), (2, 1), (3, 2)])
def test_advection_cfl1_is_exact_shift(flux, dim, axis):
    """Upwind first order at Courant number 1 moves dyadic data by exactly one cell per
    step: every operation of the scheme is exact on such data."""
    n = 16
    rng = np.random.default_rng(7)
    shape = (n if dim == 3 else 1, n if dim >= 2 else 1, n)
    U0 = rng.integers(-8, 9, size=(1, 1) + shape).astype(np.float64)
    vel = [0.0, 0.0, 0.0]
    vel[axis] = 1.0
    p = O.Problem(dim=dim, n=(n,) * dim, eq="advection", flux=flux, recon="first_order",
                  integrator="forward_euler", vel=tuple(vel))
    steps = 5
    U, t, k, err = O.evolve(p, U0, steps / n, 1.0)
    assert k[0] == steps
    assert same(U, np.roll(U0, steps, axis=4 - axis))


@pytest.mark.parametrize("recon,integ,lo_order", [
    ("first_order", "forward_euler", 0.85),
    ("muscl_minmod", "ssprk2", 1.5),
    ("weno3", "ssprk3", 1.8),
])
def test_advection_smooth_convergence(recon, integ, lo_order):
    errs = []
    for N in (32, 64, 128, 256):
        p = O.Problem(dim=1, n=(N,), eq="advection", flux="rusanov", recon=recon,
                      integrator=integ, vel=(1.0, 0, 0))
        U0 = fi.sine_state_scalar(N)
        U, *_ = O.evolve(p, U0, 1.0, 0.5)
        errs.append(np.abs(U - U0).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert orders[-1] >= lo_order, orders
    assert errs[-1] < errs[0]


# --------------------------------------------------------------------------- Burgers

def _burgers_characteristics(x, t, u0, du0):
    """u(x, t) = u0(xi) with x = xi + u0(xi) t, solved by Newton before breaking."""
    xi = x.copy()
    for _ in range(60):
        g = xi + u0(xi) * t - x
        xi = xi - g / (1.0 + du0(xi) * t)
    return u0(xi)


@pytest.mark.parametrize("recon,integ,lo_order", [
    ("muscl_minmod", "ssprk2", 1.5), ("weno3", "ssprk3", 1.8)])
@pytest.mark.parametrize("flux", ["rusanov", "hll"])
def test_burgers_smooth_against_characteristics(recon, integ, lo_order, flux):
    u0 = lambda x: 0.5 + 0.25 * np.sin(2 * np.pi * x)
    du0 = lambda x: 0.25 * 2 * np.pi * np.cos(2 * np.pi * x)
    T = 0.3  # breaking time is 1 / (0.5 pi) ~ 0.64
    errs = []
    for N in (64, 128, 256, 512):
        p = O.Problem(dim=1, n=(N,), eq="burgers", flux=flux, recon=recon, integrator=integ)
        U0 = fi.sine_state_scalar(N, amp=0.25, offset=0.5)
        # cell averages of the initial data are not needed at this order: compare point values
        U, *_ = O.evolve(p, U0, T, 0.5)
        exact = _burgers_characteristics(fi.cell_centres(N), T, u0, du0)
        errs.append(np.abs(U[0, 0, 0, 0] - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert orders[-1] >= lo_order, (orders, errs)


@pytest.mark.parametrize("flux", ["rusanov", "hll"])
def test_burgers_riemann_shock_and_rarefaction(flux):
    N = 400
    x = fi.cell_centres(N)
    for uL, uR in ((1.0, 0.0), (-1.0, 1.0)):
        U0 = np.where(x < 0.5, uL, uR)[None, None, None, None, :].astype(np.float64)
        p = O.Problem(dim=1, n=(N,), eq="burgers", flux=flux, recon="first_order",
                      integrator="forward_euler", bc=("transmissive",))
        T = 0.2
        U, t, k, err = O.evolve(p, U0, T, 0.5)
        exact = ER.burgers_sample(uL, uR, (x - 0.5) / T)
        assert np.abs(U[0, 0, 0, 0] - exact).mean() < 0.02
        # total: int u grows by (F(uL) - F(uR)) T through the boundary fluxes
        total = math.fsum(U.ravel()) / N
        expect = math.fsum(U0.ravel()) / N + (0.5 * uL * uL - 0.5 * uR * uR) * T
        assert abs(total - expect) < 1e-13


# --------------------------------------------------------------------------- smooth Euler

def _entropy_wave(dim, N, vel, shift):
    """rho = 1 + 0.2 sin(2 pi (x + y + z - (u + v + w) t)), uniform velocity and pressure."""
    x = fi.cell_centres(N)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    arg = sum(g - v * shift for g, v in zip(grids, vel))
    r = (1.0 + 0.2 * np.sin(2 * np.pi * arg)).transpose()          # -> [z][y][x]
    return r.reshape((1,) * (3 - dim) + r.shape)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("flux", ["rusanov", "hll", "hllc"])
def test_euler_entropy_wave_convergence(dim, flux):
    """A density wave carried by a uniform flow at uniform pressure is an exact solution,
    rho(x - u t); the WENO3 + SSP-RK3 error falls at close to third order once resolved."""
    vel = (1.0, 0.5)[:dim]
    errs = []
    T = 0.25
    for N in (32, 64, 128):
        r0 = _entropy_wave(dim, N, vel, 0.0)
        fields = [r0] + [r0 * v for v in vel] + [1.0 / (1.4 - 1.0) + 0.5 * r0 * sum(v * v for v in vel)]
        U0 = np.stack(fields)[None]
        p = O.Problem(dim=dim, n=(N,) * dim, eq="euler", flux=flux, recon="weno3",
                      integrator="ssprk3")
        U, *_ = O.evolve(p, U0, T, 0.4)
        errs.append(np.abs(U[0, 0] - _entropy_wave(dim, N, vel, T)).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] >= 2.5, (orders, errs)


@pytest.mark.parametrize("flux", ["rusanov", "hll", "hllc"])
def test_cyclic_axis_permutation_3d(flux):
    """(x, y, z) -> (y, z, x) with the momenta permuted alike maps solutions onto
    solutions. The divergence adds the x, y and z terms in that order, and a three-term sum
    is not associative in floating point, so agreement is to roundoff, not bitwise."""
    U0 = fi.random_smooth_state(6, (6, 6, 6), 3)
    def perm(U):  # new x = old y, new y = old z, new z = old x
        return U.transpose(0, 1, 4, 2, 3)[:, [0, 2, 3, 1, 4]].copy()
    p = O.Problem(dim=3, n=(6, 6, 6), eq="euler", flux=flux, recon="weno3", integrator="ssprk3")
    U, *_ = O.evolve(p, U0, 0.03, 0.4)
    V, *_ = O.evolve(p, perm(U0), 0.03, 0.4)
    assert np.abs(perm(U) - V).max() <= 1e-13 * np.abs(V).max()


@pytest.mark.parametrize("flux", ["rusanov", "hllc"])
def test_z_invariant_3d_run_equals_2d(flux):
    U2 = fi.random_smooth_state(8, (1, 12, 16), 2)
    U3 = np.zeros((1, 5, 3, 12, 16))
    U3[:, [0, 1, 2, 4]] = U2
    p2 = O.Problem(dim=2, n=(16, 12), eq="euler", flux=flux, recon="weno3", integrator="ssprk3")
    p3 = O.Problem(dim=3, n=(16, 12, 3), eq="euler", flux=flux, recon="weno3",
                   integrator="ssprk3", hi=(1.0, 1.0, 3.0))
    A, _, k2, _ = O.evolve(p2, U2, 0.05, 0.4)
    B, _, k3, _ = O.evolve(p3, U3, 0.05, 0.4)
    assert k2[0] == k3[0]
    for kz in range(3):
        assert same(B[0, [0, 1, 2, 4], kz], A[0, :, 0])
    assert np.all(B[0, 3] == 0.0)


# --------------------------------------------------------------------------- invariants

EQ_FLUX = [("advection", "rusanov"), ("advection", "hll"), ("burgers", "rusanov"),
           ("burgers", "hll"), ("euler", "rusanov"), ("euler", "hll"), ("euler", "hllc")]


@pytest.mark.parametrize("eq,flux", EQ_FLUX)
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_constant_state_is_preserved_bitwise(eq, flux, dim):
    n = (8, 6, 5)[:dim]
    vals = {"advection": [0.7], "burgers": [-0.3],
            "euler": [1.3] + [0.4, -0.2, 0.1][:dim] + [3.1]}[eq]
    for recon, integ, bc in itertools.product(
            ["first_order", "muscl_minmod", "weno3"], ["forward_euler", "ssprk2", "ssprk3"],
            ["periodic", "transmissive"]):
        p = O.Problem(dim=dim, n=n, eq=eq, flux=flux, recon=recon, integrator=integ,
                      bc=(bc,) * 3, vel=(0.5, -0.25, 1.0))
        U0 = fi.constant_state(tuple(reversed(list(n) + [1] * (3 - dim))), vals)
        U, t, k, err = O.evolve(p, U0, 0.05, 0.5, max_steps=3)
        assert same(U, U0), (recon, integ, bc)


@pytest.mark.parametrize("flux,recon,integ", [
    ("hllc", "weno3", "ssprk3"), ("hll", "muscl_minmod", "ssprk2"),
    ("rusanov", "first_order", "forward_euler")])
def test_periodic_conservation_kh(flux, recon, integ):
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(64, c, phi)
    p = O.Problem(dim=2, n=(64, 64), eq="euler", flux=flux, recon=recon, integrator=integ)
    U, t, k, err = O.evolve(p, U0, 0.02, 0.4)
    assert err[0] == 0 and k[0] > 5
    for q in range(4):
        scale = math.fsum(np.abs(U0[0, q]).ravel())
        drift = abs(math.fsum(U[0, q].ravel()) - math.fsum(U0[0, q].ravel()))
        assert drift <= 1e-13 * scale + 1e-13, (q, drift)
    assert np.all(U[0, 0] > 0)


@pytest.mark.parametrize("flux", ["rusanov", "hll", "hllc"])
def test_transposition_symmetry_2d(flux):
    """Swapping the x and y axes together with m_x and m_y is exact for every flux."""
    U0 = fi.random_smooth_state(3, (1, 24, 24), 2)
    T0 = U0.transpose(0, 1, 2, 4, 3)[:, [0, 2, 1, 3]].copy()
    p = O.Problem(dim=2, n=(24, 24), eq="euler", flux=flux, recon="weno3", integrator="ssprk3")
    U, *_ = O.evolve(p, U0, 0.05, 0.4)
    V, *_ = O.evolve(p, T0, 0.05, 0.4)
    assert same(U, V.transpose(0, 1, 2, 4, 3)[:, [0, 2, 1, 3]])


def test_periodic_roll_invariance():
    U0 = fi.random_smooth_state(4, (1, 16, 20), 2)
    p = O.Problem(dim=2, n=(20, 16), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    U, *_ = O.evolve(p, U0, 0.05, 0.4)
    V, *_ = O.evolve(p, np.roll(U0, (3, -5), axis=(3, 4)), 0.05, 0.4)
    assert same(np.roll(U, (3, -5), axis=(3, 4)), V)


@pytest.mark.parametrize("flux,recon", [("hllc", "weno3"), ("rusanov", "first_order"),
                                        ("hll", "muscl_minmod")])
def test_y_invariant_2d_and_3d_runs_equal_1d(flux, recon):
    N = 128
    integ = "ssprk3"
    p1 = sod_problem(N, flux, recon, integ)
    U1, t1, k1, _ = O.evolve(p1, fi.sod_state(N), 0.1, 0.4)
    S = fi.sod_state(N)
    U2d = np.zeros((1, 4, 1, 4, N))
    U2d[:, [0, 1, 3]] = S  # broadcast over y
    p2 = O.Problem(dim=2, n=(N, 4), eq="euler", flux=flux, recon=recon, integrator=integ,
                   bc=("transmissive", "periodic"))
    U2, t2, k2, _ = O.evolve(p2, U2d, 0.1, 0.4)
    assert k1[0] == k2[0]
    for j in range(4):
        assert same(U2[0, [0, 1, 3], 0, j], U1[0, :, 0, 0])
    assert np.all(U2[0, 2] == 0.0)
    U3d = np.zeros((1, 5, 3, 2, N))
    U3d[:, [0, 1, 4]] = S
    p3 = O.Problem(dim=3, n=(N, 2, 3), eq="euler", flux=flux, recon=recon, integrator=integ,
                   bc=("transmissive", "periodic", "periodic"))
    U3, t3, k3, _ = O.evolve(p3, U3d, 0.1, 0.4)
    assert k3[0] == k1[0]
    assert same(U3[0, [0, 1, 4], 2, 1], U1[0, :, 0, 0])


# --------------------------------------------------------------------------- fluxes, WENO

def _euler_flux_np(U, nd, dim, g=1.4):
    r, m, E = U[0], U[1:1 + dim], U[dim + 1]
    u = m / r
    p = (g - 1) * (E - 0.5 * r * np.sum(u * u))
    F = np.empty(dim + 2)
    F[0] = m[nd]
    F[1:1 + dim] = m * u[nd]
    F[1 + nd] += p
    F[dim + 1] = (E + p) * u[nd]
    return F


@pytest.mark.parametrize("flux", ["rusanov", "hll", "hllc"])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_numerical_flux_is_consistent(flux, dim):
    """F_hat(U, U) = F(U) for every state and direction."""
    rng = np.random.default_rng(11)
    p = O.Problem(dim=dim, n=(4,) * dim, eq="euler", flux=flux)
    for _ in range(50):
        r = rng.uniform(0.1, 3.0)
        u = rng.uniform(-2.0, 2.0, dim)
        pr = rng.uniform(0.1, 3.0)
        U = np.concatenate([[r], r * u, [pr / 0.4 + 0.5 * r * np.sum(u * u)]])
        for nd in range(dim):
            Fh = O.numerical_flux(p, nd, U, U)
            F = _euler_flux_np(U, nd, dim)
            assert np.allclose(Fh, F, rtol=1e-13, atol=1e-13)


def test_weno3_exact_on_linear_data_and_textbook_weights():
    rng = np.random.default_rng(5)
    for _ in range(200):
        b, h = rng.uniform(-3, 3), rng.uniform(-1, 1)
        # linear data: both stencils agree, the face value is b + h/2
        assert abs(O.weno3(b - h, b, b + h) - (b + 0.5 * h)) <= 4e-16 * (abs(b) + abs(h) + 1)
        a, c = rng.uniform(-3, 3, 2)
        eps = 1e-6
        b0, b1 = (b - a) ** 2, (c - b) ** 2
        al0, al1 = (2 / 3) / (eps + b1) ** 2, (1 / 3) / (eps + b0) ** 2
        text = (al0 * 0.5 * (b + c) + al1 * (1.5 * b - 0.5 * a)) / (al0 + al1)
        assert abs(O.weno3(a, b, c) - text) <= 1e-14 * (abs(text) + 1)


# --------------------------------------------------------------------------- errors

def test_validation_and_failure_codes():
    assert O.validate(O.Problem(dim=1, n=(8,), eq="burgers", flux="hllc")) == 2
    assert O.validate(O.Problem(dim=4 - 4, n=(8,))) == 1
    p = sod_problem(32)
    U0 = fi.sod_state(32)
    bad = U0.copy()
    bad[0, 0, 0, 0, 3] = -1.0
    _, _, k, err = O.evolve(p, bad, 0.1, 0.45)
    assert err[0] == 5 and k[0] == 0
    _, t, k, err = O.evolve(p, U0, 0.1, 0.45, max_steps=3)
    assert err[0] == 6 and k[0] == 3 and t[0] < 0.1
    _, err = O.evolve_fixed_dt(p, U0, 1.0, 2, cfl_bound=0.5)
    assert err[0] == 7


# --------------------------------------------------------------------------- statistics

def test_welford_against_two_pass_numpy():
    rng = np.random.default_rng(2)
    p = O.Problem(dim=2, n=(8, 8), eq="euler")
    U = fi.random_smooth_state(9, (1, 8, 8), 2, batch=40)
    U = U * (1.0 + 0.05 * rng.standard_normal(U.shape))
    st = O.Stats(p, max_h=0)
    st.accumulate(U[:17])
    st.accumulate(U[17:])
    q = np.stack([O.quantities(p, U[b]) for b in range(40)])
    assert np.allclose(st.mean, q.mean(axis=0), rtol=1e-14, atol=1e-15)
    assert np.allclose(st.variance(), q.var(axis=0), rtol=1e-11, atol=1e-16)
    assert np.allclose(st.variance(1), q.var(axis=0, ddof=1), rtol=1e-11, atol=1e-16)
    # u = m_x / rho, v = m_y / rho
    assert np.allclose(q[:, 1], U[:, 1] / U[:, 0], rtol=1e-15)


def test_identical_samples_have_zero_variance_exactly():
    p = O.Problem(dim=2, n=(6, 6), eq="euler")
    U = np.repeat(fi.random_smooth_state(1, (1, 6, 6), 2), 9, axis=0)
    st = O.Stats(p, max_h=2)
    st.accumulate(U)
    assert np.all(st.m2 == 0.0) and np.all(st.s2m2 == 0.0)
    assert same(st.mean, O.quantities(p, U[0]))


@pytest.mark.parametrize("k", [1, 3])
def test_structure_function_sine_closed_form(k):
    """q = sin(2 pi k x) on an N-periodic grid: S(h) = 2 sin^2(pi k h / N) in 1D, and half
    of that for the same data constant in y (the y lags add nothing)."""
    N = 64
    q = np.sin(2 * np.pi * k * fi.cell_centres(N))
    p1 = O.Problem(dim=1, n=(N,), eq="advection")
    p2 = O.Problem(dim=2, n=(N, N), eq="advection")
    q2 = np.broadcast_to(q, (N, N)).copy()
    for h in (1, 5, 16, 31):
        exact = 2 * math.sin(math.pi * k * h / N) ** 2
        assert abs(O.structure_function(p1, q, h) - exact) < 1e-14
        assert abs(O.structure_function(p2, q2, h) - exact / 2) < 1e-14


def test_structure_function_against_roll_formula():
    rng = np.random.default_rng(4)
    p = O.Problem(dim=3, n=(6, 5, 4), eq="advection")
    q = rng.standard_normal((4, 5, 6))
    for h in (1, 2, 3):
        ref = sum(np.sum((np.roll(q, -h, axis=ax) - q) ** 2) for ax in (2, 1, 0)) / (3 * q.size)
        assert abs(O.structure_function(p, q, h) - ref) < 1e-13


# --------------------------------------------------------------------------- multilevel MC

def _upsample(a, r):
    """Piecewise-constant prolongation of [..., ny, nx] by r on both axes."""
    return np.repeat(np.repeat(a, r, axis=-1), r, axis=-2)


def test_mlmc_level_statistics_against_numpy():
    rng = np.random.default_rng(8)
    pf = O.Problem(dim=2, n=(16, 16), eq="euler")
    pc = O.Problem(dim=2, n=(8, 8), eq="euler")
    B = 30
    Uf = fi.random_smooth_state(5, (1, 16, 16), 2, batch=B)
    Uc = fi.random_smooth_state(6, (1, 8, 8), 2, batch=B)
    Uf = Uf * (1 + 0.01 * rng.standard_normal(Uf.shape))
    lv = O.LevelStats(pf, pc)
    lv.accumulate(Uf[:11], Uc[:11])
    lv.accumulate(Uf[11:], Uc[11:])
    qf = np.stack([O.quantities(pf, Uf[b]) for b in range(B)])
    qc = np.stack([O.quantities(pc, Uc[b]) for b in range(B)])
    x = qf - _upsample(qc, 2)
    assert np.allclose(lv.mean, x.mean(axis=0), rtol=1e-13, atol=1e-15)
    assert np.allclose(lv.variance(), x.var(axis=0), rtol=1e-10, atol=1e-16)


def test_mlmc_one_level_is_plain_monte_carlo():
    p = O.Problem(dim=2, n=(8, 8), eq="euler")
    U = fi.random_smooth_state(2, (1, 8, 8), 2, batch=12)
    lv = O.LevelStats(p)
    lv.accumulate(U)
    st = O.Stats(p)
    st.accumulate(U)
    assert same(O.mlmc_combine([lv]), st.mean)


def test_mlmc_telescopes_to_finest_mean_with_shared_samples():
    """With the same samples on every level, sum_l (mean q_l - mean P q_{l-1}) telescopes to
    the plain mean of the finest level."""
    B = 10
    ps = [O.Problem(dim=2, n=(n, n), eq="euler") for n in (4, 8, 16)]
    Us = [fi.random_smooth_state(11, (1, n, n), 2, batch=B) for n in (4, 8, 16)]
    levels = [O.LevelStats(ps[0])]
    levels[0].accumulate(Us[0])
    for l in (1, 2):
        lv = O.LevelStats(ps[l], ps[l - 1])
        lv.accumulate(Us[l], Us[l - 1])
        levels.append(lv)
    est = O.mlmc_combine(levels)
    fin = O.Stats(ps[2])
    fin.accumulate(Us[2])
    assert np.allclose(est, fin.mean, rtol=1e-13, atol=1e-14)


def test_mlmc_combine_against_numpy_prolongation():
    ps = [O.Problem(dim=2, n=(n, n), eq="euler") for n in (4, 8, 16)]
    levels = []
    for l, p in enumerate(ps):
        lv = O.LevelStats(p)
        lv.accumulate(fi.random_smooth_state(20 + l, (1, p.n[1], p.n[0]), 2, batch=3))
        levels.append(lv)
    est = O.mlmc_combine(levels)
    ref = _upsample(levels[0].mean, 4) + _upsample(levels[1].mean, 2) + levels[2].mean
    assert same(est, ref)
