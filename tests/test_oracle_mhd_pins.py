"""Pins of the oracle's ideal-MHD equations (Rusanov and HLL fluxes on the fast magnetosonic
speed; the reading is stated in the oracle's header). What fixes them independently of the
code: the physical flux written out here, the closed forms of the fast speed for a field along
and across the normal, the reduction to the Euler equations at B = 0, the exact preservation of
a uniform normal field in 1D, the circularly polarised Alfven wave (an exact nonlinear
solution) with the scheme converging to it, and the mirror and rotation symmetries of the
equations."""
import math

import numpy as np
import pytest

import fv_inputs as fi
import oracle as O

G53 = 5.0 / 3.0


def phys_flux(U, nd, gamma):
    rho, m, E, B = U[0], U[1:4], U[4], U[5:8]
    u = m / rho
    pb = 0.5 * float(B @ B)
    p = (gamma - 1.0) * (E - 0.5 * rho * float(u @ u) - pb)
    F = np.zeros(8)
    F[0] = m[nd]
    F[1:4] = m * u[nd] - B[nd] * B
    F[1 + nd] += p + pb
    F[4] = (E + p + pb) * u[nd] - B[nd] * float(u @ B)
    F[5:8] = u[nd] * B - B[nd] * u
    return F


def random_state(rng, gamma):
    rho, p = 0.5 + rng.random(), 0.5 + rng.random()
    return fi.mhd_conserved(rho, rng.normal(size=3), p, rng.normal(size=3), gamma)


@pytest.mark.parametrize("flux", ["rusanov", "hll"])
def test_consistency(flux):
    rng = np.random.default_rng(11)
    for dim in (1, 2, 3):
        p = O.Problem(dim=dim, n=(4,) * dim, eq="mhd", flux=flux, gamma=G53)
        for _ in range(30):
            U = random_state(rng, G53)
            for nd in range(dim):
                F = O.numerical_flux(p, nd, U, U)
                assert np.allclose(F, phys_flux(U, nd, G53), rtol=1e-14, atol=1e-14)
                assert F[5 + nd] == 0.0


def test_fast_speed_closed_forms():
    rng = np.random.default_rng(12)
    p1 = O.Problem(dim=1, n=(1,), eq="mhd", gamma=G53)
    for _ in range(40):
        rho, pr, b = 0.3 + rng.random(), 0.3 + rng.random(), 2.0 * rng.random()
        a = math.sqrt(G53 * pr / rho)
        # field along the normal: c_f = max(a, |B_n| / sqrt(rho)); across it: sqrt(a^2 + B^2/rho)
        for B, want in (([b, 0.0, 0.0], max(a, b / math.sqrt(rho))),
                        ([0.0, b, 0.0], math.sqrt(a * a + b * b / rho)),
                        ([0.0, 0.6 * b, 0.8 * b], math.sqrt(a * a + b * b / rho))):
            U = fi.mhd_conserved(rho, [0.0, 0.0, 0.0], pr, B, G53).reshape(8, 1, 1, 1)
            M, bad = O.max_speed(p1, U)          # (|u| + c_f) / dx with dx = 1
            assert not bad and M == pytest.approx(want, rel=2e-15), (B, M, want)


@pytest.mark.parametrize("flux", ["rusanov", "hll"])
@pytest.mark.parametrize("recon", ["first_order", "weno3"])
def test_reduces_to_euler_without_field(flux, recon):
    """B = 0 and u_z = 0: the MHD right-hand side of (rho, m_x, m_y, E) is the Euler one, and
    m_z and B stay zero."""
    n = 24
    E2 = fi.random_smooth_state(4, (1, n, n), 2, batch=1)[0]         # rho, m_x, m_y, E
    U = np.zeros((8, 1, n, n))
    U[0], U[1], U[2], U[4] = E2[0], E2[1], E2[2], E2[3]
    pm = O.Problem(dim=2, n=(n, n), eq="mhd", flux=flux, recon=recon)
    pe = O.Problem(dim=2, n=(n, n), eq="euler", flux=flux, recon=recon)
    Rm = O.rhs(pm, U)
    Re = O.rhs(pe, E2)
    for qm, qe in ((0, 0), (1, 1), (2, 2), (4, 3)):
        assert np.allclose(Rm[qm], Re[qe], rtol=1e-12, atol=1e-12 * np.abs(Re[qe]).max())
    assert not Rm[3].any() and not Rm[5:].any()


def test_uniform_normal_field_is_kept_exactly_in_1d():
    N = 200
    p = O.Problem(dim=1, n=(N,), eq="mhd", flux="hll", recon="muscl_minmod", integrator="ssprk2",
                  bc=("transmissive",), gamma=2.0)
    U, t, k, err = O.evolve(p, fi.brio_wu_state(N), 0.1, 0.5)
    assert err[0] == 0 and k[0] > 50
    assert np.all(U[0, 5] == 0.75)
    assert U[0, 0].min() > 0.0


@pytest.mark.parametrize("flux", ["rusanov", "hll"])
def test_alfven_wave_convergence(flux):
    errs = []
    for N in (32, 64, 128):
        p = O.Problem(dim=1, n=(N,), eq="mhd", flux=flux, recon="weno3", integrator="ssprk3",
                      gamma=G53)
        U, t, k, err = O.evolve(p, fi.alfven_wave_average(N, 0.0), 0.2, 0.4)
        assert err[0] == 0
        exact = fi.alfven_wave_average(N, 0.2)
        errs.append(np.abs(U - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-4 and all(o >= 1.8 for o in orders), (errs, orders)


def test_mirror_symmetry():
    """x -> -x with B -> -B (both symmetries of ideal MHD): m_x and B_x change sign."""
    N = 200
    p = O.Problem(dim=1, n=(N,), eq="mhd", flux="hll", recon="muscl_minmod", integrator="ssprk2",
                  bc=("transmissive",), gamma=2.0)
    U0 = fi.brio_wu_state(N)
    S = np.array([1, -1, 1, 1, 1, -1, 1, 1], dtype=float)[None, :, None, None, None]
    M0 = (U0[..., ::-1] * S).copy()
    U, *_ = O.evolve(p, U0, 0.1, 0.5)
    V, *_ = O.evolve(p, M0, 0.1, 0.5)
    V = (V[..., ::-1] * S).copy()
    assert np.abs(U - V).max() <= 1e-13 * np.abs(U).max()


def test_rotation_symmetry_2d():
    """A quarter turn of the periodic square, (x, y) -> (y, 1 - x), with u and B rotated the
    same way, (v_x, v_y) -> (v_y, -v_x)."""
    n = 32
    U0 = fi.random_smooth_mhd(21, (1, n, n), 2, batch=1)[0]
    p = O.Problem(dim=2, n=(n, n), eq="mhd", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk2", gamma=G53)

    def turn(U):
        V = np.rot90(U, k=1, axes=(2, 3)).copy()      # V[y][x] = U[x][n-1-y]: the turned grid
        V[[1, 2]] = np.stack([V[2], -V[1]])
        V[[5, 6]] = np.stack([V[6], -V[5]])
        return V

    U, *_ = O.evolve_fixed_dt(p, U0[None], 2e-3, 10)
    V, *_ = O.evolve_fixed_dt(p, turn(U0)[None], 2e-3, 10)
    assert np.abs(turn(U[0]) - V[0]).max() <= 1e-13 * np.abs(U).max()


def test_fluxes_offered():
    for flux in ("hllc", "roe", "godunov", "ec", "ec4"):
        assert O.validate(O.Problem(dim=1, n=(8,), eq="mhd", flux=flux)) == 2
    assert O.validate(O.Problem(dim=3, n=(4, 4, 4), eq="mhd", flux="hll")) == 0
