"""Pins of the oracle's shallow-water equations (h, hu[, hv]; flux hu u + g h^2 / 2): the
exact wet-bed dam break (whose middle state satisfies both Rankine--Hugoniot conditions),
the lake at rest kept bit for bit, conservation of mass and momentum on periodic grids,
consistency, Roe's flux equal to the upwind flux for one-signed pairs and across a
hydraulic jump, mirror and x-y symmetry, and a 2D run constant in y equal to the 1D run."""
import itertools
import math

import numpy as np
import pytest

import exact_riemann as ER
import fv_inputs as fi
import oracle as O

G = 9.81


def swe(dim, n, flux="rusanov", recon="first_order", integ="forward_euler", bc="transmissive"):
    return O.Problem(dim=dim, n=n, eq="swe", flux=flux, recon=recon, integrator=integ,
                     bc=(bc,) * 3, gravity=G)


def phys_flux(U, dim, nd):
    h = U[0]
    u = U[1:1 + dim] / h
    F = np.zeros(dim + 1)
    F[0] = U[1 + nd]
    F[1:] = U[1:1 + dim] * u[nd]
    F[1 + nd] += 0.5 * G * h * h
    return F


def test_exact_dam_break_satisfies_rankine_hugoniot():
    for hL, hR in ((2.0, 1.0), (1.0, 0.1), (5.0, 4.9)):
        _, _, hm, um, S = ER.swe_dam_break(hL, hR, [0.0], G)
        assert abs(hm * um - S * (hm - hR)) < 1e-12
        assert abs((hm * um * um + 0.5 * G * hm * hm) - 0.5 * G * hR * hR - S * hm * um) < 1e-10 * hL * hL
        # the rarefaction's Riemann invariant u + 2c is constant
        assert abs(um + 2 * math.sqrt(G * hm) - 2 * math.sqrt(G * hL)) < 1e-12


@pytest.mark.parametrize("flux", ["rusanov", "hll", "roe"])
def test_dam_break_against_exact_solution(flux):
    errs = []
    T = 0.05
    for N in (256, 512, 1024, 2048):
        U, t, k, err = O.evolve(swe(1, (N,), flux), fi.swe_dam_break_1d(N), T, 0.45)
        assert err[0] == 0 and t[0] == T
        x = fi.cell_centres(N)
        h, u, *_ = ER.swe_dam_break(2.0, 1.0, (x - 0.5) / T, G)
        errs.append(np.abs(U[0, 0, 0, 0] - h).mean())
    assert errs[2] < 5e-3, errs
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(0.5 <= o <= 1.05 for o in orders), orders


@pytest.mark.parametrize("dim,flux,recon", list(itertools.product(
    [1, 2], ["rusanov", "hll", "roe"], ["first_order", "muscl_minmod", "weno3", "eno2"])))
def test_lake_at_rest_is_exact(dim, flux, recon):
    n = (12,) * dim
    p = swe(dim, n, flux, recon, "ssprk3", "periodic")
    U0 = np.zeros((1, dim + 1) + p.state_shape[1:])
    U0[:, 0] = 1.7
    U, *_ = O.evolve(p, U0, 0.1, 0.4)
    assert np.array_equal(U, U0)


@pytest.mark.parametrize("flux", ["rusanov", "hll", "roe"])
def test_periodic_conservation(flux):
    p = swe(2, (24, 20), flux, "weno3", "ssprk3", "periodic")
    U0 = fi.random_smooth_swe(3, (1, 20, 24), 2)
    U, t, k, err = O.evolve(p, U0, 0.05, 0.4)
    assert err[0] == 0 and k[0] > 5
    for f in range(3):
        assert abs(math.fsum(U[0, f].ravel()) - math.fsum(U0[0, f].ravel())) < 1e-12 * U0[0, 0].size


@pytest.mark.parametrize("dim", [1, 2])
def test_consistency_and_roe_upwinding(dim):
    rng = np.random.default_rng(dim)
    for flux in ("rusanov", "hll", "roe"):
        p = swe(dim, (4,) * dim, flux)
        for _ in range(10):
            U = np.concatenate([[0.5 + rng.random()], rng.normal(size=dim)])
            for nd in range(dim):
                assert np.allclose(O.numerical_flux(p, nd, U, U), phys_flux(U, dim, nd), rtol=1e-15, atol=1e-15)
    # one-signed pairs (supercritical flow): Roe's flux is the upwind physical flux
    p = swe(dim, (4,) * dim, "roe")
    for sign in (1.0, -1.0):
        for _ in range(20):
            nd = int(rng.integers(dim))
            hL, hR = 1.0 + 0.1 * rng.random(), 1.0 + 0.1 * rng.random()
            uL = rng.normal(scale=0.3, size=dim)
            uR = uL + rng.normal(scale=0.05, size=dim)
            uL[nd] += 8.0 * sign
            uR[nd] += 8.0 * sign
            UL = np.concatenate([[hL], hL * uL])
            UR = np.concatenate([[hR], hR * uR])
            want = phys_flux(UL if sign > 0 else UR, dim, nd)
            assert np.allclose(O.numerical_flux(p, nd, UL, UR), want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("hR_over_hL", [0.9, 0.5, 0.2])
def test_roe_hydraulic_jump_is_upwind(hR_over_hL):
    """A bore moving right into still water: the Rankine--Hugoniot pair from the exact dam
    break's shock; Roe's speed of the right-going field equals the bore speed."""
    hL0 = 1.0
    _, _, hm, um, S = ER.swe_dam_break(hL0, hR_over_hL * hL0, [0.0], G)
    hR = hR_over_hL * hL0
    UL, UR = np.array([hm, hm * um]), np.array([hR, 0.0])
    assert np.allclose(phys_flux(UR, 1, 0) - phys_flux(UL, 1, 0), S * (UR - UL), rtol=1e-10, atol=1e-12)
    p = swe(1, (4,), "roe")
    assert np.allclose(O.numerical_flux(p, 0, UL, UR), phys_flux(UL, 1, 0), rtol=1e-10)


@pytest.mark.parametrize("flux,recon", [("rusanov", "first_order"), ("hll", "muscl_minmod"),
                                        ("roe", "weno3"), ("roe", "eno2")])
def test_mirror_symmetry(flux, recon):
    N = 200
    integ = "forward_euler" if recon == "first_order" else "ssprk2"
    p = swe(1, (N,), flux, recon, integ)
    U0 = fi.swe_dam_break_1d(N, 2.0, 1.0, x0=0.37)
    M0 = U0[:, :, :, :, ::-1].copy()
    M0[:, 1] = -M0[:, 1]
    U, *_ = O.evolve(p, U0, 0.03, 0.45)
    V, *_ = O.evolve(p, M0, 0.03, 0.45)
    V = V[:, :, :, :, ::-1].copy()
    V[:, 1] = -V[:, 1]
    assert np.abs(U - V).max() <= 1e-13 * np.abs(U).max()


@pytest.mark.parametrize("flux", ["rusanov", "hll", "roe"])
def test_2d_constant_in_y_equals_1d(flux):
    N = 64
    p1 = swe(1, (N,), flux, "weno3", "ssprk3")
    p2 = swe(2, (N, 6), flux, "weno3", "ssprk3")
    U1 = fi.swe_dam_break_1d(N, 2.0, 1.0, x0=0.41)
    U2 = np.zeros((1, 3, 1, 6, N))
    U2[:, :2] = U1[:, :, :, :, :]
    R1, t1, *_ = O.evolve(p1, U1, 0.02, 0.4)
    R2, t2, *_ = O.evolve(p2, U2, 0.02, 0.4)
    # the y speed adds |v| + c on the y axis; with v = 0 and dy = 1/6 > dx the step is the same
    assert t1[0] == t2[0]
    for j in range(6):
        assert np.array_equal(R2[0, :2, 0, j], R1[0, :, 0, 0])
    assert (R2[0, 2] == 0.0).all()


def test_xy_symmetry():
    n = 24
    p = swe(2, (n, n), "hll", "muscl_minmod", "ssprk2", "periodic")
    U0 = fi.swe_circular_dam_break(n, 2.0, 1.0, 0.2)
    U, *_ = O.evolve(p, U0, 0.05, 0.4)
    h = U[0, 0, 0]
    assert np.abs(h - h.T).max() <= 1e-13 * h.max()
    assert np.abs(U[0, 1, 0] - U[0, 2, 0].T).max() <= 1e-13 * np.abs(U[0, 1]).max()


def test_validation():
    with pytest.raises(O.OracleError):
        O.evolve(swe(3, (4, 4, 4)), np.ones((1, 4, 4, 4, 4)), 0.1, 0.4)
    for flux in ("hllc", "ec"):
        with pytest.raises(O.OracleError):
            O.evolve(swe(1, (8,), flux), np.ones((1, 2, 1, 1, 8)), 0.1, 0.4)
    bad = O.Problem(dim=1, n=(8,), eq="swe", gravity=0.0)
    with pytest.raises(O.OracleError):
        O.evolve(bad, np.ones((1, 2, 1, 1, 8)), 0.1, 0.4)
    # negative depth is non-physical
    U = np.ones((1, 2, 1, 1, 8))
    U[0, 0, 0, 0, 3] = -1.0
    _, _, _, err = O.evolve(swe(1, (8,)), U, 0.1, 0.4)
    assert err[0] == 5


def test_quantities_are_depth_and_velocity():
    p = swe(2, (3, 2))
    U = fi.random_smooth_swe(1, (1, 2, 3), 2)
    q = O.quantities(p, U[0])
    assert np.array_equal(q[0], U[0, 0])
    assert np.array_equal(q[1], U[0, 1] * (1.0 / U[0, 0]))
    assert np.array_equal(q[2], U[0, 2] * (1.0 / U[0, 0]))
