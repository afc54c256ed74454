"""Pins of the oracle's entropy-conservative fluxes (Section 2.1 names high-order
entropy-conservative fluxes; the readings -- Chandrashekar's two-point flux for Euler,
Tadmor's for Burgers, LeFloch--Mercier--Rohde's fourth-order combination -- are stated in the
oracle's header). What fixes them independently of the code: Tadmor's condition
(v_R - v_L) . F = psi_R - psi_L with the entropy variables and potential of the Euler entropy
-rho s / (gamma - 1), written out here; the discrete entropy balance sum_i v_i . rhs_i = 0 on
periodic grids; consistency; the logarithmic mean against b expm1(x) / x; and the orders of
accuracy (2 and 4) of the semi-discrete operator on smooth point values, against the exact
flux derivative by complex-step differentiation."""
import math

import numpy as np
import pytest

import fv_inputs as fi
import oracle as O

GAMMA = 1.4


def conserved(rho, u, p, dim):
    u = list(u) + [0.0] * (dim - len(u))
    return np.array([rho] + [rho * v for v in u[:dim]]
                    + [p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in u[:dim])])


def entropy_vars(U, dim):
    """v = dS/dU for S = -rho s / (gamma - 1), s = ln p - gamma ln rho (arrays over cells)."""
    rho, m, E = U[0], U[1:1 + dim], U[dim + 1]
    u = m / rho
    q = (u * u).sum(axis=0)
    p = (GAMMA - 1.0) * (E - 0.5 * rho * q)
    s = np.log(p) - GAMMA * np.log(rho)
    v = np.empty_like(U)
    v[0] = (GAMMA - s) / (GAMMA - 1.0) - rho * q / (2.0 * p)
    v[1:1 + dim] = rho * u / p
    v[dim + 1] = -rho / p
    return v


def ec(dim, nd, UL, UR, eq="euler"):
    p = O.Problem(dim=dim, n=(4,) * dim, eq=eq, flux="ec")
    return O.numerical_flux(p, nd, np.atleast_1d(np.asarray(UL, float)), np.atleast_1d(np.asarray(UR, float)))


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


def test_logarithmic_mean_against_expm1():
    """logmean(b e^x, b) = b (e^x - 1) / x; the ratio is computed independently with expm1."""
    p = O.Problem(dim=1, n=(4,), eq="euler", flux="ec")
    # the density flux of a pair at rest in velocity 1 is the logarithmic mean of the densities
    for b in (0.3, 1.0, 7.0):
        for x in (0.0, 1e-12, -3e-9, 1e-6, 1e-3, 9e-3, 0.02, -0.02, 0.1, 1.0, -2.5, 5.0):
            a = b * math.exp(x)
            want = b * (math.expm1(x) / x) if x != 0.0 else b
            UL = conserved(a, [1.0], 1.0, 1)
            UR = conserved(b, [1.0], 1.0, 1)
            got = O.numerical_flux(p, 0, UL, UR)[0]
            # a = b e^x is itself rounded: the mean of the rounded a differs by up to an ulp
            assert abs(got - want) <= 6e-16 * want, (b, x, got, want)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_tadmor_condition(dim):
    """(v_R - v_L) . F(U_L, U_R) = psi_R - psi_L with psi = rho u_n."""
    rng = np.random.default_rng(70 + dim)
    for _ in range(200):
        UL = conserved(0.2 + 2 * rng.random(), rng.normal(size=dim), 0.2 + 2 * rng.random(), dim)
        UR = conserved(0.2 + 2 * rng.random(), rng.normal(size=dim), 0.2 + 2 * rng.random(), dim)
        vL, vR = entropy_vars(UL[:, None], dim)[:, 0], entropy_vars(UR[:, None], dim)[:, 0]
        for nd in range(dim):
            F = ec(dim, nd, UL, UR)
            lhs = float(np.dot(vR - vL, F))
            rhs = UR[1 + nd] - UL[1 + nd]
            scale = float(np.abs((vR - vL) * F).sum()) + abs(rhs)
            assert abs(lhs - rhs) <= 1e-13 * scale, (dim, nd, lhs, rhs)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_ec_consistency_and_symmetry(dim):
    rng = np.random.default_rng(80 + dim)
    for _ in range(50):
        U = conserved(0.2 + 2 * rng.random(), rng.normal(size=dim), 0.2 + 2 * rng.random(), dim)
        V = conserved(0.2 + 2 * rng.random(), rng.normal(size=dim), 0.2 + 2 * rng.random(), dim)
        for nd in range(dim):
            assert np.allclose(ec(dim, nd, U, U), phys_flux(U, dim, nd), rtol=1e-14, atol=1e-14)
            assert np.allclose(ec(dim, nd, U, V), ec(dim, nd, V, U), rtol=1e-14, atol=1e-15)


def _periodic_smooth_euler(dim, n, seed):
    return fi.random_smooth_state(seed, (n if dim == 3 else 1, n if dim >= 2 else 1, n), dim, batch=1)[0]


@pytest.mark.parametrize("flux", ["ec", "ec4"])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_discrete_entropy_conservation(flux, dim):
    """sum over cells of v_i . rhs_i vanishes to rounding on a periodic grid (Rusanov's is
    strictly negative)."""
    n = {1: 64, 2: 24, 3: 10}[dim]
    U = _periodic_smooth_euler(dim, n, 5 + dim)
    nf = dim + 2
    v = entropy_vars(U.reshape(nf, -1), dim)
    for fl in (flux, "rusanov"):
        p = O.Problem(dim=dim, n=(n,) * dim, eq="euler", flux=fl)
        R = O.rhs(p, U).reshape(nf, -1)
        terms = (v * R).sum(axis=0)
        total, scale = terms.sum(), np.abs(terms).sum()
        if fl == "rusanov":
            assert total < -1e-6 * scale
        else:
            assert abs(total) <= 1e-12 * scale, (fl, total, scale)


@pytest.mark.parametrize("flux", ["ec", "ec4"])
def test_burgers_discrete_entropy_conservation(flux):
    rng = np.random.default_rng(9)
    for dim, n in ((1, 200), (2, 30), (3, 9)):
        shape = (1, 1) + tuple([n if dim == 3 else 1, n if dim >= 2 else 1, n])
        U = rng.normal(size=shape)
        p = O.Problem(dim=dim, n=(n,) * dim, eq="burgers", flux=flux)
        R = O.rhs(p, U)
        terms = U.reshape(R.shape) * R
        assert abs(terms.sum()) <= 1e-13 * np.abs(terms).sum(), (dim, flux)


def _euler_point_values(x):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u = 0.3 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.15 * np.sin(2 * np.pi * x + 1.0)
    E = p / (GAMMA - 1.0) + 0.5 * rho * u * u
    return np.stack([rho, rho * u, E])


def _euler_flux_of_x(x):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u = 0.3 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.15 * np.sin(2 * np.pi * x + 1.0)
    E = p / (GAMMA - 1.0) + 0.5 * rho * u * u
    return np.stack([rho * u, rho * u * u + p, (E + p) * u])


@pytest.mark.parametrize("flux,order", [("ec", 2), ("ec4", 4)])
def test_operator_order_on_smooth_point_values(flux, order):
    """The semi-discrete operator on point values at the cell centres against -dF/dx, from
    complex-step differentiation of the exact flux (exact to rounding)."""
    errs_e, errs_b = [], []
    Ns = (16, 32, 64, 128)
    for N in Ns:
        x = fi.cell_centres(N)
        exact = -np.imag(_euler_flux_of_x(x + 1e-30j)) / 1e-30
        p = O.Problem(dim=1, n=(N,), eq="euler", flux=flux)
        R = O.rhs(p, _euler_point_values(x)[:, None, None, :])[:, 0, 0]
        errs_e.append(np.abs(R - exact).max())
        u = 0.5 + 0.3 * np.sin(2 * np.pi * x)
        pb = O.Problem(dim=1, n=(N,), eq="burgers", flux=flux)
        Rb = O.rhs(pb, u[None, None, None, :])[0, 0, 0]
        errs_b.append(np.abs(Rb + u * 0.3 * 2 * np.pi * np.cos(2 * np.pi * x)).max())
    for errs in (errs_e, errs_b):
        orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(Ns) - 1)]
        assert all(order - 0.25 <= o <= order + 0.5 for o in orders[1:]), (flux, orders)


def test_fourth_order_flux_needs_cell_values():
    assert O.validate(O.Problem(dim=1, n=(8,), eq="euler", flux="ec4", recon="muscl_minmod")) == 2
    assert O.validate(O.Problem(dim=1, n=(8,), eq="advection", flux="ec4")) == 2
    assert O.validate(O.Problem(dim=1, n=(8,), eq="swe", flux="ec")) == 2
    assert O.validate(O.Problem(dim=2, n=(8, 8), eq="euler", flux="ec4")) == 0
