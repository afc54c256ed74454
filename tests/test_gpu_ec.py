"""GPU parity of the entropy-conservative fluxes against the oracle, through the C-ABI:
Chandrashekar's two-point Euler flux with every reconstruction, and the fourth-order
combination for Burgers and Euler, in 1D, 2D and 3D with every stepper, on ragged grids
(several tiles and ragged tails) with periodic and transmissive boundaries; plus the
Kelvin--Helmholtz shear layer with the fourth-order Euler flux.

Burgers is bit for bit (no transcendental functions). The Euler flux takes logarithmic means
through log1p() once the two values differ by more than about 2%, and the device library's
log1p and the C library's need not round alike; the bar is then the relative L1 of 1e-12
(each face flux differs by a few ulp where log1p is taken, and a few steps amplify that by
far less than 100), plus 1e-11 in the max norm, with equal step counts."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note

pytestmark = pytest.mark.gpu

SHAPES = {1: (600,), 2: (150, 20), 3: (20, 12, 9)}
RECONS = ("first_order", "muscl_minmod", "weno3", "eno2")
PAIRS = [("euler", "ec", r) for r in RECONS] + [("euler", "ec4", "first_order"),
                                                 ("burgers", "ec4", "first_order")]
COMBOS = [(d, eq, fl, rc, it) for d in (1, 2, 3) for eq, fl, rc in PAIRS
          for it in ("forward_euler", "ssprk2", "ssprk3")]


def _initial(p, seed):
    nz, ny, nx = p.n[2], p.n[1], p.n[0]
    if p.eq == "euler":
        return fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)
    rng = np.random.default_rng(seed)
    base = fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)[:, :1] - 1.0
    return np.ascontiguousarray(base * 5.0 + 0.1 * rng.standard_normal(base.shape))


def _check(G, R, eq, what):
    if eq == "euler":
        assert_parity(G, R, tol=1e-12, bitwise=False, what=what)
        assert np.abs(G - R).max() <= 1e-11 * np.abs(R).max(), what
    else:
        assert_parity(G, R, what=what)


@pytest.mark.parametrize("dim,eq,flux,recon,integ", COMBOS)
def test_ec_fluxes_match_oracle(dim, eq, flux, recon, integ):
    idx = COMBOS.index((dim, eq, flux, recon, integ))
    bc = ("transmissive",) * 3 if idx % 2 == 0 else ("periodic",) * 3
    p = O.Problem(dim=dim, n=SHAPES[dim], eq=eq, flux=flux, recon=recon, integrator=integ, bc=bc)
    U0 = _initial(p, 91 + dim)
    note("ec", dim, eq, flux, recon, integ, bc[0])
    K = 6
    R, rt, rsteps, rerr = O.evolve(p, U0, 1e3, 0.3, max_steps=K)
    G, gt, gsteps, gerr, st = gpu_evolve(p, U0, 1e3, 0.3, max_steps=K, mode="advance")
    assert np.all(rerr == 6) and np.all(gerr == 0) and st == 0
    assert np.all(gsteps == K)
    if eq == "euler":
        assert np.allclose(gt, rt, rtol=1e-13, atol=0.0)
    else:
        assert np.array_equal(gt, rt)
    _check(G, R, eq, f"{dim}D {eq} {flux} {recon} {integ}")


def test_ec4_kh():
    c, phi = fi.kh_coefficients(1912, [0, 1])
    U0 = fi.kh2d_state(128, c, phi)
    p = O.Problem(dim=2, n=(128, 128), eq="euler", flux="ec4", integrator="ssprk3")
    note("ec4 kh")
    R, rt, rs, re = O.evolve(p, U0, 2.0, 0.3, max_steps=20)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 2.0, 0.3, max_steps=20, mode="advance")
    assert np.all(gs == 20)
    assert np.allclose(gt, rt, rtol=1e-13, atol=0.0)
    _check(G, R, "euler", "ec4 kh")


def test_ec4_needs_cell_values():
    import paper_1912_07645_amd.fv as fv
    from paper_1912_07645_amd import Solver
    for recon in ("muscl_minmod", "weno3", "eno2"):
        with pytest.raises(fv.FVError) as e:
            Solver(dim=2, n=(16, 16), eq="euler", flux="ec4", recon=recon)
        assert e.value.status == fv.FV_ENOTSUP
