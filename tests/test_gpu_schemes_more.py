"""GPU parity of the Roe flux, Tadmor's entropy-conservative Burgers flux and the
second-order ENO reconstruction against the oracle, bit for bit, in 1D, 2D and 3D with every
stepper, on ragged grids (several tiles and ragged tails) with periodic and transmissive
boundaries; plus the full Sod configuration with Roe and the Kelvin--Helmholtz shear layer
with WENO3 + Roe."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note

pytestmark = pytest.mark.gpu

SHAPES = {1: (600,), 2: (150, 20), 3: (20, 12, 9)}
RECONS = ("first_order", "muscl_minmod", "weno3", "eno2")
PAIRS = ([("euler", "roe", r) for r in RECONS] +
         [("euler", f, "eno2") for f in ("rusanov", "hll", "hllc")] +
         [("burgers", "roe", r) for r in RECONS] + [("burgers", "ec", r) for r in RECONS] +
         [("burgers", f, "eno2") for f in ("rusanov", "hll")] +
         [("advection", "roe", r) for r in RECONS] +
         [("advection", f, "eno2") for f in ("rusanov", "hll")])
COMBOS = [(d, eq, fl, rc, it) for d in (1, 2, 3) for eq, fl, rc in PAIRS
          for it in ("forward_euler", "ssprk2", "ssprk3")]


def _initial(p, seed):
    nz, ny, nx = p.n[2], p.n[1], p.n[0]
    if p.eq == "euler":
        return fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)
    rng = np.random.default_rng(seed)
    base = fi.random_smooth_state(seed, (nz, ny, nx), p.dim, batch=2)[:, :1] - 1.0
    return np.ascontiguousarray(base * 5.0 + 0.1 * rng.standard_normal(base.shape))


@pytest.mark.parametrize("dim,eq,flux,recon,integ", COMBOS)
def test_more_schemes_match_oracle(dim, eq, flux, recon, integ):
    idx = COMBOS.index((dim, eq, flux, recon, integ))
    bc = ("transmissive",) * 3 if idx % 2 == 0 else ("periodic",) * 3
    p = O.Problem(dim=dim, n=SHAPES[dim], eq=eq, flux=flux, recon=recon, integrator=integ, bc=bc,
                  vel=(0.7, -0.4, 0.3))
    U0 = _initial(p, 31 + dim)
    note("scheme", dim, eq, flux, recon, integ, bc[0])
    K = 6
    R, rt, rsteps, rerr = O.evolve(p, U0, 1e3, 0.4, max_steps=K)
    G, gt, gsteps, gerr, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=K, mode="advance")
    assert np.all(rerr == 6) and np.all(gerr == 0) and st == 0
    assert np.all(gsteps == K) and np.array_equal(gt, rt)
    assert_parity(G, R, what=f"{dim}D {eq} {flux} {recon} {integ}")


def test_sod_roe_full_configuration():
    N = 1024
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="roe", recon="eno2", integrator="ssprk2",
                  bc=("transmissive",))
    U0 = fi.sod_state(N)
    note("sod roe eno2")
    R, rt, rs, re = O.evolve(p, U0, 0.2, 0.45)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.2, 0.45)
    assert gs[0] == rs[0] and gt[0] == rt[0] == 0.2
    assert_parity(G, R, what="sod roe eno2")


def test_kh_weno3_roe_bitwise():
    c, phi = fi.kh_coefficients(1912, [0, 1])
    U0 = fi.kh2d_state(128, c, phi)
    p = O.Problem(dim=2, n=(128, 128), eq="euler", flux="roe", recon="weno3", integrator="ssprk3")
    note("kh roe")
    R, rt, rs, re = O.evolve(p, U0, 2.0, 0.4, max_steps=40)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 2.0, 0.4, max_steps=40, mode="advance")
    assert np.all(gs == 40) and np.array_equal(gt, rt)
    assert_parity(G, R, what="kh roe")


def test_ec_rejected_for_advection_and_shallow_water():
    import paper_1912_07645_amd.fv as fv
    from paper_1912_07645_amd import Solver
    for eq in ("advection", "swe"):
        for flux in ("ec", "ec4"):
            with pytest.raises(fv.FVError) as e:
                Solver(dim=1, n=(16,), eq=eq, flux=flux)
            assert e.value.status == fv.FV_ENOTSUP


def test_kh_roe_1024_full_size_bitwise():
    """The WENO3 + Roe benchmark configuration at its full 1024^2 size, 3 steps, every cell."""
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(1024, c, phi)
    p = O.Problem(dim=2, n=(1024, 1024), eq="euler", flux="roe", recon="weno3", integrator="ssprk3")
    note("kh roe 1024 oracle")
    R, rt, rs, re = O.evolve(p, U0, 2.0, 0.4, max_steps=3)
    note("kh roe 1024 gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 2.0, 0.4, max_steps=3, mode="advance")
    assert gs[0] == 3 and gt[0] == rt[0]
    assert_parity(G, R, what="kh roe 1024")
