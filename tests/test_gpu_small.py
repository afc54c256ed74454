"""The single-workgroup time loop for small 1D grids (offered as the last tile variant), for
every 1D equation and flux except the fourth-order EC flux:
bit for bit against the oracle and against the tiled path -- states, times, step counts and
per-sample status -- for every 1D scheme it is built for, every stepper and both boundary
kinds, on grids from 1 cell to its largest; the Sod configuration; runs longer than one
launch's chunk of steps; the stop rules (t_end, max_steps as error or limit, non-physical
states, fixed steps and their CFL bound)."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu

RECONS = ("first_order", "muscl_minmod", "weno3", "eno2")
PAIRS = ([("euler", f) for f in ("rusanov", "hll", "hllc", "roe", "godunov", "ec")] +
         [("burgers", f) for f in ("rusanov", "hll", "roe", "godunov", "ec")] +
         [("advection", f) for f in ("rusanov", "hll", "roe", "godunov")] +
         [("swe", f) for f in ("rusanov", "hll", "roe")] + [("mhd", f) for f in ("rusanov", "hll")])
# the Euler Godunov and entropy-conservative fluxes call pow/exp/log: against the oracle they
# agree to rounding (as on the tiled path); against the tiled path bit for bit
ROUNDING = {("euler", "godunov"), ("euler", "ec")}
COMBOS = [(eq, fl, rc, it) for eq, fl in PAIRS for rc in RECONS
          for it in ("forward_euler", "ssprk2", "ssprk3")]


def _small_variant(s):
    nv = s.num_variants()
    s.set_variant(nv - 1)
    (bx, by, bz), v = s.tile()
    assert v == nv - 1 and bx == s.n[0] and by == bz == 1
    return nv - 1


def _initial(p, seed, batch=3):
    nx = p.n[0]
    if p.eq == "swe":
        return fi.random_smooth_swe(seed, (1, 1, nx), 1, batch=batch)
    if p.eq == "mhd":
        return fi.random_smooth_mhd(seed, (1, 1, nx), 1, batch=batch)
    if p.eq == "euler":
        return fi.random_smooth_state(seed, (1, 1, nx), 1, batch=batch)
    rng = np.random.default_rng(seed)
    base = fi.random_smooth_state(seed, (1, 1, nx), 1, batch=batch)[:, :1] - 1.0
    return np.ascontiguousarray(base * 5.0 + 0.1 * rng.standard_normal(base.shape))


@pytest.mark.parametrize("eq,flux,recon,integ", COMBOS)
def test_small_matches_oracle_and_tiled(eq, flux, recon, integ):
    idx = COMBOS.index((eq, flux, recon, integ))
    bc = "transmissive" if idx % 2 == 0 else "periodic"
    n = (600, 37, 1, 1024, 5)[idx % 5]
    if eq == "mhd":
        n = min(n, 477)          # the largest MHD grid the single workgroup takes
    p = O.Problem(dim=1, n=(n,), eq=eq, flux=flux, recon=recon, integrator=integ, bc=(bc,),
                  vel=(0.7, 0.0, 0.0), gamma=5.0 / 3.0 if eq == "mhd" else 1.4)
    U0 = _initial(p, 11 + idx)
    note("small", eq, flux, recon, integ, bc, n)
    K = 7
    R, rt, rs, rerr = O.evolve(p, U0, 1e3, 0.4, max_steps=K)
    s = solver_for(p)
    G0, t0, s0, e0, st0 = gpu_evolve(p, U0, 1e3, 0.4, max_steps=K, mode="advance", solver=s)
    _small_variant(s)
    G1, t1, s1, e1, st1 = gpu_evolve(p, U0, 1e3, 0.4, max_steps=K, mode="advance", solver=s)
    # the oracle reports the step limit as status 6; advance takes it as a plain stop. (An
    # entropy-conservative flux without dissipation can leave the physical states, which both
    # sides report alike.)
    want = np.where(rerr == 6, 0, rerr)
    assert np.array_equal(e0, want) and np.array_equal(e1, want) and st1 == st0
    assert np.array_equal(s1, s0) and np.all(s1[rerr == 6] == K)
    # a sample that failed may hold NaN from its last step, alike on both paths
    assert np.array_equal(t1, t0) and np.array_equal(G1, G0, equal_nan=True)
    what = f"small {eq} {flux} {recon} {integ} {bc} {n}"
    ok = rerr == 6
    if (eq, flux) in ROUNDING:
        assert np.allclose(t1, rt, rtol=1e-13, atol=0.0)
        assert_parity(G1[ok], R[ok], tol=1e-12, bitwise=False, what=what)
    else:
        assert np.array_equal(t1, rt)
        assert_parity(G1[ok], R[ok], what=what)


def test_small_sod_full_configuration():
    N = 1024
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="rusanov", recon="first_order",
                  integrator="forward_euler", bc=("transmissive",))
    U0 = fi.sod_state(N)
    R, rt, rs, re = O.evolve(p, U0, 0.2, 0.45)
    s = solver_for(p)
    _small_variant(s)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.2, 0.45, solver=s)
    assert st == 0 and gs[0] == rs[0] and gt[0] == rt[0] == 0.2 and ge[0] == 0
    assert_parity(G, R, what="small sod")


def test_small_largest_grid_and_no_variant_beyond():
    """Euler with WENO3 at the largest grid the variant takes, and no such variant above it."""
    from paper_1912_07645_amd import Solver
    s = Solver(dim=1, n=(1277,), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    nv = s.num_variants()
    s2 = Solver(dim=1, n=(1278,), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    assert s2.num_variants() == nv - 1
    p = O.Problem(dim=1, n=(1277,), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    U0 = _initial(p, 5, batch=2)
    R, rt, rs, re = O.evolve(p, U0, 1e3, 0.4, max_steps=5)
    s = solver_for(p)
    _small_variant(s)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=5, mode="advance", solver=s)
    assert np.all(gs == 5) and np.array_equal(gt, rt)
    assert_parity(G, R, what="small 1277")


def test_small_runs_longer_than_one_launch():
    """About 70 000 steps of a 16-cell advection run: more than one launch's chunk (65 536
    steps); the result equals the tiled path's."""
    p = O.Problem(dim=1, n=(16,), eq="advection", flux="rusanov", integrator="forward_euler",
                  vel=(1.0, 0.0, 0.0))
    rng = np.random.default_rng(3)
    U0 = rng.standard_normal((2,) + p.state_shape)
    t_end = 70000 * 0.9 / 16
    s = solver_for(p)
    note("small long run, tiled")
    G0, t0, s0, e0, st0 = gpu_evolve(p, U0, t_end, 0.9, solver=s)
    _small_variant(s)
    note("small long run, single workgroup")
    G1, t1, s1, e1, st1 = gpu_evolve(p, U0, t_end, 0.9, solver=s)
    assert st0 == st1 == 0 and np.all(s1 > 65536)
    assert np.array_equal(s1, s0) and np.array_equal(t1, t0) and np.array_equal(G1, G0)


def test_small_stop_rules():
    torch = torch_gpu()
    import paper_1912_07645_amd.fv as fv
    p = O.Problem(dim=1, n=(64,), eq="euler", flux="hll", recon="muscl_minmod",
                  integrator="ssprk2", bc=("transmissive",))
    U0 = _initial(p, 17, batch=3)
    U0[1, 0, 0, 0, 10] = -0.5                     # sample 1 starts non-physical
    s = solver_for(p)
    outs = []
    for v in (0, s.num_variants() - 1):
        s.set_variant(v)
        row = []
        # max_steps reached before t_end: an error for evolve, a limit for advance
        for mode in ("evolve", "advance"):
            G, t, st_, e, status = gpu_evolve(p, U0, 1e3, 0.4, max_steps=4, mode=mode, solver=s)
            row.append((G, t, st_, e, status))
        # fixed steps: within the bound, then beyond it
        for dt in (1e-3, 10.0):
            U = torch.from_numpy(U0.copy()).cuda()
            err = torch.zeros(3, dtype=torch.int32, device="cuda")
            status = s.evolve_fixed_dt(U, dt, 6, 0.9, err)
            row.append((U.cpu().numpy(), None, None, err.cpu().numpy(), status))
        outs.append(row)
    tiled, small = outs
    for a, b in zip(tiled, small):
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[3], b[3]) and a[4] == b[4]
        if a[1] is not None:
            assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    ev, ad, fx, fb = small
    assert list(ev[3]) == [fv.FV_EMAXSTEPS, fv.FV_ENONPHYS, fv.FV_EMAXSTEPS] and ev[4] == fv.FV_EMAXSTEPS
    assert list(ad[3]) == [0, fv.FV_ENONPHYS, 0] and list(ad[2]) == [4, 0, 4]
    assert list(fx[3]) == [0, fv.FV_ENONPHYS, 0]
    assert list(fb[3]) == [fv.FV_ECFL, fv.FV_ENONPHYS, fv.FV_ECFL]


def test_tuner_times_the_single_workgroup_variant():
    """The tuner times every variant, the single-workgroup one included, and the run with its
    choice equals the oracle bit for bit."""
    torch = torch_gpu()
    N = 1024
    p = O.Problem(dim=1, n=(N,), eq="euler", flux="rusanov", recon="first_order",
                  integrator="forward_euler", bc=("transmissive",))
    U0 = fi.sod_state(N)
    s = solver_for(p)
    chosen = s.tune(torch.from_numpy(U0).cuda())
    assert 0 <= chosen < s.num_variants() and s.tile()[1] == chosen
    R, rt, rs, re = O.evolve(p, U0, 0.2, 0.45)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.2, 0.45, solver=s)
    assert gs[0] == rs[0] and gt[0] == rt[0]
    assert_parity(G, R, what=f"sod with tuned variant {chosen}")
