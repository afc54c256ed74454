"""GPU parity of ideal MHD against the oracle, through the C-ABI, bit for bit (the same
operation-exact arithmetic on both sides): Rusanov and HLL with every reconstruction and
stepper in 1D, 2D and 3D on ragged grids with both boundary kinds; the Brio--Wu shock tube to
its usual final time; the Orszag--Tang vortex (128^2 for 100 steps, and the 1024^2 benchmark
configuration for 3 steps, every cell); statistics, PDFs and shell structure functions of MHD
samples; the rejected fluxes."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0
SHAPES = {1: (600,), 2: (150, 20), 3: (20, 12, 9)}
RECONS = ("first_order", "muscl_minmod", "weno3", "eno2")
COMBOS = [(d, fl, rc, it) for d in (1, 2, 3) for fl in ("rusanov", "hll") for rc in RECONS
          for it in ("forward_euler", "ssprk2", "ssprk3")]


@pytest.mark.parametrize("dim,flux,recon,integ", COMBOS)
def test_mhd_schemes_match_oracle(dim, flux, recon, integ):
    idx = COMBOS.index((dim, flux, recon, integ))
    bc = ("transmissive",) * 3 if idx % 2 == 0 else ("periodic",) * 3
    p = O.Problem(dim=dim, n=SHAPES[dim], eq="mhd", flux=flux, recon=recon, integrator=integ,
                  bc=bc, gamma=G53)
    U0 = fi.random_smooth_mhd(40 + dim, p.state_shape[1:], dim, batch=2)
    note("mhd", dim, flux, recon, integ, bc[0])
    K = 6
    R, rt, rsteps, rerr = O.evolve(p, U0, 1e3, 0.4, max_steps=K)
    G, gt, gsteps, gerr, st = gpu_evolve(p, U0, 1e3, 0.4, max_steps=K, mode="advance")
    assert np.all(rerr == 6) and np.all(gerr == 0) and st == 0
    assert np.all(gsteps == K) and np.array_equal(gt, rt)
    assert_parity(G, R, what=f"{dim}D mhd {flux} {recon} {integ}")


@pytest.mark.parametrize("recon", ["muscl_minmod", "eno2"])
def test_brio_wu_to_final_time(recon):
    N = 800
    p = O.Problem(dim=1, n=(N,), eq="mhd", flux="hll", recon=recon, integrator="ssprk2",
                  bc=("transmissive",), gamma=2.0)
    U0 = fi.brio_wu_state(N)
    note("brio-wu", recon)
    R, rt, rs, re = O.evolve(p, U0, 0.1, 0.5)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 0.1, 0.5)
    assert st == 0 and gs[0] == rs[0] and gt[0] == rt[0] == 0.1
    assert np.all(G[0, 5] == 0.75)
    assert_parity(G, R, what=f"brio-wu {recon}")


def test_orszag_tang_128():
    n = 128
    p = O.Problem(dim=2, n=(n, n), eq="mhd", flux="hll", recon="muscl_minmod", integrator="ssprk2",
                  gamma=G53)
    U0 = fi.orszag_tang_state(n, G53)
    note("orszag-tang 128")
    R, rt, rs, re = O.evolve(p, U0, 10.0, 0.4, max_steps=100)
    G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=100, mode="advance")
    assert gs[0] == 100 and gt[0] == rt[0]
    assert_parity(G, R, what="orszag-tang 128")


def test_orszag_tang_1024_full_size_bitwise():
    """The MHD benchmark configuration (1024^2, MUSCL + Rusanov + SSP-RK2) at full size, 3
    steps, every cell. (With HLL and MUSCL on the conserved variables this vortex reaches a
    negative pressure near t = 0.08 at this size, on both sides alike; Rusanov runs past
    t = 0.45, so the benchmark uses it.)"""
    n = 1024
    p = O.Problem(dim=2, n=(n, n), eq="mhd", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk2", gamma=G53)
    U0 = fi.orszag_tang_state(n, G53)
    note("orszag-tang 1024 oracle")
    R, rt, rs, re = O.evolve(p, U0, 10.0, 0.4, max_steps=3)
    note("orszag-tang 1024 gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=3, mode="advance")
    assert gs[0] == 3 and gt[0] == rt[0]
    assert_parity(G, R, what="orszag-tang 1024")


def test_mhd_statistics_match_oracle():
    torch = torch_gpu()
    from paper_1912_07645_amd import Stats
    n = 40
    p = O.Problem(dim=2, n=(n, n), eq="mhd", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk2", gamma=G53)
    U0 = fi.random_smooth_mhd(88, (1, n, n), 2, batch=10)
    G, *_ = gpu_evolve(p, U0, 1e3, 0.4, max_steps=4, mode="advance")
    s = solver_for(p)
    st = Stats(s, max_h=5)
    Ud = torch.from_numpy(G).to("cuda")
    st.accumulate(Ud)
    res = st.read()
    R = O.Stats(p, max_h=5)
    R.accumulate(G)
    assert res["count"] == 10
    assert np.array_equal(res["mean"].cpu().numpy(), R.mean)
    assert np.array_equal(res["var"].cpu().numpy(), R.variance())
    assert np.allclose(res["s2_mean"].cpu().numpy(), R.s2(), rtol=1e-12, atol=0)
    pts = [0, 9, n * n - 1]
    for q in range(8):
        lo, hi = float(G[:, q].min()) - 0.01, float(G[:, q].max()) + 0.01
        Gp = s.point_pdf(Ud, q, pts, lo, hi, 7).cpu().numpy()
        assert np.array_equal(Gp, O.point_pdf(p, G, q, pts, lo, hi, 7)), q
    S = s.structure_shell(Ud, 3, 2, False).cpu().numpy()
    Rs = O.structure_shell_batch(p, G, 3, 2, False)
    assert (np.abs(S - Rs) <= 1e-12 * np.abs(Rs)).all()


def test_mhd_rejections():
    import paper_1912_07645_amd.fv as fv
    from paper_1912_07645_amd import Solver
    for flux in ("hllc", "roe", "godunov", "ec", "ec4"):
        with pytest.raises(fv.FVError) as e:
            Solver(dim=2, n=(16, 16), eq="mhd", flux=flux, gamma=G53)
        assert e.value.status == fv.FV_ENOTSUP
    with pytest.raises(fv.FVError) as e:
        Solver(dim=1, n=(16,), eq="mhd", flux="hll", gamma=1.0)
    assert e.value.status == fv.FV_EINVAL
