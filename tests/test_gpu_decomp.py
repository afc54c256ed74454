"""Split-buffer decomposition (fv_decomp_*): subdomains with stored ghost layers, a halo
exchange (pack, device-to-device copies on a second stream, unpack) every Runge--Kutta stage,
and interior-first overlap. The bar is the unsplit solver's result, bit for bit: same
states, times, step counts and statuses, for every split, with and without overlap."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu


def _unsplit(s, U0, t_end, cfl, nsteps):
    torch = torch_gpu()
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    B = U.shape[0]
    t = torch.zeros(B, dtype=torch.float64, device="cuda")
    k = torch.zeros(B, dtype=torch.int64, device="cuda")
    e = torch.zeros(B, dtype=torch.int32, device="cuda")
    st = s.advance(U, t, t_end, cfl, nsteps, k, e)
    torch.cuda.synchronize()
    return U.cpu().numpy(), t.cpu().numpy(), k.cpu().numpy(), e.cpu().numpy(), st


def _split(s, parts, U0, t_end, cfl, nsteps, overlap, chunks=1, dma=False):
    torch = torch_gpu()
    from paper_1912_07645_amd.decomp import Decomposition
    B = U0.shape[0]
    d = Decomposition(s, parts, B)
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    d.scatter(U)
    t = torch.zeros(B, dtype=torch.float64, device="cuda")
    k = torch.zeros(B, dtype=torch.int64, device="cuda")
    e = torch.zeros(B, dtype=torch.int32, device="cuda")
    st = 0
    done = 0
    k_acc = torch.zeros_like(k)
    for c in range(chunks):   # several calls continue from the stored subdomain states
        n = nsteps // chunks if c < chunks - 1 else nsteps - done
        st = d.advance(t, t_end, cfl, n, k, e, overlap, dma)
        k_acc += k
        done += n
    out = torch.full_like(U, float("nan"))
    d.gather(out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), t.cpu().numpy(), k_acc.cpu().numpy(), e.cpu().numpy(), st, d.info()


def _same(a, b, what):
    for x, y, name in zip(a[:4], b[:4], ("state", "t", "steps", "err")):
        assert np.array_equal(x, y), f"{what}: {name} differs"
    assert a[4] == b[4], f"{what}: status {a[4]} vs {b[4]}"


CASES = [
    # (n, parts, recon, flux, integrator, batch)
    ((100, 90), (2, 1), "weno3", "hllc", "ssprk3", 2),
    ((100, 90), (1, 2), "weno3", "hllc", "ssprk3", 2),
    ((100, 90), (2, 2), "weno3", "hllc", "ssprk3", 2),
    ((100, 90), (4, 2), "weno3", "hllc", "ssprk3", 2),
    ((32, 24), (4, 2), "weno3", "hllc", "ssprk3", 2),     # a subdomain is one ragged tile
    ((100, 90), (2, 2), "muscl_minmod", "hll", "ssprk2", 2),
    ((96, 60), (1, 2), "muscl_minmod", "rusanov", "ssprk3", 3),
    ((40, 36, 34), (1, 1, 2), "weno3", "hllc", "ssprk3", 2),
    ((40, 36, 34), (2, 1, 2), "weno3", "hllc", "ssprk3", 1),
    ((40, 36, 34), (2, 2, 2), "weno3", "hllc", "ssprk3", 1),
]


@pytest.mark.parametrize("overlap,dma", [(True, False), (False, False), (True, True)])
@pytest.mark.parametrize("n,parts,recon,flux,integ,B", CASES)
def test_split_run_equals_unsplit(n, parts, recon, flux, integ, B, overlap, dma):
    torch_gpu()
    dim = len(n)
    p = O.Problem(dim=dim, n=n, eq="euler", flux=flux, recon=recon, integrator=integ)
    shape = (n[2] if dim == 3 else 1, n[1], n[0])
    U0 = fi.random_smooth_state(5 + sum(parts), shape, dim, batch=B)
    s = solver_for(p)
    note("decomp", n, parts, recon, flux, integ, "overlap" if overlap else "serial")
    ref = _unsplit(s, U0, 10.0, 0.4, 12)
    got = _split(s, parts, U0, 10.0, 0.4, 12, overlap, chunks=2, dma=dma)
    _same(got, ref, f"{n} split {parts}")
    info = got[5]
    assert info["subdomains"] == int(np.prod(parts))
    split_axes = sum(1 for x in parts if x > 1)
    assert info["messages"] == 2 * split_axes * info["subdomains"]


def test_split_run_stops_at_t_end_per_sample():
    """Samples with different step sizes reach t_end after different numbers of steps; the
    split run clips and stops them exactly as the unsplit one."""
    torch_gpu()
    p = O.Problem(dim=2, n=(64, 48), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    U0 = fi.random_smooth_state(41, (1, 48, 64), 2, batch=3)
    U0[1] = U0[1] * np.array([1.0, 1.7, 1.7, 2.9])[:, None, None, None]   # faster sample
    s = solver_for(p)
    ref = _unsplit(s, U0, 0.02, 0.4, 400)
    assert len(set(ref[2].tolist())) > 1          # different step counts
    got = _split(s, (2, 2), U0, 0.02, 0.4, 400, True)
    _same(got, ref, "t_end")
    assert np.all(got[1] == 0.02)


def test_split_run_reports_a_non_physical_sample():
    torch_gpu()
    p = O.Problem(dim=2, n=(40, 30), eq="euler", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk2")
    U0 = fi.random_smooth_state(9, (1, 30, 40), 2, batch=3)
    U0[1, 0, 0, 20, 3] = -0.5
    s = solver_for(p)
    ref = _unsplit(s, U0, 10.0, 0.4, 6)
    got = _split(s, (2, 1), U0, 10.0, 0.4, 6, True)
    _same(got, ref, "non-physical")
    assert got[4] == 5 and got[3][1] == 5


@pytest.mark.parametrize("parts", [(2, 1), (1, 2), (2, 2)])
def test_kh_1024_split_equals_unsplit(parts):
    """The Kelvin--Helmholtz configuration at its full size (1024^2, WENO3 + HLLC + SSP-RK3,
    CFL 0.4), 30 steps, each split with overlap, and the 2 x 2 split also without."""
    torch_gpu()
    n = 1024
    p = O.Problem(dim=2, n=(n, n), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(n, c, phi)
    s = solver_for(p)
    note("decomp kh 1024", parts)
    ref = _unsplit(s, U0, 10.0, 0.4, 30)
    _same(_split(s, parts, U0, 10.0, 0.4, 30, True), ref, f"kh 1024 {parts}")
    _same(_split(s, parts, U0, 10.0, 0.4, 30, True, dma=True), ref, f"kh 1024 {parts} dma")
    if parts == (2, 2):
        _same(_split(s, parts, U0, 10.0, 0.4, 30, False), ref, "kh 1024 2x2 serial")


def test_kh3d_512_z_split_equals_unsplit():
    """The 3D Kelvin--Helmholtz configuration at its full size (512^3, WENO3 + HLLC + SSP-RK3),
    2 steps, split in two along z with overlap."""
    torch = torch_gpu()
    n = 512
    p = O.Problem(dim=3, n=(n, n, n), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    cx, px, cz, pz = fi.kh3d_coefficients(1914, [0])
    U0 = fi.kh3d_state(n, cx, px, cz, pz)
    s = solver_for(p)
    note("decomp kh3d 512 z split")
    ref = _unsplit(s, U0, 10.0, 0.4, 2)
    del s
    torch.cuda.empty_cache()
    s = solver_for(p)
    got = _split(s, (1, 1, 2), U0, 10.0, 0.4, 2, True, dma=True)
    _same(got, ref, "kh3d z split")


def test_decomposition_rejections():
    torch_gpu()
    import paper_1912_07645_amd.fv as fv
    from paper_1912_07645_amd.decomp import Decomposition

    def status(p, parts):
        with pytest.raises(fv.FVError) as e:
            Decomposition(solver_for(p), parts, 1)
        return e.value.status

    base = dict(dim=2, n=(64, 64), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    assert status(O.Problem(**base), (3, 1)) == fv.FV_EINVAL            # 3 does not divide 64
    assert status(O.Problem(**base), (1, 1, 2)) == fv.FV_EINVAL         # beyond the dimension
    assert status(O.Problem(**base), (4, 4)) == fv.FV_ENOTSUP           # 16 subdomains
    assert status(O.Problem(**dict(base, n=(8, 64))), (4, 1)) == fv.FV_EINVAL   # 2 cells each
    assert status(O.Problem(**dict(base, integrator="forward_euler")), (2, 1)) == fv.FV_ENOTSUP
    assert status(O.Problem(**dict(base, flux="roe")), (2, 1)) == fv.FV_ENOTSUP
    assert status(O.Problem(**dict(base, bc=("transmissive", "periodic"))), (2, 1)) == fv.FV_ENOTSUP
    # a transmissive axis that is not split is fine
    Decomposition(solver_for(O.Problem(**dict(base, bc=("periodic", "transmissive")))), (2, 1), 1)


@pytest.mark.parametrize("overlap,dma", [(True, False), (False, False), (True, True)])
def test_graph_replays_equal_direct_launches(overlap, dma, monkeypatch):
    """Whole chunks of 16 steps replay a graph captured over both streams; 50 steps (three
    replays and a remainder) equal the same run launched directly and the unsplit run."""
    torch_gpu()
    p = O.Problem(dim=2, n=(100, 90), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    U0 = fi.random_smooth_state(23, (1, 90, 100), 2, batch=2)
    s = solver_for(p)
    ref = _unsplit(s, U0, 10.0, 0.4, 50)
    note("decomp graph replays", overlap)
    _same(_split(s, (2, 2), U0, 10.0, 0.4, 50, overlap, dma=dma), ref, "graph")
    monkeypatch.setenv("FV_NO_GRAPH", "1")
    _same(_split(s, (2, 2), U0, 10.0, 0.4, 50, overlap, dma=dma), ref, "direct")
