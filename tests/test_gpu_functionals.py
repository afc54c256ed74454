"""GPU parity of the point PDFs, joint PDFs and cube/ball shell structure functions against
the oracle, through the C-ABI: counts equal bit for bit (the bin decision is taken in FP64 in
the same order on both sides), structure functions to 1e-12 relative (the GPU sums per cell,
then over cells; the oracle per offset over cells). Inputs are Kelvin--Helmholtz samples with
Sobol (QMC) and SplitMix64 (MC) perturbations, evolved on the GPU first, plus edge cases:
NaN and out-of-range values, ragged grids, every dimension, the largest radius each
dimension offers."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import gpu_evolve, note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu


def _kh_batch(n, samples, qmc, steps):
    if qmc:
        c, phi = fi.kh_coefficients_qmc(np.arange(samples))
    else:
        c, phi = fi.kh_coefficients(1912, np.arange(samples))
    U0 = fi.kh2d_state(n, c, phi)
    p = O.Problem(dim=2, n=(n, n), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    if steps:
        U0, _, _, _, _ = gpu_evolve(p, U0, 10.0, 0.4, max_steps=steps, mode="advance")
    return p, U0


def _to_gpu(U):
    torch = torch_gpu()
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


@pytest.mark.parametrize("qmc", [True, False])
def test_point_and_joint_pdfs_bitwise(qmc):
    p, U = _kh_batch(64, 48, qmc, steps=5)
    s = solver_for(p)
    Ud = _to_gpu(U)
    N = p.cells
    points = [0, 1, 63, 64 * 31 + 17, N // 2, N - 1]
    # ranges that cut through the values, so every case (in, below, above) occurs
    ranges = {0: (0.5, 1.8, 13), 1: (-0.4, 0.4, 8), 2: (-0.005, 0.005, 5), 3: (2.6, 3.2, 31)}
    for q, (lo, hi, nb) in ranges.items():
        note("point pdf", "qmc" if qmc else "mc", "quantity", q)
        G = s.point_pdf(Ud, q, points, lo, hi, nb).cpu().numpy()
        R = O.point_pdf(p, U, q, points, lo, hi, nb)
        assert np.array_equal(G, R), (q, G, R)
        assert (G.sum(axis=1) == U.shape[0]).all()
    pairs = [(0, 1), (N // 2, N // 2 + 64), (N - 1, 0), (5, 5)]
    note("joint pdf")
    G = s.joint_pdf(Ud, 0, 3, pairs, 0.5, 1.8, 2.6, 3.2, 7).cpu().numpy()
    R = O.joint_pdf(p, U, 0, 3, pairs, 0.5, 1.8, 2.6, 3.2, 7)
    assert np.array_equal(G, R)
    # counts are added to the caller's array: a second call doubles them
    torch = torch_gpu()
    acc = torch.zeros((len(points), 15), dtype=torch.int64, device="cuda")
    s.point_pdf(Ud, 0, points, 0.5, 1.8, 13, acc)
    s.point_pdf(Ud, 0, points, 0.5, 1.8, 13, acc)
    assert np.array_equal(acc.cpu().numpy(), 2 * O.point_pdf(p, U, 0, points, 0.5, 1.8, 13))


def test_pdf_edge_values_bitwise():
    # NaN, values on bin edges, the rounding edge below hi, values outside the range
    p = O.Problem(dim=1, n=(9,), eq="euler")
    vals = [float("nan"), -0.5, 0.2, 0.375, 0.55, float(np.nextafter(0.9, 0.0)), 0.9, 1e300, -1e300]
    U = np.ones((len(vals),) + p.state_shape)
    for b, v in enumerate(vals):
        U[b, 0, 0, 0, :] = v
        U[b, 0, 0, 0, 3] = 1.0 + b
    s = solver_for(p)
    Ud = _to_gpu(U)
    for nb in (1, 4, 7):
        for q in (0, 1, 2):
            G = s.point_pdf(Ud, q, list(range(9)), 0.2, 0.9, nb).cpu().numpy()
            R = O.point_pdf(p, U, q, list(range(9)), 0.2, 0.9, nb)
            assert np.array_equal(G, R), (nb, q)
        G = s.joint_pdf(Ud, 0, 1, [(0, 3), (2, 2)], 0.2, 0.9, 0.0, 2.0, nb).cpu().numpy()
        R = O.joint_pdf(p, U, 0, 1, [(0, 3), (2, 2)], 0.2, 0.9, 0.0, 2.0, nb)
        assert np.array_equal(G, R)


def test_pdf_argument_errors():
    import paper_1912_07645_amd.fv as fv
    p = O.Problem(dim=2, n=(8, 8), eq="euler")
    s = solver_for(p)
    U = _to_gpu(np.ones((2,) + p.state_shape))
    for args in [(4, [0], 0.0, 1.0, 4), (0, [64], 0.0, 1.0, 4), (0, [-1], 0.0, 1.0, 4),
                 (0, [0], 1.0, 1.0, 4), (0, [0], 0.0, float("nan"), 4), (0, [0], 0.0, 1.0, 0)]:
        with pytest.raises(fv.FVError) as e:
            s.point_pdf(U, *args)
        assert e.value.status == fv.FV_EINVAL


SHELL_CASES = [
    (1, (300,), "euler", 40),        # a 1D tile is 256 cells: two tiles, the second ragged
    (2, (37, 29), "euler", 12),      # ragged tiles on both axes
    (2, (80, 72), "burgers", 36),    # the largest radius a 2D tile's halo allows
    (3, (11, 13, 9), "euler", 4),
    (3, (14, 14, 14), "advection", 6),
]


@pytest.mark.parametrize("dim,n,eq,H", SHELL_CASES)
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ball", [False, True])
def test_shell_structure_functions_match_oracle(dim, n, eq, H, order, ball):
    p = O.Problem(dim=dim, n=n, eq=eq)
    rng = np.random.default_rng(dim * 100 + H)
    if eq == "euler":
        U = fi.random_smooth_state(7 + dim, p.state_shape[1:], dim, batch=3)
    else:
        U = rng.normal(size=(3,) + p.state_shape)
    note("shell", dim, n, eq, H, order, "ball" if ball else "cube")
    s = solver_for(p)
    G = s.structure_shell(_to_gpu(U), H, order, ball).cpu().numpy()
    R = O.structure_shell_batch(p, U, H, order, ball)
    assert G.shape == R.shape
    rel = np.abs(G - R) / np.maximum(np.abs(R), 1e-300)
    assert rel.max() <= 1e-12, rel.max()


def test_shell_errors():
    import paper_1912_07645_amd.fv as fv
    for p, H, want in [(O.Problem(dim=2, n=(16, 16), bc=("transmissive", "periodic")), 2, fv.FV_ENOTSUP),
                       (O.Problem(dim=2, n=(16, 8)), 8, fv.FV_ENOTSUP),
                       (O.Problem(dim=3, n=(16, 16, 16)), 7, fv.FV_ENOTSUP),
                       (O.Problem(dim=2, n=(16, 16)), 0, fv.FV_EINVAL)]:
        s = solver_for(p)
        U = _to_gpu(np.ones((1,) + p.state_shape))
        with pytest.raises(fv.FVError) as e:
            s.structure_shell(U, H)
        assert e.value.status == want


def test_full_batch_functionals():
    """The batched Monte Carlo configuration (256^2, 1024 QMC samples, 3 steps): PDFs of
    every quantity at 16 points and 4 pairs bit for bit; shell structure functions of radius
    up to 8 on sampled samples to 1e-12."""
    p, U = _kh_batch(256, 1024, True, steps=3)
    s = solver_for(p)
    Ud = _to_gpu(U)
    N = p.cells
    points = [int(v) for v in np.linspace(0, N - 1, 16)]
    for q, (lo, hi) in enumerate([(0.9, 2.1), (-0.6, 0.6), (-0.02, 0.02), (2.4, 3.6)]):
        note("full batch point pdf, quantity", q)
        G = s.point_pdf(Ud, q, points, lo, hi, 50).cpu().numpy()
        assert np.array_equal(G, O.point_pdf(p, U, q, points, lo, hi, 50))
    pairs = [(N // 2, N // 2 + d) for d in (1, 2, 8, 256)]
    G = s.joint_pdf(Ud, 1, 1, pairs, -0.6, 0.6, -0.6, 0.6, 20).cpu().numpy()
    assert np.array_equal(G, O.joint_pdf(p, U, 1, 1, pairs, -0.6, 0.6, -0.6, 0.6, 20))
    note("full batch shell structure functions")
    S = s.structure_shell(Ud, 8, 2, False).cpu().numpy()
    assert S.shape == (1024, 4, 8) and np.isfinite(S).all()
    for b in (0, 511, 1023):
        R = O.structure_shell_batch(p, U[b:b + 1], 8, 2, False)[0]
        rel = np.abs(S[b] - R) / np.maximum(np.abs(R), 1e-300)
        assert rel.max() <= 1e-12, (b, rel.max())
