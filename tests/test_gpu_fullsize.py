"""Parity at the full sizes of the benchmark configurations, against the oracle: the 1024^2
Kelvin--Helmholtz run over 100 steps, the batched run of 1024 samples of 256^2 (states of
samples at both ends and in the middle of the batch), the statistics of a full 1024-sample
batch with structure functions up to lag 32, and the device division and square root on
10^8 inputs."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from gpu_helpers import assert_parity, gpu_evolve, note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu


def _kh_problem(n):
    return O.Problem(dim=2, n=(n, n), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")


@pytest.mark.timeout(900)
def test_kh_1024_hundred_steps_bitwise():
    """2D KH, 1024^2, WENO3 + HLLC + SSP-RK3, CFL 0.4: 100 steps, every cell, bit for bit."""
    c, phi = fi.kh_coefficients(1912, [0])
    U0 = fi.kh2d_state(1024, c, phi)
    p = _kh_problem(1024)
    O.set_threads(0)
    note("kh1024 x 100 oracle")
    R, rt, rs, re = O.evolve(p, U0, 2.0, 0.4, max_steps=100)
    note("kh1024 x 100 gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 2.0, 0.4, max_steps=100, mode="advance")
    assert rs[0] == gs[0] == 100 and ge[0] == 0 and gt[0] == rt[0]
    assert_parity(G, R, what="kh1024 x 100")


@pytest.mark.timeout(600)
def test_batch_of_1024_samples_sampled_against_oracle():
    """The batched configuration: 1024 samples of 256^2 (seed 1912), WENO3 + HLLC + SSP-RK3, 20
    steps in one launch per stage; samples 0, 1, 513 and 1023 against the oracle bit for bit
    (states, times, step counts)."""
    B, n, steps = 1024, 256, 20
    c, phi = fi.kh_coefficients(1912, np.arange(B))
    U0 = fi.kh2d_state(n, c, phi)
    p = _kh_problem(n)
    note("mc 1024 x 256^2 gpu")
    G, gt, gs, ge, st = gpu_evolve(p, U0, 10.0, 0.4, max_steps=steps, mode="advance")
    assert st == 0 and np.all(gs == steps) and np.all(ge == 0)
    pick = [0, 1, 513, 1023]
    O.set_threads(0)
    note("mc sampled oracle")
    R, rt, rs, re = O.evolve(p, U0[pick], 10.0, 0.4, max_steps=steps)
    assert np.array_equal(gs[pick], rs) and np.array_equal(gt[pick], rt)
    for i, b in enumerate(pick):
        assert_parity(G[b], R[i], what=f"sample {b}")


def _stats_batch(B, n):
    """A batch of 1024 states with every quantity varying: the Kelvin--Helmholtz initial data of
    seed 1912 with a vertical momentum 0.1 m_x sin(2 pi (x + 2 y)) (so v = 0.1 u sin(...))."""
    c, phi = fi.kh_coefficients(1912, np.arange(B))
    U = fi.kh2d_state(n, c, phi)
    x = (np.arange(n) + 0.5) / n
    wave = np.sin(2.0 * np.pi * (x[None, :] + 2.0 * x[:, None]))
    U[:, 2, 0] = 0.1 * U[:, 1, 0] * wave
    return U


@pytest.mark.timeout(600)
def test_statistics_of_the_full_batch_lag_32():
    """Per-cell Welford mean and variance of (rho, u, v, E) over 1024 samples of 256^2, and
    S_q(h) for h = 1..32 with its mean and variance over samples, against the oracle: mean and
    variance bit for bit, S^2 within 1e-12 (its spatial sums run in another order)."""
    torch = torch_gpu()
    from paper_1912_07645_amd import Stats
    B, n, H = 1024, 256, 32
    U = _stats_batch(B, n)
    p = _kh_problem(n)
    note("stats full batch gpu")
    st = Stats(solver_for(p), max_h=H)
    Ud = torch.from_numpy(U).cuda()
    st.accumulate(Ud[:300])
    st.accumulate(Ud[300:])
    out = st.read()
    del Ud
    O.set_threads(0)
    note("stats full batch oracle")
    ref = O.Stats(p, max_h=H)
    ref.accumulate(U)
    assert out["count"] == ref.n == B
    assert_parity(out["mean"].cpu().numpy(), ref.mean, what="mean")
    assert_parity(out["var"].cpu().numpy(), ref.variance(), what="var")
    assert_parity(out["s2_mean"].cpu().numpy(), ref.s2(), bitwise=False, what="S2 mean")
    assert_parity(out["s2_var"].cpu().numpy(), ref.s2_variance(), tol=1e-10, bitwise=False,
                  what="S2 var")


@pytest.mark.timeout(600)
def test_device_division_and_sqrt_on_1e8_inputs():
    """The device's '/' and sqrt equal the host's correctly rounded IEEE results on 10^8
    random inputs (uniform, log-uniform over the whole exponent range, subnormal numerators),
    in chunks of 10^7."""
    torch = torch_gpu()
    import paper_1912_07645_amd.fv as fv
    rng = np.random.default_rng(20250)
    chunk, total = 10_000_000, 100_000_000
    for k in range(total // chunk):
        kind = k % 3
        if kind == 0:
            a, b = rng.uniform(0, 10, chunk), rng.uniform(0.1, 10, chunk)
        elif kind == 1:
            a, b = np.exp(rng.uniform(-700, 700, chunk)), np.exp(rng.uniform(-700, 700, chunk))
        else:
            a, b = rng.uniform(0, 1, chunk) * 1e-308, rng.uniform(0.5, 4, chunk)
        A, Bt = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        q, r = torch.empty_like(A), torch.empty_like(A)
        fv.fv_check_arith(A, Bt, q, r)
        with np.errstate(over="ignore", under="ignore"):
            expect = a / b
        assert np.array_equal(q.cpu().numpy(), expect), k
        assert np.array_equal(r.cpu().numpy(), np.sqrt(a)), k
