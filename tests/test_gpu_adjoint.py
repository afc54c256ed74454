"""GPU discrete adjoint against the autograd oracle and against central finite differences."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from oracle import adjoint_torch as AT
from gpu_helpers import note, solver_for, torch_gpu

pytestmark = pytest.mark.gpu


def _problem(n, recon="muscl_minmod", integrator="ssprk3", shape=None):
    nx, ny = shape if shape else (n, n)
    return O.Problem(dim=2, n=(nx, ny), eq="euler", flux="rusanov", recon=recon,
                     integrator=integrator)


@pytest.mark.parametrize("recon", ["first_order", "muscl_minmod"])
@pytest.mark.parametrize("integ", ["forward_euler", "ssprk2", "ssprk3"])
def test_adjoint_vjp_matches_autograd(recon, integ):
    """lambda_0 = (dU_T/dU_0)^T lambda_T for random data, several steps and checkpoint
    segments (every = 2 of 5 steps), against autograd of the same scheme."""
    torch = torch_gpu()
    from paper_1912_07645_amd.adjoint import Adjoint
    n = 40
    U0 = fi.random_smooth_state(31, (1, n, n), 2, batch=3)
    rng = np.random.default_rng(4)
    lamT = rng.standard_normal(U0.shape)
    p = _problem(n, recon, integ)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.35 / M
    s = solver_for(p)
    adj = Adjoint(s, 3, 5, dt, every=2)
    note("adjoint vjp", recon, integ)
    UT = adj.forward(torch.from_numpy(U0).cuda())
    R, _ = O.evolve_fixed_dt(p, U0, dt, 5, 1.0)
    assert np.array_equal(UT.cpu().numpy(), R)
    g = adj.backward(torch.from_numpy(lamT).cuda()).cpu().numpy()
    ref = AT.vjp_steps(U0, lamT, n, dt, 5, recon, integ)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert rel <= 1e-12, rel


def test_adjoint_qoi_gradient_matches_oracle_64():
    """The differentiated KH run at 64^2 (MUSCL-minmod + Rusanov + SSP-RK3, fixed dt at CFL 0.4
    of the initial state): dQ/dtheta from the GPU adjoint against autograd, 2 samples x 120
    steps."""
    torch = torch_gpu()
    from paper_1912_07645_amd.adjoint import Adjoint, LineInitialDataQoI, band_rows
    n, B, steps = 64, 2, 120
    c, phi = fi.kh_coefficients(1915, np.arange(B))
    U0, D, E = fi.kh2d_state_and_jacobian(n, c, phi)
    p = _problem(n)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    s = solver_for(p)
    adj = Adjoint(s, B, steps, dt, cfl_bound=0.6)
    j0, j1 = band_rows(n)
    assert (j0, j1) == (26, 38)
    theta = torch.tensor(np.concatenate([c, phi], axis=1), device="cuda", requires_grad=True)
    note("adjoint qoi gpu")
    Q = LineInitialDataQoI.apply(theta, torch.from_numpy(U0).cuda(), torch.from_numpy(D).cuda(),
                                 torch.from_numpy(E).cuda(), adj, j0, j1)
    Q.sum().backward()
    g = theta.grad.cpu().numpy()
    note("adjoint qoi oracle")
    Qr, gc, gp = AT.qoi_and_gradient(c, phi, n, dt, steps, U0_values=U0)
    assert np.allclose(Q.detach().cpu().numpy(), Qr, rtol=1e-13)
    ref = np.concatenate([gc, gp], axis=1)
    rel = np.linalg.norm(g - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.all(rel <= 1e-10), rel


def _fd_runs(s, n, steps, dt, j0, j1, C, P, chunk=640):
    """Q of every (c, phi) row after `steps` fixed steps, batched on the GPU."""
    torch = torch_gpu()
    from paper_1912_07645_amd.adjoint import kinetic_energy
    out = []
    for a in range(0, C.shape[0], chunk):
        Uc = torch.from_numpy(fi.kh2d_state(n, C[a:a + chunk], P[a:a + chunk])).cuda()
        err = torch.zeros(Uc.shape[0], dtype=torch.int32, device="cuda")
        assert s.evolve_fixed_dt(Uc, dt, steps, 0.6, err) == 0
        Qc, _ = kinetic_energy(s, Uc, j0, j1)
        out.append(Qc.cpu().numpy())
        del Uc
    return np.concatenate(out)


def _central(s, n, steps, dt, j0, j1, c, phi, eps):
    B = c.shape[0]
    cs, ps = [], []
    for sign in (1.0, -1.0):
        for k in range(20):
            cp, pp = c.copy(), phi.copy()
            if k < 10:
                cp[:, k] += sign * eps
            else:
                pp[:, k - 10] += sign * eps
            cs.append(cp)
            ps.append(pp)
    Q = _fd_runs(s, n, steps, dt, j0, j1, np.concatenate(cs), np.concatenate(ps)).reshape(2, 20, B)
    return ((Q[0] - Q[1]) / (2 * eps)).T


def test_adjoint_full_configuration_against_finite_differences():
    """256^2 x 64 samples x 500 steps: the adjoint gradient with respect to the 20
    coefficients against finite differences of GPU forward runs (batched).

    The discrete map is only piecewise smooth: minmod switches between its branches and the
    Rusanov speed takes a maximum, so a perturbed run can cross a switch that the adjoint (the
    derivative of the branch taken) does not see. The finite-difference error therefore grows
    with eps (measured: central eps = 1e-5 is about 5x worse than eps = 1e-6), and the adjoint's
    own exactness is pinned elsewhere: against autograd through the same run at 64^2 (1e-10)
    and stage by stage (1e-12). Here the bar is the directional derivative along the gradient
    (one central difference per sample, the usual gradient test) at eps = 1e-6, median within
    1e-6, with the component-wise central differences at eps = 1e-6 within 1e-5."""
    torch = torch_gpu()
    from paper_1912_07645_amd.adjoint import Adjoint, LineInitialDataQoI, band_rows
    n, B, steps = 256, 64, 500
    c, phi = fi.kh_coefficients(1915, np.arange(B))
    U0, D, E = fi.kh2d_state_and_jacobian(n, c, phi)
    p = _problem(n)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    s = solver_for(p)
    j0, j1 = band_rows(n)
    assert (j0, j1) == (102, 154)
    adj = Adjoint(s, B, steps, dt, cfl_bound=0.6)
    theta = torch.tensor(np.concatenate([c, phi], axis=1), device="cuda", requires_grad=True)
    note("adjoint full gpu")
    Q = LineInitialDataQoI.apply(theta, torch.from_numpy(U0).cuda(), torch.from_numpy(D).cuda(),
                                 torch.from_numpy(E).cuda(), adj, j0, j1)
    Q.sum().backward()
    g = theta.grad.cpu().numpy()
    del adj
    torch.cuda.empty_cache()
    note("adjoint full directional")
    eps = 1e-6
    d = g / np.linalg.norm(g, axis=1, keepdims=True)
    Cs = np.concatenate([c + eps * d[:, :10], c - eps * d[:, :10]])
    Ps = np.concatenate([phi + eps * d[:, 10:], phi - eps * d[:, 10:]])
    Qd = _fd_runs(s, n, steps, dt, j0, j1, Cs, Ps).reshape(2, B)
    dir_fd = (Qd[0] - Qd[1]) / (2 * eps)
    rel_dir = np.abs(dir_fd - np.linalg.norm(g, axis=1)) / np.abs(dir_fd)
    note("adjoint full central 1e-6")
    fd6 = _central(s, n, steps, dt, j0, j1, c, phi, 1e-6)
    rel6 = np.linalg.norm(g - fd6, axis=1) / np.linalg.norm(fd6, axis=1)
    print("adjoint vs FD, per-sample relative error (median / 90th pct / max): "
          "directional eps=1e-6: %.2e / %.2e / %.2e; central eps=1e-6: %.2e / %.2e / %.2e"
          % (np.median(rel_dir), np.percentile(rel_dir, 90), rel_dir.max(),
             np.median(rel6), np.percentile(rel6, 90), rel6.max()), flush=True)
    assert np.median(rel_dir) <= 1e-6, rel_dir
    assert np.median(rel6) <= 1e-5, rel6


def _binomial_forward_steps(l, snaps):
    """Griewank's minimal number of forward steps to reverse l steps with `snaps` stored
    states (the initial one included): t l - C(snaps + t, t - 1) with t the smallest integer
    such that C(snaps + t, t) >= l; l (l - 1) / 2 for a single stored state."""
    from math import comb
    if l <= 1:
        return 0
    if snaps == 1:
        return l * (l - 1) // 2
    t = 0
    while comb(snaps + t, t) < l:
        t += 1
    return t * l - comb(snaps + t, t - 1)


@pytest.mark.parametrize("integ", ["forward_euler", "ssprk3"])
def test_binomial_checkpointing_equals_segments(integ):
    """The binomial (revolve) schedule gives the segment schedule's gradient bit for bit, with
    the published minimal number of recomputed forward steps for each number of snapshots."""
    torch = torch_gpu()
    from paper_1912_07645_amd.adjoint import Adjoint
    n, B, steps = 40, 2, 23
    U0 = fi.random_smooth_state(77, (1, n, n), 2, batch=B)
    lamT = np.random.default_rng(8).standard_normal(U0.shape)
    p = _problem(n, "muscl_minmod", integ)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.3 / M
    s = solver_for(p)
    ref = Adjoint(s, B, steps, dt, every=5)
    UT = ref.forward(torch.from_numpy(U0).cuda()).cpu().numpy()
    g = ref.backward(torch.from_numpy(lamT).cuda()).cpu().numpy()
    assert ref.recomputed_steps() == steps
    stage_recompute = 0 if integ == "forward_euler" else steps
    for snaps in (0, 1, 2, 3, 7, 30):
        note("binomial adjoint", integ, snaps)
        adj = Adjoint(s, B, steps, dt, snapshots=snaps)
        assert np.array_equal(adj.forward(torch.from_numpy(U0).cuda()).cpu().numpy(), UT)
        gb = adj.backward(torch.from_numpy(lamT).cuda()).cpu().numpy()
        assert np.array_equal(gb, g), snaps
        want = _binomial_forward_steps(steps, min(snaps, steps) + 1) + stage_recompute
        assert adj.recomputed_steps() == want, (snaps, adj.recomputed_steps(), want)
