"""Pins for the gradient oracle (oracle/adjoint_torch.py): its forward run equals the C
oracle bit for bit, its gradients agree with central finite differences of the C oracle, and
the initial-data derivative tables agree with finite differences of the input builder."""
import numpy as np
import pytest

import fv_inputs as fi
import oracle as O
from oracle import adjoint_torch as AT


def _problem(n, recon="muscl_minmod", integrator="ssprk3"):
    return O.Problem(dim=2, n=(n, n), eq="euler", flux="rusanov", recon=recon,
                     integrator=integrator)


@pytest.mark.parametrize("recon,integ", [("muscl_minmod", "ssprk3"), ("first_order", "forward_euler"),
                                         ("muscl_minmod", "ssprk2")])
def test_torch_forward_equals_c_oracle(recon, integ):
    n = 24
    U0 = fi.random_smooth_state(12, (1, n, n), 2, batch=2)
    p = _problem(n, recon, integ)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    R, err = O.evolve_fixed_dt(p, U0, dt, 7, 0.8)
    assert np.all(err == 0)
    import torch
    with torch.no_grad():
        U = torch.tensor(U0[:, :, 0])
        for _ in range(7):
            U = AT.ssprk3_step(U, dt, (float(n), float(n)), recon, integ)
    assert np.array_equal(U.numpy()[:, :, None], R)


def _qoi_c(p, n, U):
    yc = (np.arange(n) + 0.5) / n
    rows = np.nonzero(np.abs(yc - 0.5) < 0.1)[0]
    r, mx, my = U[:, 0, 0, rows], U[:, 1, 0, rows], U[:, 2, 0, rows]
    return (0.5 * (((mx * mx) + (my * my)) * (1.0 / r))).sum(axis=(1, 2)) * (1.0 / n) * (1.0 / n)


def test_gradient_against_central_differences_of_c_oracle():
    n, steps, eps = 32, 20, 1e-6
    c, phi = fi.kh_coefficients(1915, [0, 1])
    U0 = fi.kh2d_state(n, c, phi)
    p = _problem(n)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    Q, gc, gp = AT.qoi_and_gradient(c, phi, n, dt, steps, U0_values=U0)
    R, _ = O.evolve_fixed_dt(p, U0, dt, steps, 0.8)
    assert np.allclose(Q, _qoi_c(p, n, R), rtol=1e-13)
    g = np.concatenate([gc, gp], axis=1)
    fd = np.zeros_like(g)
    for k in range(20):
        cp, pp, cm, pm = c.copy(), phi.copy(), c.copy(), phi.copy()
        if k < 10:
            cp[:, k] += eps
            cm[:, k] -= eps
        else:
            pp[:, k - 10] += eps
            pm[:, k - 10] -= eps
        Qp = _qoi_c(p, n, O.evolve_fixed_dt(p, fi.kh2d_state(n, cp, pp), dt, steps, 0.8)[0])
        Qm = _qoi_c(p, n, O.evolve_fixed_dt(p, fi.kh2d_state(n, cm, pm), dt, steps, 0.8)[0])
        fd[:, k] = (Qp - Qm) / (2 * eps)
    # central differences carry a rounding error of about |Q| 1e-16 / eps per component
    rel = np.linalg.norm(g - fd, axis=1) / np.linalg.norm(fd, axis=1)
    assert np.all(rel < 2e-5), rel


def test_initial_data_jacobian_tables_against_finite_differences():
    n, eps = 32, 1e-7
    c, phi = fi.kh_coefficients(1915, [0, 1])
    U0, D, E = fi.kh2d_state_and_jacobian(n, c, phi)
    assert np.array_equal(U0, fi.kh2d_state(n, c, phi))
    for k in (0, 4, 9, 10, 15):
        cp, pp, cm, pm = c.copy(), phi.copy(), c.copy(), phi.copy()
        if k < 10:
            cp[:, k] += eps
            cm[:, k] -= eps
        else:
            pp[:, k - 10] += eps
            pm[:, k - 10] -= eps
        fd = (fi.kh2d_state(n, cp, pp) - fi.kh2d_state(n, cm, pm)) / (2 * eps)
        an = D * E[:, None, None, None, :, k]
        assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()


@pytest.mark.parametrize("recon,integ", [("muscl_minmod", "ssprk3"), ("first_order", "forward_euler"),
                                         ("muscl_minmod", "ssprk2")])
def test_reverse_mode_is_the_transpose_of_forward_mode(recon, integ):
    """Dot-product test: <lam, J v> from forward-mode differentiation (dual numbers) equals
    <J^T lam, v> from the reverse mode that the gradient oracle uses, for random v and lam,
    to rounding (the two modes evaluate different formulas for the same linear map)."""
    n, steps = 16, 4
    U0 = fi.random_smooth_state(3, (1, n, n), 2, batch=2)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(U0.shape)
    lam = rng.standard_normal(U0.shape)
    p = _problem(n, recon, integ)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    Jv = AT.jvp_steps(U0, v, n, dt, steps, recon, integ)
    JTl = AT.vjp_steps(U0, lam, n, dt, steps, recon, integ)
    for b in range(2):
        a, c = (lam[b] * Jv[b]).sum(), (JTl[b] * v[b]).sum()
        scale = np.abs(lam[b] * Jv[b]).sum()
        assert abs(a - c) <= 1e-13 * scale, (b, a, c)


def test_finite_difference_errors_come_with_branch_flips():
    """Kink audit of the gradient oracle against central differences (eps = 1e-6) of the forward
    run (which equals the C oracle bit for bit): the discrete map is only piecewise smooth
    (minmod branches, the larger Rusanov speed, |u|), so a difference quotient whose two runs
    take different branches somewhere need not approach the derivative. Every component whose
    two runs take the same branches everywhere agrees with the gradient to 1e-6 of the gradient
    norm (what remains is the rounding of the difference quotient); larger disagreements occur
    only where a branch flipped."""
    n, steps, eps = 32, 20, 1e-6
    c, phi = fi.kh_coefficients(1915, [0, 1])
    U0 = fi.kh2d_state(n, c, phi)
    p = _problem(n)
    M, _ = O.max_speed(p, U0[0])
    dt = 0.4 / M
    _, gc, gp = AT.qoi_and_gradient(c, phi, n, dt, steps, U0_values=U0)
    g = np.concatenate([gc, gp], axis=1)
    import torch
    fd = np.zeros_like(g)
    flips = np.zeros(g.shape, dtype=int)
    for k in range(20):
        cp, pp, cm, pm = c.copy(), phi.copy(), c.copy(), phi.copy()
        if k < 10:
            cp[:, k] += eps
            cm[:, k] -= eps
        else:
            pp[:, k - 10] += eps
            pm[:, k - 10] -= eps
        Up, rp = AT.forward_with_branches(fi.kh2d_state(n, cp, pp), n, dt, steps)
        Um, rm = AT.forward_with_branches(fi.kh2d_state(n, cm, pm), n, dt, steps)
        Qp = AT.qoi(torch.from_numpy(Up[:, :, 0]), n).numpy()
        Qm = AT.qoi(torch.from_numpy(Um[:, :, 0]), n).numpy()
        fd[:, k] = (Qp - Qm) / (2 * eps)
        for b in range(2):
            flips[b, k] = AT.branch_flips(rp, rm, b)
    err = np.abs(g - fd) / np.linalg.norm(fd, axis=1, keepdims=True)
    smooth = flips == 0
    assert smooth.sum() >= 30, smooth.sum()          # most pairs cross no switch at this size
    assert err[smooth].max() <= 1e-6, err[smooth].max()
    assert np.all(smooth | (err <= 1e-6) | (flips > 0))
    print("kink audit 32^2 x 20: %d of 40 components without a flip, max error %.1e; "
          "flipped components' errors %s" % (smooth.sum(), err[smooth].max(),
                                             np.array2string(err[~smooth], precision=1)))
