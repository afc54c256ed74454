"""Gradient oracle: the differentiated Kelvin--Helmholtz run written in plain PyTorch (CPU,
float64) and differentiated by autograd.

TEST INFRASTRUCTURE ONLY (used by the tests to check the GPU's hand-written discrete
adjoint). It never imports the GPU library.

The map theta -> Q is the definition of what the adjoint differentiates:
  theta = (c_1..c_10, phi_1..phi_10) -> delta(x_i) = a sum_k c_k sin(2 pi k x_i + phi_k)
  -> U0 (volume fraction of the band 0.25 + delta < y < 0.75 + delta)
  -> nsteps steps of size dt of the scheme of eq. (2.1): MUSCL-minmod reconstruction of the
     conserved variables, Rusanov flux, SSP-RK3 in increment form, periodic boundaries
  -> Q = dx dy sum over the rows |y_j - 0.5| < 0.1 of 0.5 |m|^2 / rho.
Every operation is written with the same operands and parentheses as the C oracle, so the
forward values equal it; autograd then applies the chain rule step by step. Kinks take the
branch the forward comparison selected (torch.where routes the gradient to the chosen
operand; d|u|/du = 0 at u = 0). The reverse sweep keeps every step's state and rebuilds one
step's graph at a time, so memory is the trajectory plus one step.
"""
from __future__ import annotations

import math

import numpy as np
import torch

GAMMA = 1.4


class _IEEESqrt(torch.autograd.Function):
    """Correctly rounded square root (NumPy's) with derivative 1 / (2 sqrt(x)); torch's CPU
    sqrt is not correctly rounded, and the forward values must equal the C oracle's."""

    @staticmethod
    def forward(x):
        return torch.from_numpy(np.sqrt(x.detach().numpy()))

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        return g / (2.0 * y)

    @staticmethod
    def jvp(ctx, dx):
        return dx / (2.0 * ctx.y_fwd)

    @staticmethod
    def setup_context(ctx, inputs, output):
        ctx.save_for_backward(output)
        ctx.y_fwd = output.detach()


def _sqrt(x):
    return _IEEESqrt.apply(x)


def _prim(U):
    r, mx, my, E = U[:, 0], U[:, 1], U[:, 2], U[:, 3]
    ir = 1.0 / r
    u = mx * ir
    v = my * ir
    ke = 0.5 * ((mx * u) + (my * v))
    gm1 = GAMMA - 1.0
    p = gm1 * (E - ke)
    c = _sqrt((GAMMA * p) * ir)
    return ir, u, v, p, c


def _flux(U, prim, d):
    ir, u, v, p, c = prim
    r, mx, my, E = U[:, 0], U[:, 1], U[:, 2], U[:, 3]
    if d == 0:
        return torch.stack([mx, (mx * u) + p, my * u, (E + p) * u], dim=1)
    return torch.stack([my, mx * v, (my * v) + p, (E + p) * v], dim=1)


def _vmax(a, b):
    return torch.where(a > b, a, b)


def _minmod(a, b):
    zero = torch.zeros_like(a)
    lo = torch.where(a < b, a, b)
    hi = torch.where(a > b, a, b)
    return torch.where((a > 0) & (b > 0), lo, torch.where((a < 0) & (b < 0), hi, zero))


def _rusanov(UL, UR, d):
    pl, pr = _prim(UL), _prim(UR)
    un_l = pl[1] if d == 0 else pl[2]
    un_r = pr[1] if d == 0 else pr[2]
    s = _vmax(torch.abs(un_l) + pl[4], torch.abs(un_r) + pr[4])
    FL, FR = _flux(UL, pl, d), _flux(UR, pr, d)
    return 0.5 * ((FL + FR) - (s[:, None] * (UR - UL)))


def rhs(U, inv_dx, recon="muscl_minmod"):
    """L(U) of eq. (2.1) for U[batch][4][ny][nx], periodic."""
    acc = None
    for d in (0, 1):
        ax = 3 if d == 0 else 2
        if recon == "muscl_minmod":
            Um = torch.roll(U, 1, dims=ax)
            Up = torch.roll(U, -1, dims=ax)
            sigma = _minmod(U - Um, Up - U)
            plus = U + (0.5 * sigma)          # value at i + 1/2 from cell i
            minus = U - (0.5 * sigma)         # value at i - 1/2 from cell i
        else:
            plus = U
            minus = U
        F = _rusanov(plus, torch.roll(minus, -1, dims=ax), d)   # flux at i + 1/2
        term = (F - torch.roll(F, 1, dims=ax)) * inv_dx[d]
        acc = term if acc is None else acc + term
    return -acc


BETAS = {"forward_euler": (1.0,), "ssprk2": (1.0, 0.5), "ssprk3": (1.0, 0.25, 2.0 / 3.0)}


def ssprk3_step(U, dt, inv_dx, recon="muscl_minmod", integrator="ssprk3"):
    Un = U
    Us = U
    for beta in BETAS[integrator]:
        Us = Un + (beta * ((Us - Un) + (dt * rhs(Us, inv_dx, recon))))
    return Us


def _reverse_steps(U, lam, dt, inv_dx, nsteps, recon, integrator):
    """(dU_T/dU)^T lam through nsteps steps from the tensor U: the states of every step are
    kept (no graph), then each step's graph is rebuilt from its state and differentiated,
    last step first (the chain rule of the step map, one step in memory at a time)."""
    states = [U]
    with torch.no_grad():
        for _ in range(nsteps - 1):
            states.append(ssprk3_step(states[-1], dt, inv_dx, recon, integrator))
    for Un in reversed(states):
        x = Un.detach().requires_grad_(True)
        y = ssprk3_step(x, dt, inv_dx, recon, integrator)
        (lam,) = torch.autograd.grad(y, x, grad_outputs=lam)
    return lam


def vjp_steps(U0, lamT, n, dt, nsteps, recon="muscl_minmod", integrator="ssprk3"):
    """dQ/dU0 for Q = <lamT, U_T>, U_T = nsteps steps from U0 (numpy [B][4][1][n][n])."""
    U = torch.tensor(np.asarray(U0)[:, :, 0], dtype=torch.float64)
    lam = torch.tensor(np.asarray(lamT)[:, :, 0], dtype=torch.float64)
    return _reverse_steps(U, lam, dt, (float(n), float(n)), nsteps, recon,
                          integrator).numpy()[:, :, None]


def jvp_steps(U0, v, n, dt, nsteps, recon="muscl_minmod", integrator="ssprk3"):
    """(dU_T/dU0) v by forward-mode differentiation (dual numbers through the same forward
    operations): the tangent that the reverse mode of vjp_steps transposes."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        U = fwAD.make_dual(torch.tensor(np.asarray(U0)[:, :, 0], dtype=torch.float64),
                           torch.tensor(np.asarray(v)[:, :, 0], dtype=torch.float64))
        for _ in range(nsteps):
            U = ssprk3_step(U, dt, (float(n), float(n)), recon, integrator)
        t = fwAD.unpack_dual(U).tangent
    return t.numpy()[:, :, None]


def stage_branches(U, inv_dx):
    """The branches the right-hand side of eq. (2.1) takes at state U (MUSCL-minmod + Rusanov),
    per axis: the minmod branch of every cell and field (0: zero, 1: the backward difference,
    2: the forward difference, as _minmod chooses), the side of the larger Rusanov speed of
    every face (1: left) and the sign of the normal velocity on that side."""
    out = []
    for d in (0, 1):
        ax = 3 if d == 0 else 2
        a = U - torch.roll(U, 1, dims=ax)
        b = torch.roll(U, -1, dims=ax) - U
        both_pos = (a > 0) & (b > 0)
        both_neg = (a < 0) & (b < 0)
        mm = torch.where(both_pos, torch.where(a < b, 1, 2),
                         torch.where(both_neg, torch.where(a > b, 1, 2), 0))
        sigma = _minmod(a, b)
        UL = U + (0.5 * sigma)
        UR = torch.roll(U - (0.5 * sigma), -1, dims=ax)
        pl, pr = _prim(UL), _prim(UR)
        ul = pl[1] if d == 0 else pl[2]
        ur = pr[1] if d == 0 else pr[2]
        left = (torch.abs(ul) + pl[4]) > (torch.abs(ur) + pr[4])
        sign = torch.sign(torch.where(left, ul, ur))
        out.append((mm.to(torch.int8), left.to(torch.int8), sign.to(torch.int8)))
    return out


def forward_with_branches(U0, n, dt, nsteps):
    """The SSP-RK3 forward run (numpy [B][4][1][n][n]) -> (U_T, branches), branches a list over
    (step, stage) of stage_branches at the stage's input state."""
    rec = []
    with torch.no_grad():
        U = torch.tensor(np.asarray(U0)[:, :, 0], dtype=torch.float64)
        for _ in range(nsteps):
            Un = U
            Us = U
            for beta in BETAS["ssprk3"]:
                rec.append(stage_branches(Us, (float(n), float(n))))
                Us = Un + (beta * ((Us - Un) + (dt * rhs(Us, (float(n), float(n))))))
            U = Us
    return U.numpy()[:, :, None], rec


def branch_flips(rec_a, rec_b, sample):
    """Number of (stage, axis, cell or face, field) branch choices of `sample` that differ
    between two recorded runs."""
    n = 0
    for sa, sb in zip(rec_a, rec_b):
        for xa, xb in zip(sa, sb):
            for ya, yb in zip(xa, xb):
                n += int((ya[sample] != yb[sample]).sum())
    return n


def initial_state(c, phi, n, a=0.01):
    """U0(theta) in torch (values as fv_inputs.kh2d_state up to the rounding of sin)."""
    x = (torch.arange(n, dtype=torch.float64) + 0.5) * (1.0 / n)
    delta = torch.zeros(c.shape[0], n, dtype=torch.float64)
    for k in range(c.shape[1]):
        delta = delta + c[:, k:k + 1] * torch.sin((2.0 * math.pi * (k + 1)) * x[None, :] + phi[:, k:k + 1])
    delta = a * delta
    dy = 1.0 / n
    yj = torch.arange(n, dtype=torch.float64)
    y_lo = (yj * dy)[None, :, None]
    y_hi = ((yj + 1.0) * dy)[None, :, None]
    i1 = 0.25 + delta[:, None, :]
    i2 = 0.75 + delta[:, None, :]
    raw = (torch.where(i2 < y_hi, i2, y_hi) - torch.where(i1 > y_lo, i1, y_lo)) * float(n)
    f = torch.where(raw > 1.0, torch.ones_like(raw), torch.where(raw < 0.0, torch.zeros_like(raw), raw))
    gm1 = GAMMA - 1.0

    def cons(rho, u):
        return [rho, rho * u, 0.0 * rho, 2.5 / gm1 + 0.5 * (rho * (u * u))]
    uin = cons(2.0, 0.5)
    uout = cons(1.0, -0.5)
    return torch.stack([uout[q] + f * (uin[q] - uout[q]) for q in range(4)], dim=1)


def qoi(U, n, band=0.1):
    """Kinetic energy times dx dy over the rows with |y_j - 0.5| < band."""
    yc = (np.arange(n) + 0.5) / n
    rows = np.nonzero(np.abs(yc - 0.5) < band)[0]
    j0, j1 = int(rows[0]), int(rows[-1]) + 1
    r, mx, my = U[:, 0, j0:j1], U[:, 1, j0:j1], U[:, 2, j0:j1]
    ke = 0.5 * (((mx * mx) + (my * my)) * (1.0 / r))
    return ke.sum(dim=(1, 2)) * ((1.0 / n) * (1.0 / n))


def qoi_and_gradient(c, phi, n, dt, nsteps, U0_values=None):
    """Q(theta) and dQ/dtheta for each sample (float64 numpy arrays c, phi [B][K]).

    U0_values (optional numpy [B][4][1][n][n]) replaces the forward values of the initial
    state (the derivative still comes from the torch initial data), so that the forward run
    starts from exactly the same numbers as the other implementations.
    Returns (Q [B], dQ/dc [B][K], dQ/dphi [B][K])."""
    ct = torch.tensor(c, dtype=torch.float64, requires_grad=True)
    pt = torch.tensor(phi, dtype=torch.float64, requires_grad=True)
    U = initial_state(ct, pt, n)
    if U0_values is not None:
        exact = torch.tensor(np.asarray(U0_values)[:, :, 0], dtype=torch.float64)
        U = U + (exact - U).detach()
    inv_dx = (float(n), float(n))
    with torch.no_grad():
        UT = U.detach()
        for _ in range(nsteps):
            UT = ssprk3_step(UT, dt, inv_dx)
    x = UT.requires_grad_(True)
    Q = qoi(x, n)
    (lamT,) = torch.autograd.grad(Q.sum(), x)
    lam0 = _reverse_steps(U.detach(), lamT, dt, inv_dx, nsteps, "muscl_minmod", "ssprk3")
    U.backward(lam0)
    return Q.detach().numpy(), ct.grad.numpy(), pt.grad.numpy()


def forward_only(U0, n, dt, nsteps):
    """The forward run on given initial values (numpy [B][4][1][n][n]) -> numpy."""
    with torch.no_grad():
        U = torch.tensor(np.asarray(U0)[:, :, 0], dtype=torch.float64)
        for _ in range(nsteps):
            U = ssprk3_step(U, dt, (float(n), float(n)))
    return U.numpy()[:, :, None]
