"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module builds initial data u_0 for the conservation law (1.1) and the random
perturbation coefficients of the Kelvin--Helmholtz shear layer (Section 3). It holds none
of the finite-volume scheme's arithmetic: no reconstruction, flux, divergence, time step or
statistic is computed here, only the initial states the scheme starts from.

Random numbers come from one counter-based generator, SplitMix64 (G. L. Steele, D. Lea,
C. H. Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014). Draw ``j`` of
sample ``s`` under seed ``seed`` is ``mix64(seed + G * (s * 64 + j + 1))`` with the golden
gamma ``G = 0x9E3779B97F4A7C15``; the top 53 bits give a uniform double in [0, 1).

Quasi-Monte Carlo sample points come from a Sobol sequence (I. M. Sobol', 1967) built here
from its definition: primitive polynomials over GF(2) enumerated by degree and value, unit
initial direction numbers m_1 = ... = m_s = 1 (odd and below 2^k, as the construction
requires), 32-bit direction numbers, and point n the XOR of the direction numbers of the set
bits of n; the first coordinate is the van der Corput sequence in base 2.

State layout (for every builder): float64, structure of arrays
``[batch][field][nz][ny][nx]`` with x fastest; Euler fields are (rho, m_x[, m_y[, m_z]], E).
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

__all__ = [
    "mix64", "uniform_draws", "kh_coefficients", "kh3d_coefficients", "kh_delta",
    "sod_state", "riemann_state_1d", "kh2d_state", "kh3d_state", "constant_state",
    "random_smooth_state", "sine_state_scalar", "cell_centres", "mlmc_inputs",
    "kh2d_state_and_jacobian", "primitive_polynomials", "sobol_points",
    "kh_coefficients_qmc", "swe_dam_break_1d", "swe_circular_dam_break", "random_smooth_swe",
]


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_draws(seed: int, samples, n_draws: int) -> np.ndarray:
    """Uniform doubles in [0,1): array [len(samples)][n_draws]; draw j of sample s."""
    samples = np.atleast_1d(np.asarray(samples, dtype=np.uint64))
    j = np.arange(n_draws, dtype=np.uint64)
    ctr = samples[:, None] * np.uint64(64) + j[None, :] + np.uint64(1)
    with np.errstate(over="ignore"):
        x = np.uint64(seed & MASK64) + np.uint64(GOLDEN_GAMMA) * ctr
    z = mix64(x)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def kh_coefficients(seed: int, samples, modes: int = 10):
    """Perturbation coefficients c_k ~ U[0,1), phi_k ~ U[0, 2 pi) for k = 1..modes.

    Returns (c, phi), each [len(samples)][modes]. c uses draws 0..modes-1 and phi draws
    modes..2*modes-1 of each sample.
    """
    u = uniform_draws(seed, samples, 2 * modes)
    return u[:, :modes].copy(), (2.0 * np.pi) * u[:, modes:]


def kh3d_coefficients(seed: int, samples, modes: int = 10):
    """Two independent sets (x and z modes) for the 3D shear layer: (cx, phix, cz, phiz)."""
    u = uniform_draws(seed, samples, 4 * modes)
    m = modes
    return (u[:, :m].copy(), (2.0 * np.pi) * u[:, m:2 * m],
            u[:, 2 * m:3 * m].copy(), (2.0 * np.pi) * u[:, 3 * m:4 * m])


def _gf2_mulmod(a: int, b: int, p: int, deg: int) -> int:
    """a * b modulo the polynomial p of degree deg, polynomials over GF(2) as bit masks."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> deg & 1:
            a ^= p
    return r


def _gf2_powmod(a: int, e: int, p: int, deg: int) -> int:
    r = 1
    while e:
        if e & 1:
            r = _gf2_mulmod(r, a, p, deg)
        a = _gf2_mulmod(a, a, p, deg)
        e >>= 1
    return r


def _prime_factors(n: int):
    out, f = [], 2
    while f * f <= n:
        if n % f == 0:
            out.append(f)
            while n % f == 0:
                n //= f
        f += 1
    if n > 1:
        out.append(n)
    return out


def primitive_polynomials(count: int):
    """The first `count` primitive polynomials over GF(2), by degree then value, as bit masks
    (bit k the coefficient of x^k): p is primitive iff x has multiplicative order 2^d - 1
    modulo p."""
    out, deg = [], 1
    while len(out) < count:
        order = (1 << deg) - 1
        for p in range((1 << deg) | 1, 1 << (deg + 1), 2):
            x = 2 % p if deg > 1 else 1          # the residue of x (x = 1 modulo x + 1)
            if _gf2_powmod(x, order, p, deg) != 1:
                continue
            if any(_gf2_powmod(x, order // r, p, deg) == 1 for r in _prime_factors(order) if r < order):
                continue
            out.append(p)
            if len(out) == count:
                break
        deg += 1
    return out


SOBOL_BITS = 32


def _sobol_directions(dim: int) -> np.ndarray:
    """Direction numbers V[j][k] (k = 0..31 for bit k + 1) of the first `dim` coordinates."""
    V = np.zeros((dim, SOBOL_BITS), dtype=np.uint64)
    for k in range(SOBOL_BITS):
        V[0, k] = 1 << (SOBOL_BITS - 1 - k)                   # van der Corput
    polys = primitive_polynomials(max(dim - 1, 0))
    for j in range(1, dim):
        p = polys[j - 1]
        s = p.bit_length() - 1                                 # degree
        a = [(p >> (s - i)) & 1 for i in range(1, s)]          # a_1 .. a_{s-1}
        m = [1] * s                                            # unit initial numbers
        for k in range(s, SOBOL_BITS):
            v = m[k - s] ^ (m[k - s] << s)
            for i in range(1, s):
                if a[i - 1]:
                    v ^= m[k - i] << i
            m.append(v)
        for k in range(SOBOL_BITS):
            V[j, k] = m[k] << (SOBOL_BITS - 1 - k)
    return V


def sobol_points(n: int, dim: int, skip: int = 0) -> np.ndarray:
    """Points skip .. skip + n - 1 of the dim-dimensional Sobol sequence: float64 [n][dim] in
    [0, 1), multiples of 2^-32."""
    V = _sobol_directions(dim)
    idx = np.arange(skip, skip + n, dtype=np.uint64)
    X = np.zeros((n, dim), dtype=np.uint64)
    for k in range(SOBOL_BITS):
        bit = ((idx >> np.uint64(k)) & np.uint64(1)).astype(bool)
        X[bit] ^= V[:, k]
    return X.astype(np.float64) * 2.0 ** -SOBOL_BITS


def kh_coefficients_qmc(samples, modes: int = 10, skip: int = 1):
    """Quasi-Monte Carlo counterpart of kh_coefficients: sample s takes Sobol point
    s + skip (point 0 is the origin) of dimension 2 * modes; c_k is coordinate k - 1 and
    phi_k = 2 pi times coordinate modes + k - 1."""
    samples = np.asarray(samples, dtype=np.int64)
    pts = sobol_points(int(samples.max()) + 1, 2 * modes, skip=skip)[samples]
    return pts[:, :modes].copy(), 2.0 * np.pi * pts[:, modes:]


def cell_centres(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * ((hi - lo) / n)


def kh_delta(c: np.ndarray, phi: np.ndarray, x: np.ndarray, a: float = 0.01) -> np.ndarray:
    """Interface displacement delta(x) = a * sum_k c_k sin(2 pi k x + phi_k), summed k = 1.. in order.

    c, phi: [batch][modes]; x: [nx]. Returns [batch][nx].
    """
    c = np.atleast_2d(c)
    phi = np.atleast_2d(phi)
    acc = np.zeros((c.shape[0], x.shape[0]), dtype=np.float64)
    for k in range(c.shape[1]):
        acc = acc + c[:, k:k + 1] * np.sin((2.0 * np.pi * (k + 1)) * x[None, :] + phi[:, k:k + 1])
    return a * acc


def _euler_conserved(rho, u, v, w, p, gamma, dim):
    gm1 = gamma - 1.0
    if dim == 1:
        ke = 0.5 * (rho * (u * u))
        return [rho, rho * u, p / gm1 + ke]
    if dim == 2:
        ke = 0.5 * (rho * (u * u + v * v))
        return [rho, rho * u, rho * v, p / gm1 + ke]
    ke = 0.5 * (rho * (u * u + v * v + w * w))
    return [rho, rho * u, rho * v, rho * w, p / gm1 + ke]


def riemann_state_1d(n: int, left, right, gamma: float = 1.4, x0: float = 0.5) -> np.ndarray:
    """1D Euler Riemann initial data: primitive (rho, u, p) left/right of x0. [1][3][1][1][n]."""
    x = cell_centres(n)
    lf = x < x0
    rho = np.where(lf, left[0], right[0])
    u = np.where(lf, left[1], right[1])
    p = np.where(lf, left[2], right[2])
    f = _euler_conserved(rho, u, None, None, p, gamma, 1)
    return np.stack(f)[None, :, None, None, :].astype(np.float64)


def sod_state(n: int = 1024, gamma: float = 1.4) -> np.ndarray:
    """Sod shock tube on [0,1]: (1, 0, 1) | (0.125, 0, 0.1) split at x = 0.5."""
    return riemann_state_1d(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma)


def _band_fraction(y_lo, y_hi, i1, i2, inv_dy):
    """Fraction of the cell [y_lo, y_hi] inside the band (i1, i2) (volume fraction)."""
    f = (np.minimum(y_hi, i2) - np.maximum(y_lo, i1)) * inv_dy
    return np.minimum(1.0, np.maximum(0.0, f))


def kh2d_state(n: int, c: np.ndarray, phi: np.ndarray, gamma: float = 1.4, a: float = 0.01,
               ny: int | None = None) -> np.ndarray:
    """2D Kelvin--Helmholtz shear layer on the periodic unit square.

    p = 2.5 and v = 0 everywhere; rho = 2, u = 0.5 inside the band 0.25 + delta(x) < y <
    0.75 + delta(x), rho = 1, u = -0.5 outside. Each cell takes the conserved state
    U_out + f (U_in - U_out), with f the fraction of its y-extent (at the x-centre) inside the
    band. Returns [batch][4][1][ny][nx].
    """
    nx = n
    ny = n if ny is None else ny
    c = np.atleast_2d(c)
    phi = np.atleast_2d(phi)
    xc = cell_centres(nx)
    dy = 1.0 / ny
    yj = np.arange(ny, dtype=np.float64)
    y_lo = (yj * dy)[None, :, None]
    y_hi = ((yj + 1.0) * dy)[None, :, None]
    delta = kh_delta(c, phi, xc, a)[:, None, :]          # [b][1][nx]
    f = _band_fraction(y_lo, y_hi, 0.25 + delta, 0.75 + delta, float(ny))  # [b][ny][nx]
    uin = _euler_conserved(2.0, 0.5, 0.0, 0.0, 2.5, gamma, 2)
    uout = _euler_conserved(1.0, -0.5, 0.0, 0.0, 2.5, gamma, 2)
    out = np.empty((c.shape[0], 4, 1, ny, nx), dtype=np.float64)
    for q in range(4):
        out[:, q, 0] = uout[q] + f * (uin[q] - uout[q])
    return out


def kh3d_state(n: int, cx, phix, cz, phiz, gamma: float = 1.4, a: float = 0.01) -> np.ndarray:
    """3D shear layer in y on the periodic unit cube, interface delta(x) + delta(z), w = 0.

    Returns [batch][5][n][n][n]. Built one z-plane at a time to bound host memory.
    """
    cx = np.atleast_2d(cx)
    b = cx.shape[0]
    xc = cell_centres(n)
    dx_ = kh_delta(cx, phix, xc, a)          # [b][n] over x
    dz_ = kh_delta(cz, phiz, xc, a)          # [b][n] over z
    dy = 1.0 / n
    yj = np.arange(n, dtype=np.float64)
    y_lo = (yj * dy)[:, None]
    y_hi = ((yj + 1.0) * dy)[:, None]
    uin = _euler_conserved(2.0, 0.5, 0.0, 0.0, 2.5, gamma, 3)
    uout = _euler_conserved(1.0, -0.5, 0.0, 0.0, 2.5, gamma, 3)
    out = np.empty((b, 5, n, n, n), dtype=np.float64)
    for s in range(b):
        for k in range(n):
            delta = (dx_[s] + dz_[s, k])[None, :]
            f = _band_fraction(y_lo, y_hi, 0.25 + delta, 0.75 + delta, float(n))
            for q in range(5):
                out[s, q, k] = uout[q] + f * (uin[q] - uout[q])
    return out


def swe_dam_break_1d(n: int, hL: float = 2.0, hR: float = 1.0, x0: float = 0.5) -> np.ndarray:
    """Shallow-water dam break on [0, 1]: depth hL left of x0, hR right of it, at rest.
    Fields (h, hu): [1][2][1][1][n]."""
    x = cell_centres(n)
    U = np.zeros((1, 2, 1, 1, n))
    U[0, 0, 0, 0] = np.where(x < x0, hL, hR)
    return U


def swe_circular_dam_break(n: int, h_in: float = 2.0, h_out: float = 1.0, r0: float = 0.2,
                           batch: int = 1) -> np.ndarray:
    """Shallow water on the periodic unit square: depth h_in inside the circle of radius r0
    about the centre (cell centres decide), h_out outside, at rest. Fields (h, hu, hv):
    [batch][3][1][n][n]."""
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    h = np.where((X - 0.5) ** 2 + (Y - 0.5) ** 2 < r0 * r0, h_in, h_out)
    U = np.zeros((batch, 3, 1, n, n))
    U[:, 0, 0] = h
    return U


def random_smooth_swe(seed: int, shape_cells, dim: int, batch: int = 1) -> np.ndarray:
    """Smooth periodic shallow-water data: h = 1 + 0.2 (low Fourier modes, |.| < 1) and
    velocities of size 0.3, as (h, hu[, hv]) [batch][dim + 1][nz][ny][nx]."""
    E = random_smooth_state(seed, shape_cells, dim, batch=batch)
    rho = E[:, 0]
    h = 1.0 + 0.2 * (rho - rho.mean()) / (np.abs(rho - rho.mean()).max() + 1e-300)
    U = np.zeros((batch, dim + 1) + tuple(shape_cells))
    U[:, 0] = h
    for k in range(dim):
        vel = E[:, 1 + k] / rho
        U[:, 1 + k] = h * 0.3 * vel / (np.abs(vel).max() + 1e-300)
    return U


def mhd_conserved(rho, u, p, B, gamma: float) -> np.ndarray:
    """Ideal-MHD conserved fields (rho, m_x, m_y, m_z, E, B_x, B_y, B_z) from density, three
    velocity components, pressure and three field components (arrays of one shape), with
    E = p/(gamma - 1) + rho |u|^2 / 2 + |B|^2 / 2."""
    u = [np.asarray(c, dtype=np.float64) for c in u]
    B = [np.asarray(c, dtype=np.float64) for c in B]
    rho = np.asarray(rho, dtype=np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) \
        + 0.5 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], E, B[0], B[1], B[2]])


def orszag_tang_state(n: int, gamma: float = 5.0 / 3.0) -> np.ndarray:
    """The Orszag--Tang vortex on the periodic unit square, n x n cells, sampled at cell
    centres: rho = gamma^2, p = gamma, u = (-sin 2 pi y, sin 2 pi x, 0),
    B = (-sin 2 pi y, sin 4 pi x, 0). Returns [1][8][1][n][n]."""
    x = cell_centres(n)[None, :]
    y = cell_centres(n)[:, None]
    one = np.ones((n, n))
    U = mhd_conserved(gamma * gamma * one, [-np.sin(2 * np.pi * y) * one, np.sin(2 * np.pi * x) * one, 0 * one],
                      gamma * one, [-np.sin(2 * np.pi * y) * one, np.sin(4 * np.pi * x) * one, 0 * one], gamma)
    return U[None, :, None]


def brio_wu_state(n: int, gamma: float = 2.0) -> np.ndarray:
    """The Brio--Wu shock tube: rho, p, B_y = (1, 1, 1) left of x = 1/2 and (0.125, 0.1, -1)
    right, B_x = 0.75, at rest. Returns [1][8][1][1][n]."""
    x = cell_centres(n)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros(n)
    U = mhd_conserved(rho, [z, z, z], p, [0.75 + z, np.where(left, 1.0, -1.0), z], gamma)
    return U[None, :, None, None]


def alfven_wave_average(n: int, t: float, amp: float = 0.1, p0: float = 0.1,
                        gamma: float = 5.0 / 3.0) -> np.ndarray:
    """Cell averages at time t of the circularly polarised Alfven wave along x (rho = 1,
    B_x = 1, so the Alfven speed is 1): B_y = amp sin 2 pi (x - t), B_z = amp cos 2 pi (x - t),
    u_y = -B_y, u_z = -B_z, u_x = 0, p = p0. Each sinusoid's cell average is its centre value
    times sin(pi dx) / (pi dx); the energy is constant. Returns [1][8][1][1][n]."""
    x = cell_centres(n)
    k = np.sin(np.pi / n) / (np.pi / n)
    sy = amp * k * np.sin(2 * np.pi * (x - t))
    sz = amp * k * np.cos(2 * np.pi * (x - t))
    one = np.ones(n)
    E = p0 / (gamma - 1.0) + 0.5 * amp * amp + 0.5 * (1.0 + amp * amp)
    U = np.stack([one, 0 * one, -sy, -sz, E * one, one, sy, sz])
    return U[None, :, None, None]


def random_smooth_mhd(seed: int, shape_cells, dim: int, batch: int = 1,
                      gamma: float = 5.0 / 3.0) -> np.ndarray:
    """Smooth periodic MHD data [batch][8][nz][ny][nx]: density, the velocity components and
    pressure from random_smooth_state (the components beyond dim from a second draw), and a
    field B of size about 0.6 from a third draw's velocities."""
    E1 = random_smooth_state(seed, shape_cells, 3, batch=batch, gamma=gamma)
    E2 = random_smooth_state(seed + 7919, shape_cells, 3, batch=batch, gamma=gamma)
    rho = E1[:, 0]
    u = [E1[:, 1 + k] / rho for k in range(3)]
    ke = 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    p = (gamma - 1.0) * (E1[:, 4] - ke)
    B = [0.5 * E2[:, 1 + k] / E2[:, 0] + 0.2 * (k + 1) for k in range(3)]
    out = np.stack([mhd_conserved(rho[b], [c[b] for c in u], p[b], [c[b] for c in B], gamma)
                    for b in range(batch)])
    return np.ascontiguousarray(out)


def constant_state(shape_cells, values, batch: int = 1) -> np.ndarray:
    """Every cell equal to ``values`` (one per field). shape_cells = (nz, ny, nx)."""
    nz, ny, nx = shape_cells
    vals = np.asarray(values, dtype=np.float64)
    out = np.empty((batch, vals.size, nz, ny, nx), dtype=np.float64)
    out[:] = vals[None, :, None, None, None]
    return out


def random_smooth_state(seed: int, shape_cells, dim: int, batch: int = 1, gamma: float = 1.4,
                        amp: float = 0.1, modes: int = 3) -> np.ndarray:
    """Smooth periodic Euler data: rho, u, v, w, p each a sum of random low Fourier modes.

    rho and p stay within 1 +- amp*modes, so the data is physical for amp*modes < 1. The
    velocities have amplitude 4*amp*modes, enough to make wave speeds of both signs appear
    at faces. Used for short parity runs that exercise every branch of the fluxes.
    """
    nz, ny, nx = shape_cells
    z = np.arange(nz, dtype=np.float64)[:, None, None] / nz
    y = np.arange(ny, dtype=np.float64)[None, :, None] / ny
    x = np.arange(nx, dtype=np.float64)[None, None, :] / nx
    per = 5 * modes * 2
    draws = uniform_draws(seed, np.arange(batch), per)
    out = np.empty((batch, dim + 2, nz, ny, nx), dtype=np.float64)
    for s in range(batch):
        fields = []
        for v in range(5):
            acc = np.zeros((nz, ny, nx))
            for m in range(modes):
                a_m, ph = draws[s, 2 * (v * modes + m)], draws[s, 2 * (v * modes + m) + 1]
                k = m + 1
                arg = k * x + (k * y if dim >= 2 else 0.0) + (k * z if dim == 3 else 0.0)
                acc = acc + (2.0 * a_m - 1.0) * np.sin(2.0 * np.pi * (arg + ph))
            fields.append(amp * acc)
        rho = 1.0 + fields[0]
        p = 1.0 + fields[4]
        u, v_, w = 4.0 * fields[1], 4.0 * fields[2], 4.0 * fields[3]
        out[s] = np.stack(_euler_conserved(rho, u, v_, w, p, gamma, dim))
    return out


def sine_state_scalar(n: int, k: int = 1, amp: float = 1.0, offset: float = 0.0,
                      dim: int = 1) -> np.ndarray:
    """Scalar u(x) = offset + amp sin(2 pi k x) at cell centres, constant in y and z."""
    x = cell_centres(n)
    u = offset + amp * np.sin(2.0 * np.pi * k * x)
    if dim == 1:
        return u[None, None, None, None, :].copy()
    if dim == 2:
        return np.broadcast_to(u[None, None, None, None, :], (1, 1, 1, n, n)).copy()
    return np.broadcast_to(u[None, None, None, None, :], (1, 1, n, n, n)).copy()


def mlmc_inputs(ns, Ms, seed: int = 1913, gamma: float = 1.4):
    """Initial states of a multilevel Kelvin--Helmholtz run, one array per grid ("group").

    Level l (grid ns[l], Ms[l] samples) draws the coefficients of samples
    offset_l .. offset_l + Ms[l] - 1, offset_l = Ms[0] + ... + Ms[l-1]. Group l holds level l's
    samples on grid ns[l], followed by level l+1's samples (the same coefficients) on grid ns[l]
    as the coarse partners of the coupled pairs.
    """
    offs = np.concatenate([[0], np.cumsum(Ms)]).astype(np.int64)
    groups = []
    for l, n in enumerate(ns):
        ids = list(range(offs[l], offs[l] + Ms[l]))
        if l + 1 < len(ns):
            ids += list(range(offs[l + 1], offs[l + 1] + Ms[l + 1]))
        c, phi = kh_coefficients(seed, np.array(ids, dtype=np.int64))
        groups.append(kh2d_state(n, c, phi, gamma))
    return groups


def kh2d_state_and_jacobian(n: int, c: np.ndarray, phi: np.ndarray, gamma: float = 1.4,
                            a: float = 0.01):
    """The 2D Kelvin--Helmholtz initial state together with its derivative tables.

    The state depends on the coefficients theta = (c_1..c_K, phi_1..phi_K) only through the
    interface displacement delta(x_i) of each column i. Returns (U0, D, E):
      U0 [b][4][1][n][n]   the state (as kh2d_state);
      D  [b][4][1][n][n]   dU0/d delta(x_i) for the cell's own column (nonzero only in the
                           cells the two interfaces cross: df/d delta = +-1/dy there);
      E  [b][n][2K]        d delta(x_i)/d theta_k: a sin(2 pi k x + phi_k) for c_k and
                           a c_k cos(2 pi k x + phi_k) for phi_k.
    """
    c = np.atleast_2d(c)
    phi = np.atleast_2d(phi)
    U0 = kh2d_state(n, c, phi, gamma, a)
    B, K = c.shape
    xc = cell_centres(n)
    dy = 1.0 / n
    yj = np.arange(n, dtype=np.float64)
    y_lo = (yj * dy)[None, :, None]
    y_hi = ((yj + 1.0) * dy)[None, :, None]
    delta = kh_delta(c, phi, xc, a)[:, None, :]
    i1 = 0.25 + delta
    i2 = 0.75 + delta
    raw = (np.minimum(y_hi, i2) - np.maximum(y_lo, i1)) * float(n)
    draw = (np.where(i2 < y_hi, 1.0, 0.0) - np.where(i1 > y_lo, 1.0, 0.0)) * float(n)
    dfd = np.where((raw > 0.0) & (raw < 1.0), draw, 0.0)          # [b][ny][nx]
    uin = _euler_conserved(2.0, 0.5, 0.0, 0.0, 2.5, gamma, 2)
    uout = _euler_conserved(1.0, -0.5, 0.0, 0.0, 2.5, gamma, 2)
    D = np.empty_like(U0)
    for q in range(4):
        D[:, q, 0] = dfd * (uin[q] - uout[q])
    E = np.empty((B, n, 2 * K), dtype=np.float64)
    for k in range(K):
        arg = (2.0 * np.pi * (k + 1)) * xc[None, :] + phi[:, k:k + 1]
        E[:, :, k] = a * np.sin(arg)
        E[:, :, K + k] = a * c[:, k:k + 1] * np.cos(arg)
    return U0, D, E
