"""Pins of the oracle's point and joint PDFs and shell structure functions (the statistics
that Section 2.2 names after Fjordholm, Lye and Mishra, read as stated in the oracle's
header): hand-counted histograms, the rounding edge of the bin rule, marginals, closed forms
of the shell sums for a sine and a checkerboard, a brute-force shell sum written with numpy
rolls, and the radius-1 ball against the axis structure function."""
import math

import numpy as np
import pytest

import oracle as O


def _rho_state(values, dim=1, n=(4,)):
    """Euler states whose density at cell 0 takes the given values, one sample each (the
    other fields are 1, so rho is the only quantity that changes)."""
    p = O.Problem(dim=dim, n=n, eq="euler")
    U = np.ones((len(values),) + p.state_shape)
    U[:, 0].reshape(len(values), -1)[:, 0] = values
    return p, U


def test_point_pdf_hand_counted():
    # lo = 0, hi = 1, 4 bins of width 1/4; bin k = floor(v * 4)
    vals = [-0.5, 0.0, 0.25, 0.49, 0.5, 0.999, 1.0, float("nan")]
    p, U = _rho_state(vals)
    c = O.point_pdf(p, U, 0, [0, 1], 0.0, 1.0, 4)
    # -0.5 below; 0.0 -> 0; 0.25 -> 1; 0.49 -> 1; 0.5 -> 2; 0.999 -> 3; 1.0 and NaN above
    assert c[0].tolist() == [1, 2, 1, 1, 1, 2]
    # cell 1 keeps rho = 1 = hi in every sample: all above
    assert c[1].tolist() == [0, 0, 0, 0, 0, 8]


def test_point_pdf_rounding_edge_stays_in_last_bin():
    # (v - 0.2) / (0.9 - 0.2) rounds to exactly 1.0 for the largest double below 0.9, so
    # floor(1.0 * nbins) = nbins; the value is inside [lo, hi) and goes to the last bin
    v = float(np.nextafter(0.9, 0.0))
    assert ((v - 0.2) / (0.9 - 0.2)) == 1.0
    p, U = _rho_state([v])
    for nb in (1, 3, 8):
        c = O.point_pdf(p, U, 0, [0], 0.2, 0.9, nb)
        assert c[0, nb - 1] == 1 and c[0].sum() == 1


def test_point_pdf_velocity_uses_m_over_rho():
    # u = m * (1 / rho): rho = 4, m = 3 gives 0.75 -> bin 3 of 4 on [0, 1)
    p = O.Problem(dim=1, n=(2,), eq="euler")
    U = np.ones((1,) + p.state_shape)
    U[0, 0, 0, 0, 0] = 4.0
    U[0, 1, 0, 0, 0] = 3.0
    c = O.point_pdf(p, U, 1, [0], 0.0, 1.0, 4)
    assert c[0].tolist() == [0, 0, 0, 1, 0, 0]


def test_point_pdf_counts_add_up_and_invalid_arguments():
    p = O.Problem(dim=2, n=(5, 3), eq="euler")
    U = np.random.default_rng(3).normal(size=(17,) + p.state_shape) + 2.0
    c = O.point_pdf(p, U, 3, [0, 7, 14], 1.5, 2.5, 6)
    assert (c.sum(axis=1) == 17).all()
    with pytest.raises(O.OracleError):
        O.point_pdf(p, U, 4, [0], 0.0, 1.0, 4)   # no quantity 4 in 2D Euler
    with pytest.raises(O.OracleError):
        O.point_pdf(p, U, 0, [15], 0.0, 1.0, 4)  # cell out of range
    with pytest.raises(O.OracleError):
        O.point_pdf(p, U, 0, [0], 1.0, 1.0, 4)   # empty range
    with pytest.raises(O.OracleError):
        O.point_pdf(p, U, 0, [0], 0.0, 1.0, 0)


def test_joint_pdf_hand_counted_and_marginals():
    p = O.Problem(dim=1, n=(3,), eq="euler")
    rng = np.random.default_rng(11)
    U = np.ones((40,) + p.state_shape)
    U[:, 0, 0, 0, :] = rng.random((40, 3))          # rho in [0, 1)
    U[:, 2, 0, 0, :] = 2.0 + rng.random((40, 3))    # E in [2, 3)
    J = O.joint_pdf(p, U, 0, 2, [[0, 2], [1, 1]], 0.0, 1.0, 2.0, 3.0, 4)
    assert J.shape == (2, 17) and (J[:, -1] == 0).all() and (J.sum(axis=1) == 40).all()
    # hand count of pair 0 from the bin rule
    want = np.zeros(17, dtype=np.int64)
    for s in range(40):
        ka = math.floor(((U[s, 0, 0, 0, 0] - 0.0) / 1.0) * 4)
        kb = math.floor(((U[s, 2, 0, 0, 2] - 2.0) / 1.0) * 4)
        want[ka * 4 + kb] += 1
    assert J[0].tolist() == want.tolist()
    # marginals equal the point PDFs
    Pa = O.point_pdf(p, U, 0, [0], 0.0, 1.0, 4)
    Pb = O.point_pdf(p, U, 2, [2], 2.0, 3.0, 4)
    assert J[0, :16].reshape(4, 4).sum(axis=1).tolist() == Pa[0, :4].tolist()
    assert J[0, :16].reshape(4, 4).sum(axis=0).tolist() == Pb[0, :4].tolist()
    # a pair of one cell with itself and one quantity lies on the diagonal
    D = O.joint_pdf(p, U, 0, 0, [[1, 1]], 0.0, 1.0, 0.0, 1.0, 4)[0, :16].reshape(4, 4)
    assert (D == np.diag(np.diag(D))).all() and D.trace() == 40


def test_joint_pdf_outside_counter():
    p, U = _rho_state([0.5, 2.0, -1.0, 0.5])
    J = O.joint_pdf(p, U, 0, 0, [[0, 1]], 0.0, 1.0, 0.0, 2.0, 2)
    # sample 0: (0.5, 1) -> (1, 1); sample 1: rho(0) = 2 out of [0, 1) -> outside;
    # sample 2: -1 -> outside; sample 3: (1, 1)
    assert J[0].tolist() == [0, 0, 0, 2, 2]


def _shell(h, dim, ball):
    r = range(-h, h + 1)
    offs = []
    for oz in (r if dim >= 3 else [0]):
        for oy in (r if dim >= 2 else [0]):
            for ox in r:
                if ball:
                    if (h - 1) ** 2 < ox * ox + oy * oy + oz * oz <= h * h:
                        offs.append((ox, oy, oz))
                elif max(abs(ox), abs(oy), abs(oz)) == h:
                    offs.append((ox, oy, oz))
    return offs


def test_shell_sizes():
    for h in (1, 2, 3):
        assert len(_shell(h, 2, False)) == (2 * h + 1) ** 2 - (2 * h - 1) ** 2
        assert len(_shell(h, 3, False)) == (2 * h + 1) ** 3 - (2 * h - 1) ** 3
    assert len(_shell(1, 2, True)) == 4 and len(_shell(2, 2, True)) == 8


@pytest.mark.parametrize("dim,n", [(1, (11,)), (2, (7, 5)), (3, (5, 4, 6))])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ball", [False, True])
def test_shell_brute_force_numpy(dim, n, order, ball):
    p = O.Problem(dim=dim, n=n, eq="advection")
    q = np.random.default_rng(dim * 10 + order).normal(size=p.cells)
    Q = q.reshape(p.n[2], p.n[1], p.n[0])
    for h in range(1, min(n)):
        tot = 0.0
        offs = _shell(h, dim, ball)
        for ox, oy, oz in offs:
            d = np.roll(Q, shift=(-oz, -oy, -ox), axis=(0, 1, 2)) - Q
            tot += (np.abs(d) if order == 1 else d * d).sum()
        want = tot / (p.cells * len(offs))
        got = O.structure_shell(p, q, h, order, ball)
        assert got == pytest.approx(want, rel=1e-13)


def test_shell_sine_closed_form():
    # q = sin(2 pi k i / n): the sum over cells of (q(x + o) - q(x))^2 is N (1 - cos(2 pi k o_x / n))
    n, k = 32, 3
    p = O.Problem(dim=2, n=(n, n), eq="advection")
    i = np.arange(n)
    q = np.tile(np.sin(2 * np.pi * k * i / n), n)
    for h in (1, 2, 5, 9):
        for ball in (False, True):
            offs = _shell(h, 2, ball)
            want = sum(1.0 - math.cos(2 * math.pi * k * ox / n) for ox, _, _ in offs) / len(offs)
            assert O.structure_shell(p, q, h, 2, ball) == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_shell_checkerboard_order_one():
    # q = (-1)^(i + j): |q(x + o) - q(x)| = 2 when o_x + o_y is odd, else 0
    n = 8
    p = O.Problem(dim=2, n=(n, n), eq="advection")
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    q = np.where((i + j) % 2 == 0, 1.0, -1.0).ravel()
    for h in (1, 2, 3):
        for ball in (False, True):
            offs = _shell(h, 2, ball)
            odd = sum((ox + oy) % 2 for ox, oy, _ in offs)
            assert O.structure_shell(p, q, h, 1, ball) == pytest.approx(2.0 * odd / len(offs), rel=1e-15)


def test_ball_radius_one_is_axis_structure_function():
    p = O.Problem(dim=3, n=(6, 5, 7), eq="advection")
    q = np.random.default_rng(5).normal(size=p.cells)
    assert O.structure_shell(p, q, 1, 2, True) == pytest.approx(O.structure_function(p, q, 1), rel=1e-14)


def test_shell_constant_zero_and_batch_layout():
    p = O.Problem(dim=2, n=(6, 6), eq="euler")
    U = np.random.default_rng(8).random((3,) + p.state_shape) + 1.0
    U[1] = U[1].mean(axis=(1, 2, 3), keepdims=True)    # sample 1 constant per field
    S = O.structure_shell_batch(p, U, 3, 2, False)
    assert S.shape == (3, 4, 3)
    assert (S[1] == 0.0).all()
    q = O.quantities(p, U[2])
    for qi in range(4):
        for h in (1, 2, 3):
            assert S[2, qi, h - 1] == O.structure_shell(p, q[qi].ravel(), h, 2, False)
    with pytest.raises(O.OracleError):
        O.structure_shell_batch(p, U, 6, 2, False)     # max_h >= n
    with pytest.raises(O.OracleError):
        O.structure_shell_batch(p, U, 2, 3, False)     # order 3 not offered
