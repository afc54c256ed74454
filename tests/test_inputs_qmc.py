"""Pins of the Sobol quasi-Monte Carlo points used as Kelvin--Helmholtz sample inputs: the
primitive polynomials (counts per degree from Euler's totient, the textbook first few), the
stratification every Sobol coordinate has (the first 2^m values are the multiples of 2^-m),
the (0, m, 2)-net property of the first two coordinates, and the second coordinate worked
out by hand from its recurrence."""

import numpy as np

import fv_inputs as fi


def _phi(n):
    r, m, f = n, n, 2
    while f * f <= m:
        if m % f == 0:
            while m % f == 0:
                m //= f
            r -= r // f
        f += 1
    if m > 1:
        r -= r // m
    return r


def test_primitive_polynomials():
    polys = fi.primitive_polynomials(52)
    # x + 1, x^2 + x + 1, x^3 + x + 1, x^3 + x^2 + 1, x^4 + x + 1, x^4 + x^3 + 1
    assert polys[:6] == [0b11, 0b111, 0b1011, 0b1101, 0b10011, 0b11001]
    deg = [p.bit_length() - 1 for p in polys]
    assert deg == sorted(deg)
    for d in range(1, 8):
        assert deg.count(d) == _phi(2 ** d - 1) // d


def test_coordinates_are_stratified():
    for m in range(1, 11):
        X = fi.sobol_points(2 ** m, 21)
        for j in range(21):
            assert sorted((X[:, j] * 2 ** m).tolist()) == list(range(2 ** m))


def test_first_two_coordinates_form_a_0m2_net():
    for m in range(1, 9):
        X = fi.sobol_points(2 ** m, 2)
        for i in range(m + 1):
            boxes = np.floor(X[:, 0] * 2 ** i).astype(int) * 2 ** (m - i) + np.floor(X[:, 1] * 2 ** (m - i)).astype(int)
            assert sorted(boxes.tolist()) == list(range(2 ** m))


def test_second_coordinate_by_hand():
    # x + 1: m_k = 2 m_(k-1) xor m_(k-1) from m_1 = 1, so m = 1, 3, 5, 15, ... and
    # v_k = m_k / 2^k = 1/2, 3/4, 5/8; point n is the xor of v_k over the set bits of n
    X = fi.sobol_points(8, 2)
    assert X[:, 1].tolist() == [0.0, 0.5, 0.75, 0.25, 0.625, 0.125, 0.375, 0.875]
    assert X[:, 0].tolist() == [0.0, 0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875]


def test_skip_and_kh_coefficients():
    A = fi.sobol_points(40, 20)
    B = fi.sobol_points(30, 20, skip=10)
    assert np.array_equal(A[10:], B)
    c, phi = fi.kh_coefficients_qmc(np.arange(16))
    assert c.shape == (16, 10) and phi.shape == (16, 10)
    assert np.array_equal(c, A[1:17, :10]) and np.array_equal(phi, 2 * np.pi * A[1:17, 10:])
    assert (c >= 0).all() and (c < 1).all() and (phi >= 0).all() and (phi < 2 * np.pi).all()
    # a subset of samples picks the same points
    c2, _ = fi.kh_coefficients_qmc([3, 7])
    assert np.array_equal(c2, c[[3, 7]])
