"""Pins of the SRAD oracle (oracle/hxo_srad.h) against facts other than its
own formulas: conservation, symmetries, a library routine, numpy's
statistics and a hand-worked pixel."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle


def speckle(h, w, seed):
    rng = np.random.default_rng(seed)
    base = np.full((h, w), 0.4)
    base[h // 4: 3 * h // 4, w // 3: 2 * w // 3] = 1.0
    return (base * rng.gamma(4.0, 0.25, (h, w)) + 0.05).astype(np.float32)


SHAPES = [(1, 1), (1, 6), (6, 1), (2, 2), (5, 7), (16, 9), (33, 40)]


@pytest.mark.parametrize("shape", SHAPES)
def test_mass_is_conserved(shape):
    """The flux between two neighbours uses one coefficient on both sides
    and the clamped border has no flux, so sum(J) never changes."""
    J = speckle(*shape, 1)
    out, _ = oracle.srad(J, 5, 0.5)
    s0 = J.astype(np.float64).sum()
    assert abs(out.sum() - s0) <= 1e-12 * abs(s0)


def test_power_of_two_scaling_is_exact():
    J = speckle(20, 17, 2)
    a, qa = oracle.srad(J, 4, 0.5)
    b, qb = oracle.srad(J * np.float32(4.0), 4, 0.5)
    assert np.array_equal(b, 4.0 * a)
    assert np.array_equal(qa, qb)


def test_transpose_equivariance():
    J = speckle(23, 31, 3)
    a, qa = oracle.srad(J, 3, 0.5)
    b, qb = oracle.srad(np.ascontiguousarray(J.T), 3, 0.5)
    assert np.allclose(b, a.T, rtol=1e-13, atol=0)
    assert np.allclose(qa, qb, rtol=1e-13)


def test_flat_image_is_a_fixed_point():
    J = np.full((9, 11), 0.7, np.float32)
    out, q = oracle.srad(J, 3, 0.5)
    # the one-pass variance of a flat image is 0 up to rounding (here just
    # below it); c is 1 there and every derivative is 0
    assert np.array_equal(out, J.astype(np.float64)) and np.all(np.abs(q) <= 1e-14)
    assert np.all(oracle.srad_coeff(J, 0.0) == 1.0)
    assert np.all(oracle.srad_coeff(J, -1e-15) == 1.0)


def test_update_with_unit_coefficient_is_a_heat_step():
    """With c = 1 everywhere, D is the 5-point Laplacian with replicated
    borders: scipy.ndimage.laplace(mode='nearest')."""
    J = speckle(12, 15, 4).astype(np.float64)
    out = oracle.srad_update(J, np.ones_like(J), 0.3)
    want = J + 0.25 * 0.3 * ndi.laplace(J, mode="nearest")
    assert np.allclose(out, want, rtol=1e-14, atol=1e-15)


def test_stats_match_numpy():
    J = speckle(30, 41, 5).astype(np.float64)
    q, m, v = oracle.srad_stats(J)
    assert abs(m - J.mean()) <= 1e-14 * m
    assert abs(v - J.var()) <= 1e-10 * v
    assert abs(q - J.var() / J.mean() ** 2) <= 1e-10 * q


def test_coefficient_of_a_hand_worked_pixel():
    """Centre 1 with one neighbour 2 (north), the others 1: dN = 1, so
    g2 = 1, l = 1, q^2 = (1/2 - 1/16) / (5/4)^2 = 0.28; with q0^2 = 0.25,
    c = 1 / (1 + 0.03 / 0.3125) = 1 / 1.096."""
    J = np.ones((3, 3))
    J[0, 1] = 2.0
    c = oracle.srad_coeff(J, 0.25)
    assert abs(c[1, 1] - 1.0 / 1.096) <= 1e-15
    # a pixel whose neighbours all equal it has q^2 = 0: c = (1 + q0^2) / q0^2 > 1 -> 1
    J2 = np.ones((3, 3))
    assert oracle.srad_coeff(J2, 0.25)[1, 1] == 1.0


def test_zero_iterations_return_the_input():
    J = speckle(4, 5, 6)
    out, q = oracle.srad(J, 0, 0.5)
    assert np.array_equal(out, J.astype(np.float64)) and q.size == 0
