"""Pins of the oracle's corrected (higher-order) quadrature (CPU only).

The rule is pinned to things it does not compute itself: the published value
of the cubic lattice sum, brute-force lattice sums, the independence of the
Ewald splitting parameter, and the continuous potential of a Gaussian source
(a 1-D radial integral) at the paper's lambda/6 spacing and one level finer.
"""

import math

import numpy as np
import pytest

import oracle


def test_lattice_zeta_half_is_the_published_cubic_lattice_sum():
    """Z(1/2), the analytically continued sum of 1/|n| over Z^3 minus the origin, is the
    lattice constant -2.8372974794806... of the literature on cubic lattice sums."""
    assert oracle.lattice_zeta(0.5) == pytest.approx(-2.8372974794806, abs=1e-12)


def test_lattice_zeta_does_not_depend_on_the_splitting():
    for s in (0.5, -0.5, 2.5, 3.0):
        ref = oracle.lattice_zeta(s, alpha=1.0)
        for a in (0.6, 1.7):
            assert oracle.lattice_zeta(s, alpha=a) == pytest.approx(ref, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("s", [2.5, 3.0])
def test_lattice_zeta_matches_brute_force_where_the_sum_converges(s):
    R = 60
    r = np.arange(-R, R + 1, dtype=np.float64)
    n2 = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    inside = (n2 > 0) & (n2 <= R * R)
    brute = float(np.sum(n2[inside] ** (-s)))
    tail = 4.0 * math.pi * R ** (3.0 - 2.0 * s) / (2.0 * s - 3.0)  # int_R^inf 4 pi r^2 r^{-2s} dr
    assert oracle.lattice_zeta(s) == pytest.approx(brute + tail, rel=2e-6)


def test_corrected_weights_reduce_to_the_laplace_constants():
    """k -> 0: w_self -> h^2 (Z(-1/2) - Z(1/2)) / (4 pi), w_face = -h^2 Z(-1/2) / (24 pi)."""
    h = 0.37
    ws, wf = oracle.corrected_weights(1e-9, h)
    z1, z2 = oracle.lattice_zeta(0.5), oracle.lattice_zeta(-0.5)
    assert ws == pytest.approx(h * h * (z2 - z1) / (4 * math.pi), rel=1e-8)
    assert wf == pytest.approx(-h * h * z2 / (24 * math.pi), rel=1e-12)


def test_corrected_direct_sum_equals_its_circulant_form():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((7, 5, 6)) + 1j * rng.standard_normal((7, 5, 6))
    h, k = 0.8, 1.3 + 0.02j
    a = oracle.conv_direct_corrected(f, h, k)
    b = oracle.conv_circulant_corrected(f, h, k, M=(13, 9, 11))
    assert oracle.rel_l2(b, a) < 1e-13
    # the correction is local: a point source spreads to itself and its faces only
    d = np.zeros((5, 5, 5), complex)
    d[2, 2, 2] = 1.0
    diff = oracle.conv_direct_corrected(d, h, k) - oracle.conv_direct(d, h, k)
    ws, wf = oracle.corrected_weights(k, h)
    assert diff[2, 2, 2] == pytest.approx(ws - oracle.self_cell(k, h), rel=1e-14)
    for off in ((1, 0, 0), (0, -1, 0), (0, 0, 1)):
        assert diff[2 + off[0], 2 + off[1], 2 + off[2]] == pytest.approx(wf, rel=1e-14)
    assert np.count_nonzero(np.abs(diff) > 1e-18) == 7


def _gaussian_errors(N, h, sigma, k):
    """Max error (relative to the max of the exact values) of the paper's rule and the
    corrected rule on the x axis of an N^3 grid centred on a Gaussian source."""
    x = (np.arange(N) - N / 2 + 0.5) * h
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    f = np.exp(-r2 / (2 * sigma * sigma))
    ball = oracle.conv_circulant(f, h, k)
    corr = oracle.conv_circulant_corrected(f, h, k)
    idx = [(N // 2 + i, N // 2, N // 2) for i in range(0, N // 2 - 2, max(1, N // 12))]
    ex = np.array([oracle.gaussian_potential(math.sqrt(r2[t]), k, sigma) for t in idx])
    scale = np.abs(ex).max()
    e_ball = np.abs(np.array([ball[t] for t in idx]) - ex).max() / scale
    e_corr = np.abs(np.array([corr[t] for t in idx]) - ex).max() / scale
    return e_ball, e_corr


def test_corrected_rule_at_lambda_over_6_and_its_order():
    """kh = 2 pi / 6 (the paper's spacing), sigma = 4.5 h: the paper's rule misses the continuous
    potential by a few percent and converges at second order; the corrected rule is within
    5e-4 and gains more than 2^5 per halving of h."""
    k = 1.05 + 0.01j
    b1, c1 = _gaussian_errors(48, 1.0, 4.5, k)
    b2, c2 = _gaussian_errors(96, 0.5, 4.5, k)
    assert 1e-2 < b1 < 6e-2
    assert c1 < 5e-4
    assert 3.0 < b1 / b2 < 6.0
    assert c1 / c2 > 32.0


def test_corrected_dense_operator_equals_the_corrected_sum():
    rng = np.random.default_rng(8)
    for n in ((4, 3, 5), (6, 1, 2)):
        f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        h, k = 0.9, 1.1 + 0.05j
        A = oracle.dense_operator(k, h, n, rule="corrected")
        assert oracle.rel_l2((A @ f.ravel()).reshape(n), oracle.conv_direct_corrected(f, h, k)) < 1e-14
