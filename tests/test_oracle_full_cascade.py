"""Pins of the oracle's full harmonic cascade (the difference-frequency terms the paper drops)."""

import math

import numpy as np
import pytest

import oracle
from oracle import full_cascade as FC
from workload import bowl, configs

WATER = configs.WATER
F0 = 1.1e6


def test_full_source_is_the_fourier_coefficient_of_p_squared():
    """With p(t) = 1/2 sum_n (p_n e^{-i n w t} + c.c.), the coefficient of e^{-i n w t} in p(t)^2
    is 1/4 sum_m p_m (p_{n-m} + 2 p*_{m-n}), which is what equation cascade_1 expands: checked by
    sampling p(t)^2 over one period and summing its Fourier coefficients by brute force."""
    rng = np.random.default_rng(4)
    N = 5
    v = {m: complex(*rng.standard_normal(2)) for m in range(1, N + 1)}
    T = 64
    wt = 2 * math.pi * np.arange(T) / T
    p = sum(0.5 * (v[m] * np.exp(-1j * m * wt) + np.conj(v[m]) * np.exp(1j * m * wt)) for m in v).real
    for n in range(1, N + 1):
        c = np.sum(p * p * np.exp(1j * n * wt)) / T
        assert 4 * c == pytest.approx(FC.full_source(n, v, N), abs=1e-13), n
        if n < N:  # the dropped part is not small in general
            assert abs(FC.full_source(n, v, N) - (0 if n == 1 else oracle.source_term(n, v))) > 0.1


@pytest.mark.parametrize("order", [1, 3])
def test_zero_outside_transfer_reproduces_polynomials_inside_the_hull(order):
    src = oracle.Grid((0.0, 0.0, 0.0), 1.0, (10, 8, 9))
    dst = oracle.Grid((-2.3, 1.4, -0.6), 0.45, (30, 12, 25))
    xs, ys, zs = src.coords(0)[:, None, None], src.coords(1)[None, :, None], src.coords(2)[None, None, :]
    poly = (lambda x, y, z: (1.0 + 0.5j) + 0.3 * x - 0.2j * y + 0.7 * z) if order == 1 else \
        (lambda x, y, z: 0.01 * x ** 3 - 0.2 * x * y + 0.05j * y ** 2 * z + z ** 3 * 0.003 - 1.0)
    out = FC.transfer_zero(poly(xs, ys, zs), src, dst, order)
    X, Y, Z = dst.coords(0)[:, None, None], dst.coords(1)[None, :, None], dst.coords(2)[None, None, :]
    inside = ((X >= 0) & (X <= 9)) & ((Y >= 0) & (Y <= 7)) & ((Z >= 0) & (Z <= 8))
    exact = np.broadcast_to(poly(X, Y, Z), out.shape)
    assert np.any(inside) and np.any(~inside)
    assert np.max(np.abs(out[inside] - exact[inside])) < 1e-12
    assert np.all(out[~inside] == 0)


def tiny(amplitude, N=3):
    focus = (15e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (10, 9, 8), (5, 4, 4))
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (8 + 2 * n, 11, 10), (6, 5, 4))
          for n in range(2, N + 1)}
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(7.5e-3, 15e-3, 128, 1)
    p1 = bowl.incident_field(pts, 7.5e-3, 15e-3, k1, amplitude, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    return g1, gn, p1


def test_fixed_point_satisfies_the_truncated_system():
    """Each converged harmonic equals [n = 1] p_inc + C_n times the direct midpoint sum of its full
    source, built from the converged fields."""
    g1, gn, p1 = tiny(3e6)
    p, sweeps, change = FC.full_cascade(p1, g1, gn, F0, WATER, 3, tol=1e-13)
    assert change <= 1e-13 and sweeps < 50
    g = dict(gn)
    g[1] = g1
    N = max(gn)
    for n in range(1, N + 1):
        v = {m: FC.transfer_to(p[m], g[m], g[n], 3, m > n) for m in range(1, N + 1)}
        f = FC.full_source(n, v, N) * np.ones(g[n].n)
        rhs = oracle.cascade_constant(n, F0, WATER) * oracle.conv_direct(f, g[n].h, oracle.wavenumber(n, F0, WATER))
        if n == 1:
            rhs = rhs + p1
        assert oracle.rel_l2(p[n], rhs) < 1e-11, n


def test_difference_terms_scale_with_the_amplitude():
    """p_2 ~ a^2 and p_3 ~ a^3, so the change of p_1 (from 2 p_2 conj p_1) grows as a^3 and that
    of p_2 (from 2 p_3 conj p_1) as a^4: doubling a small amplitude multiplies them by 8 and 16."""
    d = {}
    for a in (1e4, 2e4):
        g1, gn, p1 = tiny(a)
        full, _, _ = FC.full_cascade(p1, g1, gn, F0, WATER, 3, tol=1e-14)
        paper = oracle.cascade(p1, g1, gn, F0, WATER, 3)
        d[a] = (np.linalg.norm(full[1] - p1), np.linalg.norm(full[2] - paper[2]))
    assert d[2e4][0] / d[1e4][0] == pytest.approx(8.0, rel=1e-3)
    assert d[2e4][1] / d[1e4][1] == pytest.approx(16.0, rel=1e-3)
