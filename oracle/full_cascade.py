"""ORACLE — test infrastructure only (see the package docstring).

The harmonic cascade with the terms that the paper drops.  Matching the
coefficients of e^{-i n w t} in the Westervelt equation gives equation
"cascade_1" of Section 2, whose right-hand side for harmonic n is

    (beta w^2 n^2 / (2 rho0 c0^4)) sum_{m >= 1} p_m (p_{n-m} + 2 p*_{m-n}),   p_j = 0 for j <= 0.

The paper keeps only the sum-frequency products p_m p_{n-m} (m < n), giving
equation "cascade_2", a one-way cascade.  With N harmonics kept, the full
system adds the difference-frequency products 2 sum_{m=n+1}^{N} p_m conj(p_{m-n})
to every harmonic, p_1 included; they carry energy from the higher harmonics
back down, so the harmonics no longer follow from one pass in order.

Reading (the paper leaves this case to future work): the truncated system is
solved by a fixed-point iteration.  Sweep 0 is the paper's cascade.  Each
later sweep recomputes p_1, ..., p_N in order, harmonic n from the newest
values of all the others:

    p_n = [n = 1] p_inc + C_n sum_j K_{k_n}(x_i - x_j) (S_n + D_n)(x_j),
    S_n = sum_{m<n} p_m p_{n-m}    (the paper's source, transferred as in Section 6),
    D_n = 2 sum_{m=n+1}^{N} p_m conj(p_{m-n}),

until no harmonic changes by more than `tol` in relative L2.  Transfers onto
p_n's grid: a lower harmonic (m < n) as in Section 6 (clamped into its hull;
its box contains p_n's); a higher harmonic (m > n) is zero outside its own,
smaller box, so it is interpolated with zero at targets outside the hull of
its voxel centres.
"""

import numpy as np

from .core import (cascade_constant, conv_circulant, source_term, transfer, transfer_axis,
                   wavenumber)

_HULL_EPS = 1e-9  # in source voxels: a target this close to the hull counts as inside


def transfer_axis_zero(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order):
    """transfer_axis, with the weights of targets outside the source hull of centres set to zero."""
    base, w = transfer_axis(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order)
    x = dst_origin + np.arange(dst_n, dtype=np.float64) * dst_h
    s = (x - src_origin) / src_h
    outside = (s < -_HULL_EPS) | (s > float(src_n - 1) + _HULL_EPS)
    w = w.copy()
    w[outside, :] = 0.0
    return base, w


def transfer_zero(field, src, dst, order):
    """Tensor-product interpolation of `field` (on grid src) at the centres of grid dst, zero at
    targets outside src's hull on any axis."""
    out = np.asarray(field, dtype=np.complex128)
    for a in range(3):
        base, w = transfer_axis_zero(dst.origin[a], dst.h, dst.n[a], src.origin[a], src.h, src.n[a], order)
        acc = None
        for j in range(w.shape[1]):
            sh = [1, 1, 1]
            sh[a] = dst.n[a]
            term = np.take(out, base + j, axis=a) * w[:, j].reshape(sh)
            acc = term if acc is None else acc + term
        out = acc
    return out


def transfer_to(field, src, dst, order, zero_outside):
    """transfer_zero if zero_outside else the paper's (clamped) transfer; a field on dst itself as is."""
    if src.same_as(dst):
        return np.asarray(field, dtype=np.complex128).copy()
    return transfer_zero(field, src, dst, order) if zero_outside else transfer(field, src, dst, order)


def difference_term(dst, a, ga, za, b, gb, zb, order, scale):
    """scale * T_a(a) * conj(T_b(b)) on grid dst; T_x = transfer_to(..., zero_outside=z_x)."""
    return scale * transfer_to(a, ga, dst, order, za) * np.conj(transfer_to(b, gb, dst, order, zb))


def full_source(n, v, N):
    """S_n + D_n for values v = {m: v_m}, m = 1..N (the bracket of equation cascade_1, truncated at N)."""
    s = 0.0 if n == 1 else source_term(n, v)
    for m in range(n + 1, N + 1):
        s = s + 2.0 * v[m] * np.conj(v[m - n])
    return s


def _potential(f, grid, k):
    return conv_circulant(f, grid.h, k)


def full_cascade(p_inc, g1, grids, f0, medium, order, tol=1e-10, max_sweeps=50):
    """Fixed point of the truncated system; grids = {n: Grid} for n = 2..N.

    Returns ({n: p_n} for n = 1..N, sweeps, last relative change)."""
    N = max(grids)
    g = dict(grids)
    g[1] = g1
    p_inc = np.asarray(p_inc, dtype=np.complex128)
    p = {1: p_inc.copy()}
    for n in range(2, N + 1):  # sweep 0: the paper's cascade
        v = {m: transfer(p[m], g[m], g[n], order) for m in range(1, n)}
        p[n] = cascade_constant(n, f0, medium) * _potential(source_term(n, v), g[n], wavenumber(n, f0, medium))
    change = np.inf
    sweeps = 0
    while change > tol and sweeps < max_sweeps:
        sweeps += 1
        change = 0.0
        for n in range(1, N + 1):
            v = {m: transfer_to(p[m], g[m], g[n], order, m > n) for m in range(1, N + 1)}
            f = full_source(n, v, N) * np.ones(g[n].n)
            new = cascade_constant(n, f0, medium) * _potential(f, g[n], wavenumber(n, f0, medium))
            if n == 1:
                new = new + p_inc
            change = max(change, float(np.linalg.norm(new - p[n]) / np.linalg.norm(new)))
            p[n] = new
    return p, sweeps, change
