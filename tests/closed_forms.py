"""Closed forms and 1-D quadratures that pin the oracle independently of its own code.

Notation: V(r) = int G_k(x, y) f(y) dy with G_k = exp(i k |x-y|) / (4 pi |x-y|);
the volume potential of the paper is u = -V.
"""

import math

import numpy as np
from scipy.integrate import cumulative_trapezoid, quad


def ball_potential(r, k, b):
    """V for f = 1 on the ball |y| <= b (derived by integrating G over the ball).

    inside:  (1/k^2) [ sin(kr)/(kr) e^{ikb} (1 - ikb) - 1 ]
    outside: e^{ikr} (sin kb - kb cos kb) / (k^3 r)
    """
    r = np.asarray(r, dtype=np.float64)
    k = complex(k)
    out = np.empty(r.shape, dtype=np.complex128)
    ins = r <= b
    ri = np.where(r[ins] == 0.0, 1e-300, r[ins])
    sinc = np.where(r[ins] == 0.0, 1.0, np.sin(k * ri) / (k * ri))
    out[ins] = (sinc * np.exp(1j * k * b) * (1 - 1j * k * b) - 1.0) / (k * k)
    ro = r[~ins]
    out[~ins] = np.exp(1j * k * ro) * (np.sin(k * b) - k * b * np.cos(k * b)) / (k ** 3 * ro)
    return out


def radial_potential(f, k, r_eval, r_max, n_fine=200001):
    """V(r) for a radial density f(s) by the l = 0 term of the addition theorem.

    V(r) = i k [ h0(kr) int_0^r s^2 j0(ks) f ds + j0(kr) int_r^inf s^2 h0(ks) f ds ],
    j0(x) = sin x / x, h0(x) = -i e^{ix} / x.  Cumulative trapezoid on a fine grid.
    """
    k = complex(k)
    s = np.linspace(0.0, r_max, n_fine)
    s[0] = 1e-30
    fs = f(s)
    j0 = np.sin(k * s) / (k * s)
    h0 = -1j * np.exp(1j * k * s) / (k * s)
    g1 = s * s * j0 * fs
    g2 = s * s * h0 * fs
    I1 = cumulative_trapezoid(g1, s, initial=0.0)
    I2all = cumulative_trapezoid(g2, s, initial=0.0)
    I2 = I2all[-1] - I2all
    V = 1j * k * ((-1j * np.exp(1j * k * s) / (k * s)) * I1 + np.sin(k * s) / (k * s) * I2)
    r_eval = np.asarray(r_eval, dtype=np.float64)
    return np.interp(r_eval, s, V.real) + 1j * np.interp(r_eval, s, V.imag)


def ball_centre_integral(k, a):
    """int over the ball of radius a of G_k(0, y) dy = int_0^a s e^{iks} ds (adaptive quadrature)."""
    k = complex(k)
    re = quad(lambda s: (s * np.exp(1j * k * s)).real, 0.0, a, epsabs=0, epsrel=1e-13)[0]
    im = quad(lambda s: (s * np.exp(1j * k * s)).imag, 0.0, a, epsabs=0, epsrel=1e-13)[0]
    return complex(re, im)


def centred_grid(N, L):
    """Cube of side L with N voxels per axis, centres symmetric about the origin."""
    h = L / N
    c = (np.arange(N) - (N - 1) / 2.0) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return h, np.sqrt(X * X + Y * Y + Z * Z)


def lagrange_brute(field, src_origin, src_h, tgt_pts, order):
    """Non-separable evaluation: sum over the full (order+1)^3 stencil per target point."""
    n = field.shape
    out = np.zeros(len(tgt_pts), dtype=np.complex128)
    for t, x in enumerate(tgt_pts):
        idx = []
        wts = []
        for a in range(3):
            s = (x[a] - src_origin[a]) / src_h
            s = min(max(s, 0.0), n[a] - 1.0)
            i0 = min(math.floor(s), n[a] - 2)
            if order == 1:
                nodes = [i0, i0 + 1]
            else:
                b = min(max(i0 - 1, 0), n[a] - 4)
                nodes = [b, b + 1, b + 2, b + 3]
            w = []
            for j, xj in enumerate(nodes):
                p = 1.0
                for m, xm in enumerate(nodes):
                    if m != j:
                        p *= (s - xm) / (xj - xm)
                w.append(p)
            idx.append(nodes)
            wts.append(w)
        acc = 0.0
        for i, wi in zip(idx[0], wts[0]):
            for j, wj in zip(idx[1], wts[1]):
                for kk, wk in zip(idx[2], wts[2]):
                    acc += wi * wj * wk * field[i, j, kk]
        out[t] = acc
    return out
