"""ORACLE — test infrastructure only (see the package docstring).

A higher-order quadrature for the volume potential, the refinement that
Section 3.1 leaves open after equation "quad" (the paper keeps the midpoint
rule with an equal-volume ball on the self voxel and notes that a more
sophisticated rule could be used).

The rule is a locally corrected lattice (midpoint) rule in the manner of the
corrected trapezoidal rules for singular integrands (Marin, Runborg and
Tornberg, IMA J. Numer. Anal. 34, 2014): the midpoint sum over every voxel but
the target's own is kept, and the error that the singularity of G leaves in
it is removed by weights on the target voxel and its six face neighbours.

Derivation.  Put the target at the origin.  Near r = 0,

    G(r) = e^{ikr} / (4 pi r) = 1/(4 pi r) + ik/(4 pi) - k^2 r/(8 pi) + (terms smooth at 0 or O(r^3)).

For a smooth, decaying g and the cubic lattice h Z^3, the punctured lattice
sum of g |x|^a (a > -3, a not an even integer) has the expansion

    h^3 sum_{n != 0} g(nh) |nh|^a = int g |x|^a dx + h^{3+a} Z(-a/2) g(0)
                                    + h^{5+a} Z(-a/2 - 1) (lap g)(0) / 6 + O(h^{7+a}),

where Z(s) = sum_{n != 0} |n|^{-2s} is the Epstein zeta function of Z^3
(continued analytically), and the factor 1/6 comes from the cubic symmetry
sum_n |n|^a n_i n_j = delta_ij sum_n |n|^{a+2} / 3 applied to the Hessian
term of g's Taylor series.  Applying it to the three singular terms above
(a = -1, the constant, a = 1) and approximating lap f(0) by the 7-point
stencil gives

    int G f  =  sum_{j != 0} h^3 G(|x_j|) f_j  +  w_self f_0  +  w_face sum_{6 faces} f_j  + O(h^6 ...),
    w_self = h^2 (Z(-1/2) - Z(1/2)) / (4 pi) + i k h^3 / (4 pi) + k^2 h^4 Z(-1/2) / (8 pi),
    w_face = -h^2 Z(-1/2) / (24 pi).

(The i k h^3 / (4 pi) term restores the sample of the constant part of G at
the target, which the punctured sum leaves out.)  The discrete operator is
still a convolution: the paper's kernel with K(0) replaced by w_self and
w_face added at the six offsets of length one.  For a source f cut off at
the box edges the correction reads zero outside the grid, as the sum does.

Z(1/2) and Z(-1/2) are computed here by the Ewald (incomplete-gamma)
splitting of the Mellin integral of the lattice theta function, written out
below; the test suite pins Z(1/2) to the published value of the cubic
lattice sum and the rule to the continuous potential of a Gaussian source.
"""

import math

import numpy as np
from scipy import integrate as _integ
from scipy import special as _sp

from .core import conv_circulant, conv_direct, self_cell


# --------------------------------------------------------------------------
# Epstein zeta function of the cubic lattice Z^3
# --------------------------------------------------------------------------

def _upper_gamma(a, x):
    """Upper incomplete gamma function Gamma(a, x) for x > 0 and any real a (a <= 0 by recurrence)."""
    if a > 0:
        return _sp.gamma(a) * _sp.gammaincc(a, x)
    if a == 0:
        return _sp.exp1(x)
    # Gamma(a, x) = (Gamma(a + 1, x) - x^a e^{-x}) / a
    return (_upper_gamma(a + 1.0, x) - x ** a * np.exp(-x)) / a


def lattice_zeta(s, alpha=1.0, R=8):
    """Z(s) = sum over n in Z^3, n != 0, of |n|^{-2 s}, for s not in {0, 3/2}.

    Mellin: pi^{-s} Gamma(s) |n|^{-2s} = int_0^inf t^{s-1} e^{-pi |n|^2 t} dt.  Split
    the t-integral at alpha; on (0, alpha) apply Poisson summation to the lattice
    theta function (Z^3 is its own dual, volume 1):

      pi^{-s} Gamma(s) Z(s) = alpha^{s-3/2} / (s - 3/2) - alpha^s / s
          + sum_{n != 0} [ (pi n^2)^{-s} Gamma(s, pi n^2 alpha)
                           + (pi n^2)^{s-3/2} Gamma(3/2 - s, pi n^2 / alpha) ].

    The result does not depend on alpha (a check of the formula); both sums
    converge like e^{-pi n^2 min(alpha, 1/alpha)}, so |n| <= R suffices.
    """
    r = np.arange(-R, R + 1, dtype=np.float64)
    n2 = (r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2).ravel()
    n2 = n2[n2 > 0]
    x = math.pi * n2
    tot = alpha ** (s - 1.5) / (s - 1.5) - alpha ** s / s
    tot += np.sum(x ** (-s) * _upper_gamma(s, x * alpha) + x ** (s - 1.5) * _upper_gamma(1.5 - s, x / alpha))
    return float(tot * math.pi ** s / _sp.gamma(s))


# --------------------------------------------------------------------------
# the corrected weights and the operator
# --------------------------------------------------------------------------

def corrected_weights(k, h):
    """(w_self, w_face) of the corrected rule (module docstring), complex."""
    k = complex(k)
    z_half, z_mhalf = lattice_zeta(0.5), lattice_zeta(-0.5)
    w_self = (h * h * (z_mhalf - z_half) / (4.0 * math.pi) + 1j * k * h ** 3 / (4.0 * math.pi)
              + k * k * h ** 4 * z_mhalf / (8.0 * math.pi))
    w_face = -h * h * z_mhalf / (24.0 * math.pi)
    return complex(w_self), complex(w_face)


def _local_correction(f, h, k):
    """(w_self - K_ball) f_i + w_face (sum of f over the six face neighbours inside the grid)."""
    f = np.asarray(f, dtype=np.complex128)
    w_self, w_face = corrected_weights(k, h)
    out = (w_self - self_cell(k, h)) * f
    nb = np.zeros_like(f)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        nb[tuple(lo)] += f[tuple(hi)]
        nb[tuple(hi)] += f[tuple(lo)]
    return out + w_face * nb


def conv_direct_corrected(f, h, k, targets=None):
    """out_i = sum_j K_c(x_i - x_j) f_j with the corrected kernel: the paper's direct sum plus
    the local correction.  targets: flat C-order indices, or None for every voxel."""
    if targets is None:
        return conv_direct(f, h, k) + _local_correction(f, h, k)
    return conv_direct(f, h, k, targets=targets) + _local_correction(f, h, k).ravel()[np.asarray(targets)]


def conv_circulant_corrected(f, h, k, M=None):
    """The same by the circulant FFT cross-check."""
    return conv_circulant(f, h, k, M=M) + _local_correction(f, h, k)


def volume_potential_corrected(f, h, k, method="direct", M=None):
    """u = -int_D G_k f with the corrected rule (the raw operator's sign convention)."""
    if method == "direct":
        return -conv_direct_corrected(f, h, k)
    return -conv_circulant_corrected(f, h, k, M=M)


# --------------------------------------------------------------------------
# a continuous reference: the potential of a Gaussian source
# --------------------------------------------------------------------------

def gaussian_potential(r, k, sigma):
    """int_{R^3} G_k(|x - y|) exp(-|y|^2 / (2 sigma^2)) dy at |x| = r.

    For a radial source the angular integral of G over the sphere |y| = s is
    s (e^{ik(r+s)} - e^{ik|r-s|}) / (2 i k r), so the potential is a 1-D
    integral over s, evaluated by adaptive quadrature (r = 0: its limit,
    int_0^inf s e^{iks} f(s) ds)."""
    k = complex(k)

    def f(s):
        return math.exp(-s * s / (2.0 * sigma * sigma))

    def integrand(s, part):
        if r == 0.0:
            v = s * np.exp(1j * k * s) * f(s)
        else:
            v = s * f(s) * (np.exp(1j * k * (r + s)) - np.exp(1j * k * abs(r - s))) / (2j * k * r)
        return v.real if part == 0 else v.imag

    top = r + 14.0 * sigma
    pts = [r] if r > 0 else None
    re = _integ.quad(integrand, 0.0, top, args=(0,), points=pts, limit=500, epsabs=1e-13, epsrel=1e-11)[0]
    im = _integ.quad(integrand, 0.0, top, args=(1,), points=pts, limit=500, epsabs=1e-13, epsrel=1e-11)[0]
    return complex(re, im)
