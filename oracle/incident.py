"""ORACLE — test infrastructure only (see the package docstring).

The incident (first-harmonic) field p_1 of a transducer modelled as
equal-weight point sources on its surface (Section 3.2, the incident-field
equation): a weighted sum of free-space Green's functions

    G_k(x, y) = exp(i k |x - y|) / (4 pi |x - y|)

over the source points, evaluated here at arbitrary targets.  The weights and
the source strength are folded into one complex scale.  Plain FP64 numpy.

Pins (tests/test_oracle_pins.py):
  * every point of a spherical cap lies one radius of curvature l from the
    geometric focus, so with the Rayleigh scale of a baffled cap the sum there
    is exactly -i k h p0 exp(i k l) (h the cap height), for any point set;
  * on the axis the equal-area spiral's sum converges to O'Neil's closed form
    for the cap at second order in 1 / n_points.
"""

import math

import numpy as np


def incident_at(points, k, scale, targets, chunk=1024):
    """scale * sum_j G_k(t, p_j) at each target t (targets: (N, 3) float64) -> complex128 (N,)."""
    P = np.asarray(points, dtype=np.float64)
    T = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
    k = complex(k)
    out = np.empty(T.shape[0], dtype=np.complex128)
    for s in range(0, T.shape[0], chunk):
        d = T[s:s + chunk, None, :] - P[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        g = np.exp(1j * k * r) / (4.0 * math.pi * r)
        out[s:s + chunk] = complex(scale) * g.sum(axis=1)
    return out


def incident_field(points, k, scale, grid, chunk=1024):
    """The same sum at every voxel centre of `grid` -> complex128 array of shape grid.n."""
    X, Y, Z = np.meshgrid(grid.coords(0), grid.coords(1), grid.coords(2), indexing="ij")
    T = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return incident_at(points, k, scale, T, chunk).reshape(tuple(grid.n))


def radiated_power(points, k, scale, centre, radius, rho0, c0, n_r, n_theta):
    """Power through the disc of `radius` centred at `centre` in the plane x = centre[0]:

        1 / (2 rho0 c0) * int_0^{2 pi} int_0^radius |p(r, theta)|^2 r dr dtheta

    (Section 3.2, the radiated-power integral over a disc covering the open
    end of the bowl; the printed integrand lacks the area element r and the
    modulus, read here as |p|^2 r), by the midpoint rule with n_r x n_theta
    nodes.  Used to scale p_1 to a prescribed power P0 by sqrt(P0 / power).
    """
    dr = radius / n_r
    dth = 2.0 * math.pi / n_theta
    r = (np.arange(n_r) + 0.5) * dr
    th = (np.arange(n_theta) + 0.5) * dth
    R_, T_ = np.meshgrid(r, th, indexing="ij")
    tg = np.stack([np.full(R_.size, float(centre[0])), centre[1] + (R_ * np.cos(T_)).ravel(),
                   centre[2] + (R_ * np.sin(T_)).ravel()], axis=1)
    p = incident_at(points, k, scale, tg).reshape(n_r, n_theta)
    return float(np.sum(np.abs(p) ** 2 * R_) * dr * dth / (2.0 * rho0 * c0))
