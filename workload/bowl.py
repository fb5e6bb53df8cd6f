"""Bowl transducer: surface points and the incident (first-harmonic) field.

Geometry (paper, Section 3.2 and the domain figure of Section 3.3): a
spherical cap of radius of curvature l (the geometric focal length) and outer
radius R, apex at the origin, axis along +x, centre of curvature (the
geometric focus) at (l, 0, 0).

Points: the paper places n_p evenly spaced monopoles on the cap (after
Deserno).  Here they are an equal-area golden-angle spiral: the cap area is
uniform in cos(theta) (theta measured at the focus from the -x axis), so
point i takes cos(theta_i) = 1 - (i + 1/2) (h / l) / n_p with h the cap
height, and azimuth phi_i = i * pi * (3 - sqrt 5) + 2 pi u with one seeded
uniform offset u.  Every point lies exactly l away from the focus.

Field: the paper sums monopoles G_k(x, r_i) = exp(i k |x - r_i|) / (4 pi
|x - r_i|) with equal weights A / n_p (incident-field equation) and then scales
the sum.  The scale used here ties it to a surface pressure p0 through the
Rayleigh integral of a baffled cap, p1 = -2 i k p0 * (A / n_p) * sum G_k, which
reproduces O'Neil's on-axis closed form and gives exactly
p1(focus) = -i k h p0 exp(i k l) for any point set on the cap.
"""

import math

import numpy as np
import torch


def cap_height(R, l):
    return l - math.sqrt(l * l - R * R)


def cap_area(R, l):
    return 2.0 * math.pi * l * cap_height(R, l)


def bowl_points(R, l, n_points, seed=0):
    """(n_points, 3) float64 array of equal-area spiral points on the cap."""
    if not (0.0 < R < l):
        raise ValueError("bowl needs 0 < R < l")
    h = cap_height(R, l)
    u = np.random.default_rng(seed).random()
    i = np.arange(n_points, dtype=np.float64)
    cos_t = 1.0 - (i + 0.5) * (h / l) / n_points
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = i * math.pi * (3.0 - math.sqrt(5.0)) + 2.0 * math.pi * u
    pts = np.empty((n_points, 3), dtype=np.float64)
    pts[:, 0] = l - l * cos_t
    pts[:, 1] = l * sin_t * np.cos(phi)
    pts[:, 2] = l * sin_t * np.sin(phi)
    return pts


def bowl_points_deserno(R, l, n_target):
    """(n, 3) float64 array of Deserno's regular placement on the cap, n close to n_target.

    Deserno's regular equidistribution on a sphere (M. Deserno, "How to generate
    equidistributed points on the surface of a sphere", 2004), restricted to the
    bowl's polar-angle range [0, theta_max], sin(theta_max) = R / l, on the sphere of
    radius l about the focus: with the area per point a = A / n_target and
    d = sqrt(a) / l (an angle), the cap is cut into M_theta = round(theta_max / d)
    bands of equal angular height d_theta = theta_max / M_theta; band m, at
    theta_m = (m + 1/2) d_theta, carries M_phi = round(2 pi sin(theta_m) / d_phi)
    points, d_phi = (a / l^2) / d_theta, at phi = 2 pi j / M_phi.  Apex at the
    origin, axis +x, as bowl_points."""
    if not (0.0 < R < l) or n_target < 1:
        raise ValueError("bowl needs 0 < R < l and at least one point")
    theta_max = math.asin(R / l)
    a = cap_area(R, l) / n_target / (l * l)  # area per point on the unit sphere
    d = math.sqrt(a)
    m_theta = max(1, int(round(theta_max / d)))
    d_theta = theta_max / m_theta
    d_phi = a / d_theta
    pts = []
    for m in range(m_theta):
        theta = (m + 0.5) * d_theta
        m_phi = max(1, int(round(2.0 * math.pi * math.sin(theta) / d_phi)))
        phi = 2.0 * math.pi * np.arange(m_phi) / m_phi
        band = np.empty((m_phi, 3), dtype=np.float64)
        band[:, 0] = l - l * math.cos(theta)
        band[:, 1] = l * math.sin(theta) * np.cos(phi)
        band[:, 2] = l * math.sin(theta) * np.sin(phi)
        pts.append(band)
    return np.concatenate(pts, axis=0)


def rayleigh_scale(R, l, k1, p0, n_points):
    """Scale s of the monopole sum s * sum_j exp(i k r_j) / (4 pi r_j) that makes it the Rayleigh
    integral of a baffled cap of surface pressure p0: s = -2 i k p0 A / n_points."""
    return -2j * complex(k1) * p0 * cap_area(R, l) / n_points


def incident_field(points, R, l, k1, p0, xs, ys, zs, device="cpu", chunk=4096):
    """p1 on the tensor grid xs x ys x zs (1-D float64 coordinate arrays).

    Returns a complex128 torch tensor of shape (len(xs), len(ys), len(zs)) on
    `device`.  k1 is the complex first-harmonic wavenumber (Im k1 >= 0);
    the same k1 enters the prefactor and the exponent.
    """
    dev = torch.device(device)
    n_p = points.shape[0]
    k1 = complex(k1)
    pref = rayleigh_scale(R, l, k1, p0, n_p) / (4.0 * math.pi)
    P = torch.as_tensor(points, dtype=torch.float64, device=dev)
    X = torch.as_tensor(np.asarray(xs, dtype=np.float64), device=dev)
    Y = torch.as_tensor(np.asarray(ys, dtype=np.float64), device=dev)
    Z = torch.as_tensor(np.asarray(zs, dtype=np.float64), device=dev)
    gx, gy, gz = torch.meshgrid(X, Y, Z, indexing="ij")
    tgt = torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], dim=1)
    out = torch.empty(tgt.shape[0], dtype=torch.complex128, device=dev)
    kr, ki = k1.real, k1.imag
    for s in range(0, tgt.shape[0], chunk):
        t = tgt[s:s + chunk]
        dx = t[:, 0:1] - P[None, :, 0]
        dy = t[:, 1:2] - P[None, :, 1]
        dz = t[:, 2:3] - P[None, :, 2]
        r = torch.sqrt(dx * dx + dy * dy + dz * dz)
        del dx, dy, dz
        amp = torch.exp(-ki * r) / r
        ph = kr * r
        re = (amp * torch.cos(ph)).sum(dim=1)
        im = (amp * torch.sin(ph)).sum(dim=1)
        out[s:s + chunk] = torch.complex(re, im) * pref
    return out.reshape(len(xs), len(ys), len(zs))


def oneil_on_axis(x, R, l, k, p0):
    """O'Neil's closed form for the cap's field on its axis (x measured from the apex)."""
    h = cap_height(R, l)
    x = np.asarray(x, dtype=np.float64)
    re = np.sqrt((x - h) ** 2 + R * R)
    return p0 * (np.exp(1j * k * x) - np.exp(1j * k * re)) / (1.0 - x / l)
