"""Physical configurations of the synthetic workloads.

Each configuration is plain data: medium constants, transducer geometry,
source amplitude, and per-harmonic voxel counts with the index of the voxel
that sits on the geometric focus.  Spacings (six voxels per own wavelength)
and origins are derived from these by the grid builders of the library and of
the oracle, not here.

Medium: water with c0 = 1487 m/s (the sound speed that reproduces the paper's
printed mesh spacings of 45.1 um and 113 um in its Section 5), rho0 = 998,
beta = 3.5, and the water attenuation of the paper's medium table
(alpha0 = 0.2 dB/m at 1 MHz, power-law exponent 2).
"""

WATER = dict(c0=1487.0, rho0=998.0, beta=3.5, alpha0_db=0.2, eta=2.0)
# Liver as the paper's table of media gives it (alpha0 in dB/m at 1 MHz, power-law exponent eta).
LIVER = dict(c0=1590.0, rho0=1060.0, beta=4.4, alpha0_db=90.0, eta=1.1)

# The two transducers of the paper's transducer table (f0 in Hz, lengths in m).
H101 = dict(f0=1.1e6, l=63.2e-3, R=32e-3)
H131 = dict(f0=1.1e6, l=35e-3, R=16.5e-3)

# Tiny plain-method case: bowl R = 7.5 mm, l = 15 mm, 256 surface points,
# 1 MPa surface pressure; p1 and p2 both on one 32^3 grid at lambda_2/6 whose
# voxel 16 (per axis) is the focus; circulant size 64^3.
CFG_TINY = dict(
    name="tiny-32",
    medium=WATER, f0=1.1e6, R=7.5e-3, l=15e-3, n_points=256, seed=0, p0=1.0e6,
    n_harm=2,
    p1_grid=dict(n=(32, 32, 32), i_f=(16, 16, 16), spacing_harmonic=2),
    grids={2: dict(n=(32, 32, 32), i_f=(16, 16, 16))},
)


def focal_to_surface_pressure(P_f, R, l, f0, c0):
    """Surface pressure p0 that gives focal amplitude P_f for an ideal bowl.

    The on-axis closed form of a spherical cap gives |p(focus)| = k h p0 with
    h = l - sqrt(l^2 - R^2) the cap height and k = 2 pi f0 / c0 (attenuation
    neglected in this amplitude choice only).
    """
    import math
    h = l - math.sqrt(l * l - R * R)
    k = 2.0 * math.pi * f0 / c0
    return P_f / (k * h)


def paper_scale(P_f=3.5e6, n_points=4096, seed=0):
    """Paper-scale homogeneous run: bowl R = 7.5 cm, l = 15 cm, 1.1 MHz, 5 harmonics.

    p1 lives on 128^3 at lambda_1/6 (focus at voxel 64).  Harmonic n >= 2
    lives on (64 (n+2), 256, 256) voxels at lambda_n/6 with the focus at voxel
    128 on every axis: the pre-focal length and the width scale with the
    wavelength while the post-focal distance stays fixed (the paper's rule of
    thumb for nested domains).  The uniform baseline puts every harmonic on
    640^3 at lambda_5/6 (focus at voxel 320).
    """
    R, l, f0 = 75e-3, 150e-3, 1.1e6
    p0 = focal_to_surface_pressure(P_f, R, l, f0, WATER["c0"])
    nested = {n: dict(n=(64 * (n + 2), 256, 256), i_f=(128, 128, 128)) for n in range(2, 6)}
    uniform = {n: dict(n=(640, 640, 640), i_f=(320, 320, 320), spacing_harmonic=5)
               for n in range(2, 6)}
    return dict(
        name="paper-scale-nested",
        medium=WATER, f0=f0, R=R, l=l, n_points=n_points, seed=seed, p0=p0, P_f=P_f,
        n_harm=5,
        p1_grid=dict(n=(128, 128, 128), i_f=(64, 64, 64), spacing_harmonic=1),
        grids=nested,
        uniform_grids=uniform,
    )


def precision_subbox(P_f=5.0e6, n_points=4096, seed=0, side=96):
    """Precision sweep geometry: the paper-scale bowl on a side^3 box per harmonic.

    Every harmonic n lives on side^3 voxels at lambda_n/6 with the focus at
    voxel side/2; p1 on side^3 at lambda_1/6.
    """
    cfg = paper_scale(P_f=P_f, n_points=n_points, seed=seed)
    half = side // 2
    cfg["name"] = "precision-subbox-%d" % side
    cfg["p1_grid"] = dict(n=(side,) * 3, i_f=(half,) * 3, spacing_harmonic=1)
    cfg["grids"] = {n: dict(n=(side,) * 3, i_f=(half,) * 3) for n in range(2, 6)}
    cfg.pop("uniform_grids")
    return cfg


def batch_transducers(count=64, seed=0):
    """Seeded transducers of the batched workload: aperture radius 2-8 cm, focal length 4-16 cm,
    0.5-1.5 MHz, surface pressure 0.2-1.5 MPa, 3-5 harmonics (uniform draws; a draw with
    R > 0.8 l, which is no usable bowl, is drawn again).

    Returns a list of dicts with keys R, l, f0, p0, n_harm.
    """
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        R, l = rng.uniform(0.02, 0.08), rng.uniform(0.04, 0.16)
        f0, p0, nh = rng.uniform(0.5e6, 1.5e6), rng.uniform(0.2e6, 1.5e6), int(rng.integers(3, 6))
        if R > 0.8 * l:
            continue
        out.append(dict(R=R, l=l, f0=f0, p0=p0, n_harm=nh))
    return out
