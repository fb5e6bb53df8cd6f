"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only)."""

import json
import math
import os

import numpy as np
import pytest

import oracle
from tests import closed_forms as cf
from workload import bowl, configs, fields

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
WATER = configs.WATER
F0 = 1.1e6


# ---------------------------------------------------------------- constants

def test_cascade_constants_match_printed_harmonic_equations():
    """C_n * sum_m p_m p_{n-m} reproduces the constants and source combinations of eqs. harm2-harm5."""
    rng = np.random.default_rng(0)
    p = {m: complex(*rng.standard_normal(2)) for m in range(1, 5)}
    w = 2 * math.pi * F0
    unit = WATER["beta"] * w * w / (WATER["rho0"] * WATER["c0"] ** 4)
    for n in range(2, 6):
        g = GOLDEN["cascade_constants"][str(n)]
        printed = -g["c"] * unit * sum(coef * p[i] * p[j] for coef, i, j in g["source"])
        got = oracle.cascade_constant(n, F0, WATER) * oracle.source_term(n, p)
        assert abs(got - printed) <= 1e-14 * abs(printed)


def test_attenuation_reading_and_spacings():
    # alpha0 = 0.2 dB/m at 1 MHz, eta = 2: 8.686 dB per neper
    a1 = oracle.attenuation(0.2, 2.0, 1.0e6)
    assert abs(a1 - 0.2 / 8.685889638065035) < 1e-15
    k = oracle.wavenumber(3, F0, WATER)
    assert abs(k.imag - 9 * oracle.attenuation(0.2, 2.0, F0)) < 1e-14
    # printed spacings (Section 5)
    for n, um in GOLDEN["mesh_spacing_um"].items():
        if n.startswith("_"):
            continue
        h = oracle.spacing(int(n), F0, WATER["c0"]) * 1e6
        assert abs(h - um) / um < 0.005


# ---------------------------------------------------------------- self cell

def test_self_cell_is_ball_integral_and_newtonian_limit():
    h = 1.1265e-4
    for k in (complex(9295.8, 0.11), complex(2 * 4647.9, 500.0), complex(23239.6, 0.7)):
        a = (3 / (4 * math.pi)) ** (1 / 3) * h
        ref = cf.ball_centre_integral(k, a)
        assert abs(oracle.self_cell(k, h) - ref) <= 1e-12 * abs(ref)
    # k -> 0: Newtonian a^2 / 2 plus the first-order term i k a^3 / 3
    a = (3 / (4 * math.pi)) ** (1 / 3)
    assert abs(oracle.self_cell(1e-4, 1.0) - (a * a / 2 + 1j * 1e-4 * a ** 3 / 3)) < 1e-8


def test_native_and_numpy_kernel_tables_agree():
    k = complex(9300.0, 2.0)
    h = 1e-4
    n = (5, 4, 3)
    ref = oracle.kernel_offsets(k, h, n)
    lib = oracle.core._load()
    import ctypes
    tab = np.empty(n, dtype=np.complex128)
    lib.oracle_kernel_table(oracle.core._i64arr(n), h, k.real, k.imag,
                            tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert np.max(np.abs(tab - ref)) <= 1e-14 * np.max(np.abs(ref))


# ---------------------------------------------------------------- operator

def test_direct_equals_circulant_fft_and_M_independence():
    f = fields.random_field((7, 6, 9), 11)
    k = complex(9295.8, 3.0)
    h = 1.1e-4
    d = oracle.conv_direct(f, h, k)
    for M in [(14, 12, 18), (13, 11, 17), (12, 10, 16), (20, 16, 25)]:
        c = oracle.conv_circulant(f, h, k, M=M)
        assert oracle.rel_l2(c, d) < 1e-13, M
    # the kernel is even, so M = 2n - 2 is still exact; M = 2n - 3 wraps around
    bad = oracle.conv_circulant(f, h, k, M=(11, 9, 15))
    assert oracle.rel_l2(bad, d) > 1e-3


def test_sampled_targets_equal_full_sum():
    f = fields.random_field((6, 5, 7), 3)
    k = complex(5000.0, 10.0)
    full = oracle.conv_direct(f, 2e-4, k)
    t = np.array([0, 17, 100, 209], dtype=np.int64)
    s = oracle.conv_direct(f, 2e-4, k, targets=t)
    assert np.array_equal(s, full.ravel()[t])


def test_reciprocity_linearity_translation():
    k = complex(9295.8, 1.0)
    h = 1e-4
    f = fields.random_field((6, 6, 6), 1)
    g = fields.random_field((6, 6, 6), 2)
    Af, Ag = oracle.conv_direct(f, h, k), oracle.conv_direct(g, h, k)
    # complex-symmetric (bilinear, no conjugate)
    lhs, rhs = np.sum(g * Af), np.sum(f * Ag)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # linearity
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    Alin = oracle.conv_direct(a * f + b * g, h, k)
    assert oracle.rel_l2(Alin, a * Af + b * Ag) < 1e-13
    # translation: a source shifted by one voxel gives a shifted potential in the interior
    s = np.zeros((8, 8, 8), dtype=np.complex128)
    s[1:5, 2:6, 1:5] = f[:4, :4, :4]
    s2 = np.zeros_like(s)
    s2[2:6, 2:6, 1:5] = f[:4, :4, :4]
    u1, u2 = oracle.conv_direct(s, h, k), oracle.conv_direct(s2, h, k)
    assert oracle.rel_l2(u2[1:, :, :], u1[:-1, :, :]) < 1e-13


def test_impulse_response_is_kernel():
    k = complex(9295.8, 1.0)
    h = 1e-4
    n = (5, 6, 7)
    f = np.zeros(n, dtype=np.complex128)
    j = (1, 4, 2)
    f[j] = 1.0
    u = oracle.conv_direct(f, h, k)
    K = oracle.kernel_offsets(k, h, (5, 6, 7))
    for i in [(0, 0, 0), (1, 4, 2), (4, 0, 6), (3, 5, 1)]:
        d = tuple(abs(i[a] - j[a]) for a in range(3))
        assert abs(u[i] - K[d]) <= 1e-14 * abs(K[d])
    # K(d) itself is h^3 G_k(|d| h), G from equation "green" written out here
    r = h * math.sqrt(3 * 3 + 4 * 4 + 4 * 4)
    g = h ** 3 * complex(math.cos(k.real * r), math.sin(k.real * r)) * math.exp(-k.imag * r) / (4 * math.pi * r)
    assert abs(u[4, 0, 6] - g) <= 1e-14 * abs(g)


def test_uniform_ball_converges_to_closed_form():
    """The voxelised ball potential approaches u = -V(r); staircase-limited convergence."""
    k = 2 * 4647.91 + 0.5j
    b, L = 1e-3, 3e-3
    # closed form checked against the radial quadrature
    r_chk = np.array([0.1e-3, 0.5e-3, 0.99e-3, 1.2e-3, 2.0e-3])
    rad = cf.radial_potential(lambda s: (s <= b).astype(float), k, r_chk, 2.5e-3, n_fine=400001)
    cfv = cf.ball_potential(r_chk, k, b)
    assert np.max(np.abs(rad - cfv)) < 2e-4 * np.max(np.abs(cfv))
    errs = []
    for N in (16, 24, 32, 48):
        h, r = cf.centred_grid(N, L)
        f = (r <= b).astype(np.complex128)
        u = oracle.volume_potential(f, h, k, method="fft")
        errs.append(oracle.rel_l2(u, -cf.ball_potential(r, k, b)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.03, errs


def test_gaussian_density_second_order():
    """Smooth radial source: the quadrature converges at second order (the paper's Section 3.3)."""
    k = 2 * 4647.91 + 0.5j
    sig, L = 0.4e-3, 3e-3
    gauss = lambda s: np.exp(-0.5 * (s / sig) ** 2)
    errs, hs = [], []
    for N in (16, 24, 32, 48):
        h, r = cf.centred_grid(N, L)
        f = gauss(r).astype(np.complex128)
        u = oracle.volume_potential(f, h, k, method="fft")
        ref = -cf.radial_potential(gauss, k, r.ravel(), 8e-3).reshape(r.shape)
        errs.append(oracle.rel_l2(u, ref))
        hs.append(h)
    order = math.log(errs[0] / errs[-1]) / math.log(hs[0] / hs[-1])
    assert order > 1.8, (errs, order)
    assert errs[-1] < 0.015


# ---------------------------------------------------------------- incident field input

def test_bowl_field_focus_exact_and_oneil_on_axis():
    R, l = 7.5e-3, 15e-3
    k = oracle.wavenumber(1, F0, WATER)
    p0 = 1e6
    h = bowl.cap_height(R, l)
    errs = []
    xs = np.linspace(l / 2, 1.5 * l, 41)
    xs = xs[np.abs(xs - l) > 1e-4]
    exact = bowl.oneil_on_axis(xs, R, l, k, p0)
    for n_p in (256, 1024, 4096):
        pts = bowl.bowl_points(R, l, n_p, seed=0)
        pf = bowl.incident_field(pts, R, l, k, p0, [l], [0.0], [0.0])[0, 0, 0].item()
        ref = -1j * k * h * p0 * np.exp(1j * k * l)
        assert abs(pf - ref) <= 1e-13 * abs(ref)
        pa = bowl.incident_field(pts, R, l, k, p0, xs, [0.0], [0.0])[:, 0, 0].numpy()
        errs.append(np.max(np.abs(pa - exact)) / abs(ref))
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8, errs
    # |p1(focus)| for the tiny configuration: |k| h p0 = 9.3406 MPa, less the attenuation over l
    assert abs(abs(ref) / 1e6 - 9.3406 * math.exp(-k.imag * l)) < 1e-4


def test_incident_oracle_focus_exact_and_oneil_on_axis():
    """The oracle's monopole sum: exact at the focus for any cap point set, O'Neil on the axis."""
    R, l = 7.5e-3, 15e-3
    k = oracle.wavenumber(1, F0, WATER)
    p0 = 1e6
    h = bowl.cap_height(R, l)
    ref = -1j * k * h * p0 * np.exp(1j * k * l)
    xs = np.linspace(l / 2, 1.5 * l, 41)
    xs = xs[np.abs(xs - l) > 1e-4]
    exact = bowl.oneil_on_axis(xs, R, l, k, p0)
    errs = []
    for n_p in (256, 1024, 4096):
        pts = bowl.bowl_points(R, l, n_p, seed=3)
        s = bowl.rayleigh_scale(R, l, k, p0, n_p)
        pf = oracle.incident_at(pts, k, s, [[l, 0.0, 0.0]])[0]
        assert abs(pf - ref) <= 1e-13 * abs(ref)
        tg = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1)
        errs.append(np.max(np.abs(oracle.incident_at(pts, k, s, tg) - exact)) / abs(ref))
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8, errs
    # the grid form evaluates the same sum at the grid's centres
    g = oracle.grid_from_counts((l, 0.0, 0.0), 1e-4, (3, 2, 4), (1, 1, 2))
    pts = bowl.bowl_points(R, l, 64, seed=1)
    s = bowl.rayleigh_scale(R, l, k, p0, 64)
    f = oracle.incident_field(pts, k, s, g)
    assert f.shape == (3, 2, 4)
    assert abs(f[1, 1, 2] - ref) <= 1e-13 * abs(ref)


def test_radiated_power_of_an_axial_monopole():
    """One monopole on the axis, a from the disc plane, lossless k: the disc integral of |p|^2 r
    is |s|^2 ln(1 + R^2 / a^2) / (16 pi), so the power is that over 2 rho0 c0.  The midpoint
    rule converges to it at second order."""
    a, R, rho0, c0 = 4e-3, 10e-3, 998.0, 1487.0
    k, s = 4647.9, 3.0 - 2.0j
    pts = np.array([[-a, 0.0, 0.0]])
    exact = abs(s) ** 2 * math.log(1.0 + (R / a) ** 2) / (16.0 * math.pi) / (2.0 * rho0 * c0)
    errs = []
    for n_r in (16, 32, 64):
        errs.append(abs(oracle.radiated_power(pts, k, s, (0.0, 0.0, 0.0), R, rho0, c0, n_r, 8) / exact - 1.0))
    assert errs[2] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs
    # the power scales with |s|^2 and does not depend on the phase of s
    p1 = oracle.radiated_power(pts, k, s, (0.0, 0.0, 0.0), R, rho0, c0, 32, 8)
    p2 = oracle.radiated_power(pts, k, 2j * s, (0.0, 0.0, 0.0), R, rho0, c0, 32, 8)
    assert abs(p2 / p1 - 4.0) < 1e-12


def test_vie_oracle_identity_and_born_series():
    """No contrast: p = rhs.  Contrast eps q: p = rhs + eps V[q rhs] + eps^2 V[q V[q rhs]] + O(eps^3),
    V the direct-sum volume potential."""
    n, h = (5, 4, 6), 1e-4
    kb = 2 * 4647.91 + 0.3j
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    q = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * abs(kb) ** 2
    assert np.allclose(oracle.vie_solve(np.zeros(n, complex), rhs, h, kb), rhs, rtol=0, atol=1e-14)
    b1 = oracle.conv_direct(q * rhs, h, kb)
    b2 = oracle.conv_direct(q * b1, h, kb)
    errs = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        p = oracle.vie_solve(eps * q, rhs, h, kb)
        r = (p - rhs - eps * b1 - eps ** 2 * b2) / np.max(np.abs(b2))
        errs.append(np.max(np.abs(r)) / eps ** 2)
    # the remainder after two Born terms is O(eps^3): it halves with eps (relative to eps^2)
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs
    # the dense operator is the direct sum
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    D = oracle.dense_operator(kb, h, n)
    assert np.allclose(D @ f.reshape(-1), oracle.conv_direct(f, h, kb).reshape(-1), rtol=1e-13, atol=0)


# ---------------------------------------------------------------- grids

def test_grid_builder_reproduces_printed_voxel_counts():
    c0 = WATER["c0"]
    # H131 in water: reference mesh at lambda_5/6 on the domain of equation "domain" (d = 9.8 mm)
    t = configs.H131
    lo, hi = oracle.reference_box(t["l"], t["R"], 9.8e-3)
    focus = (t["l"], 0.0, 0.0)
    g, _ = oracle.grid_from_box(focus, lo, hi, oracle.spacing(5, t["f0"], c0))
    printed = GOLDEN["h131_water_reference_mesh"]["n"]
    assert all(abs(a - b) <= 1 for a, b in zip(g.n, printed)), g.n
    # H101 in water, rule-of-thumb nested meshes (d = 10.5 mm) and the uniform mesh
    t = configs.H101
    focus = (t["l"], 0.0, 0.0)
    for n in range(2, 6):
        lo, hi = oracle.rule_of_thumb_box(n, t["l"], t["R"], 10.5e-3)
        g, _ = oracle.grid_from_box(focus, lo, hi, oracle.spacing(n, t["f0"], c0))
        printed = GOLDEN["h101_water_nested_voxels"][str(n)]
        assert abs(g.size() - printed) / printed < 0.006, (n, g.size())
    lo, hi = oracle.reference_box(t["l"], t["R"], 10.5e-3)
    g, _ = oracle.grid_from_box(focus, lo, hi, oracle.spacing(5, t["f0"], c0))
    assert abs(g.size() - 2.9e9) / 2.9e9 < 0.01


def test_grid_focus_is_a_voxel_centre():
    h = oracle.spacing(3, F0, WATER["c0"])
    g = oracle.grid_from_counts((0.15, 0.0, 0.0), h, (320, 256, 256), (128, 128, 128))
    i = oracle.focal_index(g, (0.15, 0.0, 0.0))
    assert i == (128, 128, 128)
    assert abs(g.coords(0)[128] - 0.15) < 1e-15


# ---------------------------------------------------------------- transfer

def _grid(origin, h, n):
    return oracle.Grid(origin, h, n)


def test_transfer_order1_equals_scipy_regular_grid_interpolator():
    from scipy.interpolate import RegularGridInterpolator
    src = _grid((0.01, -0.002, 0.003), 2e-4, (9, 8, 7))
    dst = _grid((0.0104, -0.0015, 0.0032), 0.7e-4, (15, 13, 11))
    f = fields.random_field(src.n, 5)
    got = oracle.transfer(f, src, dst, 1)
    axes = [src.coords(a) for a in range(3)]
    pts = np.stack(np.meshgrid(*[np.clip(dst.coords(a), axes[a][0], axes[a][-1]) for a in range(3)],
                               indexing="ij"), axis=-1)
    ref = (RegularGridInterpolator(axes, f.real, method="linear")(pts)
           + 1j * RegularGridInterpolator(axes, f.imag, method="linear")(pts))
    assert np.max(np.abs(got - ref)) < 1e-13


def test_transfer_reproduces_polynomials_and_matches_brute_force():
    src = _grid((0.0, 0.0, 0.0), 1e-3, (7, 6, 8))
    dst = _grid((-0.0007, 0.0002, 0.0009), 0.37e-3, (20, 15, 17))
    X, Y, Z = np.meshgrid(*[src.coords(a) for a in range(3)], indexing="ij")
    Xd, Yd, Zd = np.meshgrid(*[np.clip(dst.coords(a), src.coords(a)[0], src.coords(a)[-1])
                               for a in range(3)], indexing="ij")
    s = 1e3
    aff = lambda x, y, z: (1 + 2j) + 3 * s * x - 2j * s * y + 0.5 * s * z
    cub = lambda x, y, z: (s * x) ** 3 - 2j * (s * y) ** 2 * (s * z) + (s * z) ** 3 + 1j * s * x * s * y * s * z
    g1 = oracle.transfer(aff(X, Y, Z), src, dst, 1)
    assert np.max(np.abs(g1 - aff(Xd, Yd, Zd))) < 1e-12
    g3 = oracle.transfer(cub(X, Y, Z), src, dst, 3)
    assert np.max(np.abs(g3 - cub(Xd, Yd, Zd))) < 1e-10
    f = fields.random_field(src.n, 9)
    pts = [(dst.coords(0)[i], dst.coords(1)[j], dst.coords(2)[k])
           for i, j, k in [(0, 0, 0), (5, 3, 9), (19, 14, 16), (11, 7, 2)]]
    flat = [np.ravel_multi_index((i, j, k), dst.n) for i, j, k in [(0, 0, 0), (5, 3, 9), (19, 14, 16), (11, 7, 2)]]
    for order in (1, 3):
        sep = oracle.transfer(f, src, dst, order).ravel()[flat]
        bru = cf.lagrange_brute(f, src.origin, src.h, pts, order)
        assert np.max(np.abs(sep - bru)) < 1e-13


def test_transfer_identity_and_plane_wave_midpoint_attenuation():
    g = _grid((0.0, 0.0, 0.0), 1.0, (6, 6, 6))
    f = fields.random_field(g.n, 4)
    assert np.array_equal(oracle.transfer(f, g, _grid((0.0, 0.0, 0.0), 1.0, (6, 6, 6)), 3), f)
    # six points per wavelength, midpoints between source nodes, away from edges
    kh = math.pi / 3
    src = _grid((0.0, 0.0, 0.0), 1.0, (24, 4, 4))
    dst = _grid((8.5, 1.0, 1.0), 1.0, (4, 1, 1))
    x = src.coords(0)[:, None, None] * np.ones((1, 4, 4))
    pw = np.exp(1j * kh * x)
    exact = np.exp(1j * kh * dst.coords(0))
    lin = oracle.transfer(pw, src, dst, 1)[:, 0, 0]
    cub = oracle.transfer(pw, src, dst, 3)[:, 0, 0]
    assert np.allclose(np.abs(lin / exact), math.cos(kh / 2), atol=1e-14)
    assert np.allclose(np.abs(cub / exact), 9 / 8 * math.cos(kh / 2) - 1 / 8 * math.cos(3 * kh / 2), atol=1e-14)
    assert abs(1 - math.cos(kh / 2) - 0.134) < 1e-3


# ---------------------------------------------------------------- cascade

def test_tiny_nested_cascade_direct_equals_fft():
    R, l = 7.5e-3, 15e-3
    focus = (l, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (8, 8, 8), (4, 4, 4))
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(R, l, 128, 0)
    p1 = bowl.incident_field(pts, R, l, k1, 1e6, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    grids = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (8 + 2 * n, 10, 9), (6, 5, 4))
             for n in range(2, 6)}
    for order in (1, 3):
        a = oracle.cascade(p1, g1, grids, F0, WATER, order, method="direct")
        b = oracle.cascade(p1, g1, grids, F0, WATER, order, method="fft")
        for n in range(2, 6):
            assert oracle.rel_l2(b[n], a[n]) < 1e-12, (order, n)
    # harmonics decay in size down the cascade at this amplitude
    mags = [np.max(np.abs(a[n])) for n in range(2, 6)]
    assert np.max(np.abs(p1)) > mags[0] > mags[1]


@pytest.mark.parametrize("R,l", [(32e-3, 63.2e-3), (16.5e-3, 35e-3), (75e-3, 150e-3)])
def test_deserno_placement_on_the_cap(R, l):
    """Deserno's regular placement restricted to the bowl: about the requested count, every point
    on the sphere of radius l about the focus inside the aperture, near-equal spacing at the
    spacing an equal share of the area implies, and equal areas hold equal shares of points."""
    n = 4096
    pts = bowl.bowl_points_deserno(R, l, n)
    assert abs(len(pts) - n) <= 0.01 * n
    r = np.linalg.norm(pts - np.array([l, 0.0, 0.0]), axis=1)
    assert np.max(np.abs(r - l)) < 1e-12 * l
    assert np.all(np.hypot(pts[:, 1], pts[:, 2]) <= R * (1 + 1e-12))
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    np.fill_diagonal(d, np.inf)
    nn = d.min(axis=1)
    assert nn.min() / nn.mean() > 0.8 and nn.max() / nn.mean() < 1.1
    assert abs(nn.mean() / math.sqrt(bowl.cap_area(R, l) / len(pts)) - 1.0) < 0.05
    # the points above half the cap height: their share equals that sub-cap's share of the area
    half = bowl.cap_height(R, l) / 2
    assert abs(np.mean(pts[:, 0] <= half) - 0.5) < 0.02
