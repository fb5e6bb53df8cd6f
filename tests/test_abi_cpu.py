"""The C ABI on the host: the library loads, exports every declared symbol, and its
host-side arithmetic (constants, grids, transfer tables) agrees with the oracle."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from workload import configs

P = pytest.importorskip("paper_2011_03009_amd")
from paper_2011_03009_amd import _native  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WATER = configs.WATER
F0 = 1.1e6


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nvp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nvp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_native.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding declares each of them
    assert set(syms) == set(_native.SIGNATURES)


def test_constants_equal_oracle():
    for n in range(1, 6):
        assert P.wavenumber(WATER, F0, n) == oracle.wavenumber(n, F0, WATER)
        assert abs(P.cascade_constant(WATER, F0, n) - oracle.cascade_constant(n, F0, WATER)) <= \
            1e-15 * abs(oracle.cascade_constant(n, F0, WATER))
        assert P.spacing(WATER, F0, n) == oracle.spacing(n, F0, WATER["c0"])


def test_grid_builders_bit_exact_against_oracle():
    for t, d in ((configs.H101, 10.5e-3), (configs.H131, 9.8e-3)):
        focus = (t["l"], 0.0, 0.0)
        for n in range(2, 6):
            lo, hi = P.rule_of_thumb_box(n, t["l"], t["R"], d)
            olo, ohi = oracle.rule_of_thumb_box(n, t["l"], t["R"], d)
            assert lo == olo and hi == ohi
            h = P.spacing(WATER, t["f0"], n)
            g, i_f = P.grid_from_box(focus, lo, hi, h)
            og, oi_f = oracle.grid_from_box(focus, olo, ohi, h)
            assert tuple(g.n) == og.n and tuple(g.origin) == og.origin and g.h == og.h and i_f == oi_f
    g = P.grid_from_counts((0.15, 0.0, 0.0), 7.5e-5, (320, 256, 256), (128, 128, 128))
    og = oracle.grid_from_counts((0.15, 0.0, 0.0), 7.5e-5, (320, 256, 256), (128, 128, 128))
    assert tuple(g.origin) == og.origin and tuple(g.n) == og.n


@pytest.mark.parametrize("order", [1, 3])
def test_transfer_tables_bit_exact_indices(order):
    cfg = configs.paper_scale()
    c0 = WATER["c0"]
    focus = (cfg["l"], 0.0, 0.0)
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), cfg["p1_grid"]["n"], cfg["p1_grid"]["i_f"])
    grids = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), s["n"], s["i_f"])
             for n, s in cfg["grids"].items()}
    pairs = [(g1, grids[n]) for n in range(2, 6)] + [(grids[m], grids[n]) for n in range(3, 6) for m in range(2, n)]
    # plus a coincident-node case and clamping on both sides
    pairs.append((oracle.Grid((0.0, 0.0, 0.0), 0.3, (9, 9, 9)), oracle.Grid((-0.45, 0.0, 0.15), 0.1, (40, 9, 9))))
    for src, dst in pairs:
        for a in range(3):
            b, w = P.nvp.transfer_axis(dst.origin[a], dst.h, dst.n[a], src.origin[a], src.h, src.n[a], order)
            ob, ow = oracle.transfer_axis(dst.origin[a], dst.h, dst.n[a], src.origin[a], src.h, src.n[a], order)
            assert np.array_equal(b.astype(np.int64), ob)
            assert np.max(np.abs(w - ow)) <= 1e-15


def test_circulant_sizes():
    lengths = P.transform_lengths()
    assert lengths == sorted(lengths) and lengths[0] == 16 and lengths[-1] == 8192
    for L in lengths:  # even and 2,3,5,7-smooth, each with a radix plan
        r = L
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        assert r == 1 and L % 8 == 0, L
    for n in range(1, 4097):
        m = P.circulant_size(n)
        assert m >= 2 * n - 1 and m % 2 == 0 and m in lengths
        # the smallest compiled length that embeds the axis (Section 3.1: any M >= 2n - 1 is exact)
        assert not [L for L in lengths if 2 * n - 1 <= L < m]
        if n >= 128:
            assert m <= 1.125 * (2 * n - 1), (n, m)
    assert P.circulant_size(640) == 1280 and P.circulant_size(641) == 1344 and P.circulant_size(769) == 1728
    # the paper's H101 nested meshes (576..716 x 568^2)
    assert [P.circulant_size(n) for n in (568, 576, 623, 669, 716)] == [1152, 1152, 1280, 1344, 1440]
    with pytest.raises(P.NvpError) as e:
        P.circulant_size(4097)
    assert e.value.status == 4
    for n in (0, -3):  # empty or negative axes
        with pytest.raises(P.NvpError):
            P.circulant_size(n)


def test_host_calls_reject_invalid_arguments():
    L = _native.lib()
    m = _native.Medium(1487.0, 998.0, 3.5, 0.2, 2.0)
    out = ctypes.c_double()
    assert L.nvp_cascade_constant(ctypes.byref(m), 1.1e6, 0, ctypes.byref(out)) == 1
    assert L.nvp_spacing(ctypes.byref(m), -1.0, 2, 6, ctypes.byref(out)) == 1
    bad = _native.Medium(float("nan"), 998.0, 3.5, 0.2, 2.0)
    assert L.nvp_wavenumber(ctypes.byref(bad), 1.1e6, 2, ctypes.byref(out), ctypes.byref(out)) == 1
    b = (ctypes.c_int32 * 4)()
    w = (ctypes.c_double * 16)()
    assert L.nvp_transfer_axis(0.0, 1.0, 4, 0.0, 1.0, 3, 3, b, w) == 1  # source too short for order 3
    assert L.nvp_transfer_axis(0.0, 1.0, 4, 0.0, 1.0, 8, 2, b, w) == 1  # unsupported order
    assert L.nvp_ctx_create(0, None, None) == 1
    assert L.nvp_status_str(4) == b"unsupported"


def test_h101_nested_grids_match_the_paper():
    """The rule-of-thumb boxes of H101 (1.1 MHz, l 63.2 mm, R 32 mm, d 10.5 mm) at lambda_n / 6 in water:
    the paper prints 1.86, 2.01, 2.15 and 2.30 x 10^8 voxels for p2..p5, and 2.9 x 10^9 for one mesh
    of the reference domain at lambda_5 / 6."""
    W = dict(c0=1487.0, rho0=998.0, beta=3.5, alpha0_db=0.2, eta=2.0)
    f0, l, R, d = 1.1e6, 63.2e-3, 32e-3, 10.5e-3
    counts = []
    for n in range(2, 6):
        g, _ = P.grid_from_box((l, 0.0, 0.0), *P.rule_of_thumb_box(n, l, R, d), P.spacing(W, f0, n))
        counts.append(int(g.n[0]) * int(g.n[1]) * int(g.n[2]))
    assert [round(c / 1e8, 2) for c in counts] == [1.86, 2.01, 2.16, 2.31]
    for printed, c in zip((1.86e8, 2.01e8, 2.15e8, 2.30e8), counts):
        assert abs(c / printed - 1.0) < 0.005
    g, _ = P.grid_from_box((l, 0.0, 0.0), *P.rule_of_thumb_box(2, l, R, d), P.spacing(W, f0, 5))
    assert abs(int(g.n[0]) * int(g.n[1]) * int(g.n[2]) / 2.9e9 - 1.0) < 0.01


def test_quadrature_weights_equal_oracle():
    """The library's self and face weights of both rules against the oracle's (whose lattice
    zeta values come from its own Ewald sums)."""
    for k, h in ((1.05 + 0.01j, 1.0), (4651.7 + 2.9j, 2.25e-4), (0.2 + 0.0j, 3.0)):
        s, f = P.quadrature_weights(P.NVP_QUAD_BALL, k, h)
        assert s == pytest.approx(oracle.self_cell(k, h), rel=1e-13) and f == 0
        s, f = P.quadrature_weights(P.NVP_QUAD_CORRECTED, k, h)
        ws, wf = oracle.corrected_weights(k, h)
        assert s == pytest.approx(ws, rel=1e-13)
        assert f == pytest.approx(wf, rel=1e-13)
    for bad in ((2, 1.0, 1.0), (-1, 1.0, 1.0), (1, 0.0, 1.0), (1, 1.0, 0.0), (0, float("nan"), 1.0)):
        with pytest.raises(P.NvpError):
            P.quadrature_weights(bad[0], bad[1], bad[2])
