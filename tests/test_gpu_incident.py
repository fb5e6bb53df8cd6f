"""The incident field p_1 (Section 3.2, incident-field equation) on the GPU, through the C ABI.

The HIP kernel's monopole sums are compared with the FP64 oracle's (itself
pinned to the exact focal value and O'Neil's on-axis closed form) on small
grids over every voxel, and at the paper's scale (p1 on 128^3, 4096 points
on the 7.5 cm / 15 cm bowl) on seeded voxel samples.
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from workload import bowl, configs

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")

WATER = configs.WATER
TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.sync()
    c.close()


def run(ctx, pts, k, s, g, prec):
    d = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    out = P.incident_field(ctx, k, s, d, g, prec=prec)
    torch.cuda.synchronize()
    return out.to(torch.complex128).cpu().numpy()


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("n_p", [1, 5, 256, 1023])
def test_small_grid_every_voxel(ctx, prec, n_p):
    R, l, f0 = 7.5e-3, 15e-3, 1.1e6
    k = oracle.wavenumber(1, f0, WATER)
    pts = bowl.bowl_points(R, l, n_p, seed=2)
    s = bowl.rayleigh_scale(R, l, k, 1e6, n_p)
    g = oracle.grid_from_counts((l, 0.0, 0.0), oracle.spacing(1, f0, WATER["c0"]), (19, 13, 22), (9, 6, 11))
    say("case incident small n_p=%d prec=%d" % (n_p, prec))
    got = run(ctx, pts, k, s, g, prec)
    ref = oracle.incident_field(pts, k, s, g)
    assert oracle.rel_l2(got, ref) < TOL[prec]
    # the focus is a voxel centre: the exact cap value
    h = bowl.cap_height(R, l)
    exact = -1j * k * h * 1e6 * np.exp(1j * k * l)
    assert abs(got[9, 6, 11] - exact) < TOL[prec] * abs(exact) * 10


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_paper_scale_sampled(ctx, prec):
    """p1 of the paper-scale bowl on its 128^3 grid (4096 points), checked at 400 seeded voxels."""
    cfg = configs.paper_scale(P_f=2.0e6)
    W, f0 = cfg["medium"], cfg["f0"]
    k = oracle.wavenumber(1, f0, W)
    g = oracle.grid_from_counts((cfg["l"], 0.0, 0.0), oracle.spacing(1, f0, W["c0"]), cfg["p1_grid"]["n"],
                                cfg["p1_grid"]["i_f"])
    pts = bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])
    s = bowl.rayleigh_scale(cfg["R"], cfg["l"], k, cfg["p0"], cfg["n_points"])
    say("case incident paper scale prec=%d" % prec)
    got = run(ctx, pts, k, s, g, prec)
    rng = np.random.default_rng(11)
    idx = np.stack([rng.integers(0, n, 400) for n in g.n], axis=1)
    idx[0] = cfg["p1_grid"]["i_f"]
    tg = np.stack([g.coords(a)[idx[:, a]] for a in range(3)], axis=1)
    ref = oracle.incident_at(pts, k, s, tg)
    sub = got[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert oracle.rel_l2(sub, ref) < TOL[prec]
    # the focal pressure the configuration asks for
    assert abs(abs(sub[0]) / cfg["P_f"] - 1.0) < 0.02


def test_point_on_a_voxel_centre_and_errors(ctx):
    g = oracle.Grid((0.0, 0.0, 0.0), 1e-3, (4, 3, 5))
    pts = np.array([[1e-3, 1e-3, 2e-3], [5e-2, 0.0, 0.0]])
    got = run(ctx, pts, 100.0 + 1j, 1.0, g, P.NVP_C128)
    assert not np.isfinite(got[1, 1, 2])
    mask = np.ones(got.shape, bool)
    mask[1, 1, 2] = False
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = oracle.incident_field(pts, 100.0 + 1j, 1.0, g)
    assert np.all(np.isfinite(got[mask]))
    assert oracle.rel_l2(got[mask], ref[mask]) < 1e-12
    d = torch.from_numpy(pts).to("cuda")
    for kw in (dict(k=100.0 - 1j), dict(k=float("nan"))):
        with pytest.raises(P.NvpError) as e:
            P.incident_field(ctx, kw["k"], 1.0, d, g)
        assert e.value.status == 1
    with pytest.raises(P.NvpError) as e:
        P.incident_field(ctx, 1.0, 1.0, d, oracle.Grid((0.0, 0.0, 0.0), -1.0, (2, 2, 2)))
    assert e.value.status == 1
    with pytest.raises(ValueError):
        P.incident_field(ctx, 1.0, 1.0, d[:, :2].contiguous(), g)


@pytest.mark.parametrize("placement", ["spiral", "deserno"])
@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_arbitrary_targets(ctx, prec, placement):
    R, l, f0 = 32e-3, 63.2e-3, 1.1e6
    k = oracle.wavenumber(1, f0, WATER)
    pts = bowl.bowl_points(R, l, 777, seed=4) if placement == "spiral" else bowl.bowl_points_deserno(R, l, 777)
    s = bowl.rayleigh_scale(R, l, k, 1e5, len(pts))
    rng = np.random.default_rng(5)
    tg = np.stack([rng.uniform(5e-3, 80e-3, 333), rng.uniform(-30e-3, 30e-3, 333), rng.uniform(-30e-3, 30e-3, 333)], 1)
    say("case incident targets prec=%d placement=%s" % (prec, placement))
    got = P.incident_at(ctx, k, s, torch.from_numpy(pts).to("cuda"), torch.from_numpy(tg).to("cuda"), prec=prec)
    torch.cuda.synchronize()
    ref = oracle.incident_at(pts, k, s, tg)
    assert oracle.rel_l2(got.to(torch.complex128).cpu().numpy(), ref) < TOL[prec]


def test_radiated_power_and_normalisation(ctx):
    """The H101 bowl (l 63.2 mm, R 32 mm): the disc power of the GPU matches the oracle's on the same
    nodes, and scaling the field by sqrt(P0 / power) gives P0 = 100 W."""
    R, l, f0 = 32e-3, 63.2e-3, 1.1e6
    k = oracle.wavenumber(1, f0, WATER)
    n_p = 512
    pts = bowl.bowl_points(R, l, n_p, seed=0)
    s = bowl.cap_area(R, l) / n_p
    centre = (bowl.cap_height(R, l), 0.0, 0.0)
    d = torch.from_numpy(pts).to("cuda")
    say("case radiated power")
    got = P.radiated_power(ctx, k, s, d, centre, R, WATER["rho0"], WATER["c0"], 48, 64)
    ref = oracle.radiated_power(pts, k, s, centre, R, WATER["rho0"], WATER["c0"], 48, 64)
    assert abs(got / ref - 1.0) < 1e-11
    s100 = s * math.sqrt(100.0 / got)
    again = P.radiated_power(ctx, k, s100, d, centre, R, WATER["rho0"], WATER["c0"], 48, 64)
    assert abs(again - 100.0) < 1e-9
    with pytest.raises(P.NvpError):
        P.radiated_power(ctx, k, s, d, centre, -R, WATER["rho0"], WATER["c0"], 48, 64)
    with pytest.raises(P.NvpError):
        P.radiated_power(ctx, k, s, d, centre, R, WATER["rho0"], WATER["c0"], 0, 64)
