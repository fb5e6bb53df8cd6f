"""Precision sweep on the paper-scale geometry (every harmonic on a 96^3 box per harmonic).

p2..p5 of the 7.5 cm / 15 cm bowl at 1.1 MHz and 5 MPa focal pressure, each on
96^3 voxels at lambda_n/6 around the focus (p1 on 96^3 at lambda_1/6), cubic
transfer.  The complex64 path (FFTs and pointwise work in FP32, kernel spectrum
in FP64 then downcast) and the all-FP64 path are compared with the FP64
oracle's cascade (its circulant form, itself pinned to the direct sum) over
every voxel: relative L2 error and focal-pressure error per harmonic.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from workload import bowl, configs

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")

TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}
DT = {P.NVP_C64: torch.complex64, P.NVP_C128: torch.complex128}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    cfg = configs.precision_subbox(P_f=5.0e6, side=96)
    W, f0 = cfg["medium"], cfg["f0"]
    focus = (cfg["l"], 0.0, 0.0)
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, f0, W["c0"]), cfg["p1_grid"]["n"], cfg["p1_grid"]["i_f"])
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, f0, W["c0"]), s["n"], s["i_f"])
          for n, s in cfg["grids"].items()}
    k1 = oracle.wavenumber(1, f0, W)
    pts = bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])
    p1 = bowl.incident_field(pts, cfg["R"], cfg["l"], k1, cfg["p0"], g1.coords(0), g1.coords(1), g1.coords(2),
                             device="cuda", chunk=8192).cpu().numpy()
    say("precision sweep: oracle cascade on 96^3 (circulant form)")
    ref = oracle.cascade(p1, g1, gn, f0, W, 3, method="fft")
    return cfg, g1, gn, p1, ref


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.sync()
    c.close()


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_precision_sweep_subbox(ctx, setup, prec):
    cfg, g1, gn, p1, ref = setup
    say("case precision sweep prec=%d" % prec)
    plan = P.CascadePlan(ctx, cfg["medium"], cfg["f0"], g1, [gn[n] for n in range(2, 6)], prec=prec, order=3)
    outs = plan.execute(torch.from_numpy(p1).to("cuda", DT[prec]))
    torch.cuda.synchronize()
    i_f = tuple(cfg["grids"][2]["i_f"])
    for n in range(2, 6):
        got = outs[n - 2].to(torch.complex128).cpu().numpy()
        e = oracle.rel_l2(got, ref[n])
        ef = abs(got[i_f] - ref[n][i_f]) / abs(ref[n][i_f])
        say("  p%d %s: rel L2 %.3e, focal error %.3e (|p%d(focus)| = %.4e Pa)"
            % (n, "c64" if prec == P.NVP_C64 else "c128", e, ef, n, abs(ref[n][i_f])))
        assert e < TOL[prec], n
        assert ef < TOL[prec], n
    plan.close()
