"""The full harmonic cascade on the GPU: the difference-frequency kernel and the fixed-point
sweeps against the oracle."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import full_cascade as FC
from workload import bowl, configs, fields

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")
from paper_2011_03009_amd import full_cascade as GF  # noqa: E402

WATER = configs.WATER
F0 = 1.1e6
DT = {P.NVP_C64: torch.complex64, P.NVP_C128: torch.complex128}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.sync()
    c.close()


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(DT[prec])


def host(t):
    torch.cuda.synchronize()
    return t.to(torch.complex128).cpu().numpy()


GT = oracle.Grid((0.010, -0.0012, 0.0009), 2.0e-4, (13, 11, 12))
CASES = {
    # a: finer and inside the target (zero outside), b: coarser and larger (clamped)
    "fine-inside/coarse": (oracle.Grid((0.0112, -0.0006, 0.0015), 1.0e-4, (17, 13, 14)), True,
                           oracle.Grid((0.0095, -0.0020, 0.0001), 3.0e-4, (11, 10, 10)), False),
    # a: finer, partly outside the target; b: the target grid itself
    "fine-partial/identity": (oracle.Grid((0.0085, -0.0016, 0.0021), 0.667e-4, (40, 21, 19)), True, GT, False),
    # both zero outside, both partial
    "both-zero": (oracle.Grid((0.0113, -0.0005, 0.0019), 1.5e-4, (9, 8, 12)), True,
                  oracle.Grid((0.0091, -0.0019, 0.0012), 0.5e-4, (30, 25, 28)), True),
}


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("case", sorted(CASES))
def test_difference_term_matches_oracle(ctx, case, order, prec):
    ga, za, gb, zb = CASES[case]
    a = fields.random_field(ga.n, 3)
    b = fields.random_field(gb.n, 4)
    o = fields.random_field(GT.n, 5)
    say("case difference term %s order=%d prec=%d" % (case, order, prec))
    out = dev(o, prec)
    P.difference_term(ctx, GT, out, ga, dev(a, prec), za, gb, dev(b, prec), zb, order, 2.0)
    ref = o + FC.difference_term(GT, a, ga, za, b, gb, zb, order, 2.0)
    tol = 1e-13 if prec == P.NVP_C128 else 2e-6
    assert oracle.rel_l2(host(out), ref) < tol


def test_difference_term_rejects_bad_arguments(ctx):
    t = torch.zeros(GT.n, dtype=torch.complex128, device="cuda")
    for kw in (dict(order=2), dict(alias=True)):
        with pytest.raises(P.NvpError):
            P.difference_term(ctx, GT, t, GT, t if kw.get("alias") else t.clone(), False, GT, t.clone(), False,
                              kw.get("order", 1), 1.0)
    short = oracle.Grid((0.0, 0.0, 0.0), 1e-4, (3, 3, 3))
    with pytest.raises(P.NvpError):
        P.difference_term(ctx, GT, t, short, torch.zeros(short.n, dtype=torch.complex128, device="cuda"), True,
                          GT, t.clone(), False, 3, 1.0)


def tiny(amplitude, N=3):
    focus = (15e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (10, 9, 8), (5, 4, 4))
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (8 + 2 * n, 11, 10), (6, 5, 4))
          for n in range(2, N + 1)}
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(7.5e-3, 15e-3, 128, 1)
    p1 = bowl.incident_field(pts, 7.5e-3, 15e-3, k1, amplitude, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    return g1, gn, p1


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("order", [1, 3])
def test_full_cascade_matches_oracle(ctx, order, prec):
    g1, gn, p1 = tiny(3e6, N=4)
    say("case full cascade order=%d prec=%d" % (order, prec))
    tol = 1e-12 if prec == P.NVP_C128 else 1e-6
    p, sweeps, change, paper = GF.full_cascade(ctx, WATER, F0, g1, [gn[n] for n in sorted(gn)], dev(p1, prec),
                                               order=order, tol=tol)
    ref, rs, rc = FC.full_cascade(p1, g1, gn, F0, WATER, order, tol=1e-13)
    assert change <= tol
    for n in range(1, 5):
        assert oracle.rel_l2(host(p[n - 1]), ref[n]) < (1e-10 if prec == P.NVP_C128 else 1e-5), n
    # the dropped terms change every harmonic by more than the comparison's tolerance
    base = oracle.cascade(p1, g1, gn, F0, WATER, order)
    for n in range(2, 5):
        assert oracle.rel_l2(ref[n], base[n]) > 1e-4, n
