"""The source kernel (transfer + source term of Section 6 and equation
"cascade_2") through the C ABI against the FP64 oracle, on target grids of
several (y, z) tiles with ragged edges, for x chunks from one plane per
workgroup to the whole axis.

Lower harmonics on coarser grids (the cascade's case), on slightly finer
grids (more source planes than target planes along each axis) and on the
target grid itself; linear and cubic transfer.  Tolerance: relative L2 1e-5
in complex64, 1e-12 in complex128.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from workload import configs, fields

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2011_03009_amd")

WATER = configs.WATER
F0 = 1.1e6
TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}
DT = {P.NVP_C64: torch.complex64, P.NVP_C128: torch.complex128}
E_INVALID, E_UNSUPPORTED = 1, 4  # NVP_E_INVALID, NVP_E_UNSUPPORTED
FOCUS = (15e-3, 0.0, 0.0)
TARGET = (23, 19, 70)  # 3 x 3 tiles of 8 x 32 (y, z) columns, ragged in both


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(DT[prec])


def host(t):
    torch.cuda.synchronize()
    return t.to(torch.complex128).cpu().numpy()


def grids(case):
    """g1 and the grids of p2..p4; p4 (three lower fields) is the target of the widest case."""
    h4 = oracle.spacing(4, F0, WATER["c0"])
    tgt = oracle.grid_from_counts(FOCUS, h4, TARGET, (11, 9, 35))
    if case == "coarser":  # lambda_m / 6 for p_m: ratios 1/4, 2/4, 3/4
        lower = [oracle.grid_from_counts(FOCUS, h4 * 4 / m, (9 + 4 * m, 12, 30), (5 + 2 * m, 6, 15))
                 for m in (1, 2, 3)]
    elif case == "finer":  # spacing h4 / 1.05: a source plane more every 20 target planes
        lower = [oracle.grid_from_counts(FOCUS, h4 / 1.05, (27, 23, 78), (13, 11, 39)) for _ in (1, 2, 3)]
    else:  # mixed: p1 coarser, p2 and p3 on the target grid of p4 ... and of each other
        lower = [oracle.grid_from_counts(FOCUS, h4 * 4, (13, 12, 30), (7, 6, 15)), tgt, tgt]
    return lower[0], [lower[1], lower[2], tgt]


@pytest.mark.parametrize("prec", [P.NVP_C64, P.NVP_C128])
@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("case", ["coarser", "finer", "mixed"])
def test_source_kernel_every_chunk_matches_oracle(ctx, case, order, prec):
    g1, gn = grids(case)
    g = [g1] + gn
    flds = [fields.smooth_field(gm.n, 40 + m) * 10 ** (5 - m) + 1e-3 * fields.random_field(gm.n, 50 + m)
            for m, gm in enumerate(g, start=1)]
    plan = P.CascadePlan(ctx, WATER, F0, g1, gn, prec=prec, order=order)
    try:
        for n in (2, 3, 4):
            v = {m: oracle.transfer(flds[m - 1], g[m - 1], g[n - 1], order) for m in range(1, n)}
            ref = oracle.source_term(n, v)
            for cx in (0, 1, 3, 7, 64):
                say("case source case=%s n=%d order=%d prec=%d cx=%d" % (case, n, order, prec, cx))
                plan.set_tuning(n, src=1, src_cx=cx)
                assert plan.tuning(n)["src_cx"] == cx
                f = host(plan.source_term(n, [dev(flds[m - 1], prec) for m in range(1, n)]))
                assert oracle.rel_l2(f, ref) < TOL[prec], (case, n, cx)
    finally:
        plan.close()


def test_set_tuning_rejects_bad_choices(ctx):
    g1, gn = grids("coarser")
    plan = P.CascadePlan(ctx, WATER, F0, g1, gn, prec=P.NVP_C64, order=3)
    try:
        for bad in (dict(x_tile=2), dict(quads=3), dict(src=2), dict(src_cx=65), dict(src_cx=-1)):
            with pytest.raises(P.NvpError) as e:
                plan.set_tuning(2, **bad)
            assert e.value.status == E_INVALID
        with pytest.raises(P.NvpError):
            plan.set_tuning(5, src=1)
    finally:
        plan.close()
    # source planes three times denser than the target: the blocks exceed the kernel's
    # per-thread loads, so only the fused path takes these grids
    h = oracle.spacing(2, F0, WATER["c0"])
    g1 = oracle.grid_from_counts(FOCUS, h / 3, (60, 60, 200), (30, 30, 100))
    g2 = oracle.grid_from_counts(FOCUS, h, (18, 17, 60), (9, 8, 30))
    plan = P.CascadePlan(ctx, WATER, F0, g1, [g2], prec=P.NVP_C64, order=3)
    try:
        with pytest.raises(P.NvpError) as e:
            plan.set_tuning(2, src=1)
        assert e.value.status == E_UNSUPPORTED
        plan.set_tuning(2, src=0)
        assert plan.tuning(2)["src"] == 0
    finally:
        plan.close()


@pytest.mark.parametrize("prec", [P.NVP_C64, P.NVP_C128])
def test_source_kernel_up_to_seven_fields(ctx, prec):
    """Harmonics 6..8, the source term of five to seven lower fields (the most the library takes),
    each p_m on its own coarser grid at lambda_m / 6.  In complex64 the kernel with a wavefront per
    field runs them; in complex128 a field's LDS share of the streamed kernel allows at most four
    fields, so these grids take the fused path and the source-term call reports it."""
    h8 = oracle.spacing(8, F0, WATER["c0"])
    n8 = (21, 17, 45)
    tgt = oracle.grid_from_counts(FOCUS, h8, n8, tuple(v // 2 for v in n8))
    g = []
    for m in range(1, 8):
        cnt = tuple(-(-v * m // 8) + 4 for v in n8)
        g.append(oracle.grid_from_counts(FOCUS, h8 * 8 / m, cnt, tuple(v // 2 for v in cnt)))
    g.append(tgt)
    flds = [fields.smooth_field(gm.n, 60 + m) * 10 ** (3 - 0.5 * m) + 1e-3 * fields.random_field(gm.n, 70 + m)
            for m, gm in enumerate(g, start=1)]
    plan = P.CascadePlan(ctx, WATER, F0, g[0], g[1:], prec=prec, order=3)
    try:
        for n in (6, 7, 8):
            args = [dev(flds[m - 1], prec) for m in range(1, n)]
            if prec == P.NVP_C128:
                say("case source many-fields n=%d prec=%d expect unsupported" % (n, prec))
                with pytest.raises(P.NvpError) as e:
                    plan.source_term(n, args)
                assert e.value.status == E_UNSUPPORTED
                continue
            v = {m: oracle.transfer(flds[m - 1], g[m - 1], g[n - 1], 3) for m in range(1, n)}
            ref = oracle.source_term(n, v)
            for cx in (0, 1):
                say("case source many-fields n=%d prec=%d cx=%d" % (n, prec, cx))
                plan.set_tuning(n, src=1, src_cx=cx)
                f = host(plan.source_term(n, args))
                assert oracle.rel_l2(f, ref) < TOL[prec], (n, cx)
    finally:
        plan.close()
