"""Batches of cascades, their HIP graph and the autotuner, through the C ABI.

A batch computes exactly what its problems' own plans compute (same kernels,
same order per problem): outputs are compared bitwise.  Graph replays are
compared bitwise with the eager run, with unrelated eager work between them.
A tuned plan is compared with the FP64 oracle at the usual tolerances.
"""

import os
import sys

import numpy as np
import pytest
import torch

import oracle
from workload import configs, fields

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")

WATER = configs.WATER
TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}
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


def problems(count, seed):
    """Uneven small nested problems: f0, focal distance, harmonic count and box counts vary."""
    rng = np.random.default_rng(seed)
    out = []
    c0 = WATER["c0"]
    for i in range(count):
        f0 = float(rng.uniform(0.5e6, 1.5e6))
        nh = int(rng.integers(3, 6))
        focus = (float(rng.uniform(0.04, 0.12)), 0.0, 0.0)
        n1 = tuple(int(v) for v in rng.integers(8, 20, 3))
        g1 = oracle.grid_from_counts(focus, oracle.spacing(1, f0, c0), n1, tuple(v // 2 for v in n1))
        gn = []
        for n in range(2, nh + 1):
            c = tuple(int(v) for v in rng.integers(6, 40, 3))
            gn.append(oracle.grid_from_counts(focus, oracle.spacing(n, f0, c0), c, tuple(v // 2 for v in c)))
        out.append(dict(med=WATER, f0=f0, g1=g1, grids=gn))
    return out


def inputs(probs, prec, seed):
    return [dev(fields.smooth_field(tuple(p["g1"].n), seed + i) * 1e6, prec) for i, p in enumerate(probs)]


def same(a, b):
    return all(torch.equal(x, y) for xs, ys in zip(a, b) for x, y in zip(xs, ys))


@pytest.mark.parametrize("prec", [P.NVP_C64, P.NVP_C128])
def test_batch_eager_matches_individual_plans(ctx, prec):
    probs = problems(7, 1)
    p1s = inputs(probs, prec, 10)
    say("case batch eager prec=%d" % prec)
    b = P.Batch(ctx, probs, prec=prec, order=3)
    b.set_graph(False)
    outs = b.execute(p1s, b.outputs())
    for i, pr in enumerate(probs):
        plan = P.CascadePlan(ctx, pr["med"], pr["f0"], pr["g1"], pr["grids"], prec=prec, order=3)
        ref = plan.execute(p1s[i])
        torch.cuda.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(outs[i], ref)), i
        plan.close()
    b.close()


@pytest.mark.parametrize("branches", [1, 4, 16])
def test_batch_graph_replays_match_eager(ctx, branches):
    probs = problems(9, 2)
    p1s = inputs(probs, P.NVP_C64, 20)
    say("case batch graph branches=%d" % branches)
    b = P.Batch(ctx, probs, prec=P.NVP_C64, order=1)
    b.set_graph(False)
    ref = [[t.clone() for t in o] for o in b.execute(p1s, b.outputs())]
    b.set_graph(True, branches)
    outs = b.outputs()
    b.execute(p1s, outs)  # eager warm-up run of the graph mode
    torch.cuda.synchronize()
    assert same(outs, ref)
    junk = torch.randn(1 << 20, device="cuda")
    for r in range(4):
        for o in outs:
            for t in o:
                t.zero_()
        b.execute(p1s, outs)  # captured on the first of these, then replayed
        junk = junk * 1.0001 + 1.0  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert same(outs, ref), r
    # new buffers: the graph is recorded again
    outs2 = b.outputs()
    b.execute(p1s, outs2)
    torch.cuda.synchronize()
    assert same(outs2, ref)
    b.close()


@pytest.mark.parametrize("prec", [P.NVP_C64, P.NVP_C128])
def test_autotuned_plan_matches_oracle_and_cache_round_trips(ctx, prec, tmp_path):
    focus = (15e-3, 0.0, 0.0)
    f0, c0 = 1.1e6, WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, f0, c0), (10, 9, 8), (5, 4, 4))
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, f0, c0), (8 + 2 * n, 11, 10), (6, 5, 4))
          for n in range(2, 5)}
    p1 = fields.smooth_field(g1.n, 5) * 1e6
    cache = str(tmp_path / "tune.txt")
    say("case autotune prec=%d" % prec)
    plan = P.CascadePlan(ctx, WATER, f0, g1, [gn[n] for n in range(2, 5)], prec=prec, order=3)
    plan.autotune(cache, reps=2)
    choices = [plan.tuning(n) for n in range(2, 5)]
    outs = plan.execute(dev(p1, prec))
    ref = oracle.cascade(p1, g1, gn, f0, WATER, 3, method="direct")
    torch.cuda.synchronize()
    for n in range(2, 5):
        got = outs[n - 2].to(torch.complex128).cpu().numpy()
        assert oracle.rel_l2(got, ref[n]) < TOL[prec], n
    plan.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 3 and all(len(l.split()) == 6 for l in lines)
    # a plan of the same shapes takes its choices from the cache
    plan2 = P.CascadePlan(ctx, WATER, f0, g1, [gn[n] for n in range(2, 5)], prec=prec, order=3)
    plan2.autotune(cache, reps=2)
    assert [plan2.tuning(n) for n in range(2, 5)] == choices
    plan2.close()
    # lines without the source chunk (the earlier format) read as the default chunk
    open(cache, "w").write("".join(" ".join(l.split()[:5]) + "\n" for l in lines))
    plan3 = P.CascadePlan(ctx, WATER, f0, g1, [gn[n] for n in range(2, 5)], prec=prec, order=3)
    plan3.autotune(cache, reps=2)
    assert [plan3.tuning(n) for n in range(2, 5)] == [dict(c, src_cx=0) for c in choices]
    plan3.close()


def test_batch_autotune_then_graph(ctx, tmp_path):
    probs = problems(5, 3)
    p1s = inputs(probs, P.NVP_C64, 30)
    say("case batch autotune + graph")
    b = P.Batch(ctx, probs, prec=P.NVP_C64, order=3)
    b.autotune(str(tmp_path / "t.txt"), reps=1)
    b.set_graph(False)
    ref = [[t.clone() for t in o] for o in b.execute(p1s, b.outputs())]
    b.set_graph(True, 4)
    outs = b.outputs()
    for _ in range(3):
        b.execute(p1s, outs)
        torch.cuda.synchronize()
        assert same(outs, ref)
    b.close()


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("fused", [False, True])
def test_grouped_batch_matches_eager(ctx, graph, fused, monkeypatch):
    """Multi-task launches per pass and length: the same bits as per-problem execution.
    fused: every harmonic takes the fused source path and so runs on its own."""
    if fused:
        monkeypatch.setenv("NVP_FUSED_SOURCE", "1")
    probs = problems(11, 5)
    # shared transform lengths: problems 0-3 get the same grids as problem 4
    for i in range(4):
        probs[i] = dict(probs[4])
    p1s = inputs(probs, P.NVP_C64, 40)
    say("case grouped batch graph=%d fused=%d" % (graph, fused))
    b = P.Batch(ctx, probs, prec=P.NVP_C64, order=3)
    b.set_graph(False)
    ref = [[t.clone() for t in o] for o in b.execute(p1s, b.outputs())]
    b.set_grouped(True)
    b.set_graph(graph, 4)
    outs = b.outputs()
    for r in range(3):
        for o in outs:
            for t in o:
                t.zero_()
        b.execute(p1s, outs)
        torch.cuda.synchronize()
        assert same(outs, ref), r
    b.close()


def test_batch_errors(ctx):
    probs = problems(2, 4)
    bad = dict(probs[1])
    bad["grids"] = [oracle.Grid((0.0, 0.0, 0.0), -1.0, (4, 4, 4))] * len(bad["grids"])
    with pytest.raises(P.NvpError) as e:
        P.Batch(ctx, [probs[0], bad])
    assert e.value.status == 1 and "problem 1" in str(e.value)
    b = P.Batch(ctx, probs)
    with pytest.raises(P.NvpError):
        b.set_graph(True, 17)
    b.close()


def test_batch_under_the_corrected_quadrature_matches_the_oracle():
    """A batch made while the context selects the corrected quadrature: graph replays against
    the oracle's cascades under that rule."""
    c = P.Context(0)
    try:
        P.set_quadrature(c, P.NVP_QUAD_CORRECTED)
        probs = problems(3, 5)
        p1s = inputs(probs, P.NVP_C128, 40)
        say("case batch corrected quadrature")
        b = P.Batch(c, probs, prec=P.NVP_C128, order=3)
        b.set_graph(True, 2)
        outs = b.outputs()
        for r in range(2):
            b.execute(p1s, outs)
            torch.cuda.synchronize()
            for i, pr in enumerate(probs):
                gn = {n: g for n, g in zip(range(2, len(pr["grids"]) + 2), pr["grids"])}
                ref = oracle.cascade(p1s[i].cpu().numpy(), pr["g1"], gn, pr["f0"], pr["med"], 3, method="fft",
                                     rule="corrected")
                for n, t in zip(sorted(gn), outs[i]):
                    assert oracle.rel_l2(t.cpu().numpy(), ref[n]) < 1e-12, (r, i, n)
        b.close()
    finally:
        c.sync()
        c.close()
