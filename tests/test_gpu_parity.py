"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 over the compared voxels): 1e-12 for complex128 and
1e-5 for complex64.
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from workload import bowl, configs, fields

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")

WATER = configs.WATER
F0 = 1.1e6
TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}
DT = {P.NVP_C64: torch.complex64, P.NVP_C128: torch.complex128}
LENGTHS = P.transform_lengths()


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


def grid_of(n, h=1.0e-4, origin=(0.01, -0.002, 0.003)):
    return oracle.Grid(origin, h, n)


# ------------------------------------------------------------------ raw operator

@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("L", LENGTHS)
def test_volume_potential_each_length_each_axis(ctx, L, axis, prec):
    # the longest axis of this transform length; short cross-section for the long ones, so
    # that the oracle's direct sum stays small
    n = [3, 5, 4] if L <= 2048 else [2, 3, 1]
    n[axis] = L // 2
    assert P.circulant_size(L // 2) == L
    g = grid_of(tuple(n))
    say("case vp L=%d axis=%d prec=%d n=%s" % (L, axis, prec, n))
    f = fields.random_field(g.n, 100 + L + axis)
    k = complex(2 * 4647.91, 0.5)
    u = P.volume_potential(ctx, k, g, dev(f, prec))
    ref = _direct_cached(f, g.h, k, (L, axis))
    assert oracle.rel_l2(host(u), ref) < TOL[prec]


_DIRECT = {}


def _direct_cached(f, h, k, key):
    """-conv_direct(f), kept for the other precision of the same case."""
    if key not in _DIRECT:
        _DIRECT.clear()
        _DIRECT[key] = -oracle.conv_direct(f, h, k)
    return _DIRECT[key]


@pytest.mark.parametrize("n", [(4096, 2, 3), (2, 4096, 1), (1, 3, 4096), (2049, 1, 1)])
def test_axes_beyond_2048_voxels(ctx, n):
    """Axes longer than the old limit of 1024 voxels, up to the longest transform (8192)."""
    g = grid_of(n, h=5e-5)
    say("case vp long axis n=%s" % (n,))
    f = fields.random_field(n, sum(n))
    k = complex(3 * 4647.91, 0.25)
    u = P.volume_potential(ctx, k, g, dev(f, P.NVP_C64))
    assert oracle.rel_l2(host(u), -oracle.conv_direct(f, g.h, k)) < 1e-5


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("n", [(17, 23, 30), (9, 40, 11), (1, 6, 33), (24, 1, 1)])
def test_volume_potential_ragged_boxes(ctx, n, prec):
    g = grid_of(n, h=7.5e-5)
    say("case vp ragged n=%s prec=%d" % (n, prec))
    f = fields.random_field(n, sum(n))
    k = complex(3 * 4647.91, 0.25)
    u = P.volume_potential(ctx, k, g, dev(f, prec))
    assert oracle.rel_l2(host(u), -oracle.conv_direct(f, g.h, k)) < TOL[prec]


def test_impulse_response_is_minus_kernel(ctx):
    n = (9, 10, 11)
    g = grid_of(n, h=1.1e-4)
    k = complex(2 * 4647.91, 0.1)
    f = np.zeros(n, dtype=np.complex128)
    j = (3, 7, 2)
    f[j] = 1.0
    u = host(P.volume_potential(ctx, k, g, dev(f, P.NVP_C128)))
    K = oracle.kernel_offsets(k, g.h, n)
    I = np.abs(np.arange(n[0])[:, None, None] - j[0])
    J = np.abs(np.arange(n[1])[None, :, None] - j[1])
    Kk = np.abs(np.arange(n[2])[None, None, :] - j[2])
    ref = -K[I, J, Kk]
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_repeat_runs_bitwise_identical(ctx):
    n = (20, 18, 33)
    g = grid_of(n)
    f = dev(fields.random_field(n, 7), P.NVP_C64)
    a = P.volume_potential(ctx, 9000.0 + 1j, g, f).clone()
    b = P.volume_potential(ctx, 9000.0 + 1j, g, f)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# ------------------------------------------------------------------ the cascade

def tiny_inputs():
    cfg = configs.CFG_TINY
    focus = (cfg["l"], 0.0, 0.0)
    h2 = oracle.spacing(2, cfg["f0"], WATER["c0"])
    g = oracle.grid_from_counts(focus, h2, cfg["grids"][2]["n"], cfg["grids"][2]["i_f"])
    k1 = oracle.wavenumber(1, cfg["f0"], WATER)
    pts = bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])
    p1 = bowl.incident_field(pts, cfg["R"], cfg["l"], k1, cfg["p0"], g.coords(0), g.coords(1), g.coords(2)).numpy()
    return cfg, g, p1


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_tiny_config_p2_matches_direct_sum(ctx, prec):
    """p1 of a 256-point bowl on 32^3 at lambda_2/6; p2 on the same grid (circulant 64^3)."""
    cfg, g, p1 = tiny_inputs()
    say("case tiny-32 prec=%d" % prec)
    plan = P.CascadePlan(ctx, WATER, cfg["f0"], g, [g], prec=prec, order=1)
    (p2,) = plan.execute(dev(p1, prec))
    ref = oracle.harmonic(2, {1: (p1, g)}, g, cfg["f0"], WATER, 1, method="direct")
    assert oracle.rel_l2(host(p2), ref) < TOL[prec]
    plan.close()


def nested_grids(short_x=False):
    """Tiny nested grids.  short_x: x axes of 8 voxels (circulant 16), too short to stage four
    cubic stencils in the x pass, so the source build takes its direct-gather path."""
    focus = (15e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (10, 9, 8), (5, 4, 4))
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (8 if short_x else 8 + 2 * n, 11, 10),
                                     (4 if short_x else 6, 5, 4))
          for n in range(2, 6)}
    return focus, g1, gn


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("short_x", [False, True])
@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
@pytest.mark.parametrize("order", [1, 3])
def test_tiny_nested_cascade_matches_oracle(ctx, order, prec, short_x, fused, monkeypatch):
    """fused: the source build fused into the x pass (NVP_FUSED_SOURCE=1) instead of its own tiled kernel."""
    focus, g1, gn = nested_grids(short_x)
    say("case nested-cascade order=%d prec=%d short_x=%d fused=%d" % (order, prec, short_x, fused))
    if fused:
        monkeypatch.setenv("NVP_FUSED_SOURCE", "1")
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(7.5e-3, 15e-3, 128, 1)
    p1 = bowl.incident_field(pts, 7.5e-3, 15e-3, k1, 1e6, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=prec, order=order)
    outs = plan.execute(dev(p1, prec))
    ref = oracle.cascade(p1, g1, gn, F0, WATER, order, method="direct")
    for n in range(2, 6):
        assert oracle.rel_l2(host(outs[n - 2]), ref[n]) < TOL[prec], n
    plan.close()


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_overlapped_spectra_match_in_line(ctx, prec):
    """Kernel spectra on the plan's second stream (the default) against spectra computed in line:
    the same bits, spectra recomputed on every call, with other work queued between calls."""
    focus = (40e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (24, 20, 18), (12, 10, 9))
    gn = [oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (40 + 8 * n, 36, 30), (24, 18, 15))
          for n in range(2, 6)]
    p1 = dev(fields.smooth_field(g1.n, 3) * 1e6, prec)
    say("case overlapped spectra prec=%d" % prec)
    plan = P.CascadePlan(ctx, WATER, F0, g1, gn, prec=prec, order=3)
    plan.set_kernel_cache(False)
    plan.set_overlap(False)
    ref = [t.clone() for t in plan.execute(p1)]
    plan.set_overlap(True)
    outs = [torch.empty_like(t) for t in ref]
    junk = torch.randn(1 << 20, device="cuda")
    for r in range(3):
        for t in outs:
            t.zero_()
        plan.execute(p1, outs)
        junk = junk * 1.0001 + 1.0
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ref)), r
    assert plan.workspace_bytes() > 0
    plan.close()


def test_caller_workspace_matches_plan_owned(ctx):
    """A plan run in a caller workspace (and back in buffers of its own) gives the same bits;
    short and misaligned workspaces are refused and leave the plan as it was."""
    focus, g1, gn = nested_grids()
    p1 = dev(fields.smooth_field(g1.n, 4) * 1e6, P.NVP_C64)
    say("case caller workspace")
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=P.NVP_C64, order=3)
    plan.set_kernel_cache(False)
    ref = [t.clone() for t in plan.execute(p1)]
    held = plan.workspace_bytes()
    need = plan.work_bytes()
    assert 0 < need
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.NvpError) as e:
        plan.set_workspace(ws[: need - 1])
    assert e.value.status == 1
    with pytest.raises(P.NvpError) as e:
        plan.set_workspace(ws[1:])
    assert e.value.status == 1
    ws.fill_(0xFF)  # NaN patterns: the plan must not read what it has not written
    plan.set_workspace(ws[:need])
    assert plan.workspace_bytes() < held
    for overlap in (True, False):
        plan.set_overlap(overlap)
        outs = plan.execute(p1)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ref)), overlap
    plan.set_workspace(None)
    outs = plan.execute(p1)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(outs, ref))
    plan.close()


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_single_harmonic_with_stand_in_fields(ctx, prec):
    """Harmonic 5 from seeded stand-ins for p1..p4 on coarser, offset grids (cubic transfer)."""
    focus, g1, gn = nested_grids()
    flds = {1: (fields.smooth_field(g1.n, 1) * 1e6, g1)}
    for m in range(2, 5):
        flds[m] = (fields.smooth_field(gn[m].n, m) * 10 ** (6 - m), gn[m])
    say("case harmonic-5 stand-ins prec=%d" % prec)
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=prec, order=3)
    p5 = plan.execute_harmonic(5, [dev(flds[m][0], prec) for m in range(1, 5)])
    ref = oracle.harmonic(5, flds, gn[5], F0, WATER, 3, method="direct")
    assert oracle.rel_l2(host(p5), ref) < TOL[prec]
    plan.close()


# ------------------------------------------------------------------ full sizes, sampled

def sample_targets(shape, i_f, count, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(i_f), (0, 0, 0), tuple(s - 1 for s in shape), (shape[0] - 1, 0, shape[2] // 2)]
    pts += [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(count - len(pts))]
    # the axis through the focus
    pts += [(x, i_f[1], i_f[2]) for x in np.linspace(0, shape[0] - 1, 8).astype(int)]
    return np.array([np.ravel_multi_index(p, shape) for p in pts], dtype=np.int64)


def paper_scale_inputs():
    cfg = configs.paper_scale(P_f=3.5e6)
    c0 = WATER["c0"]
    focus = (cfg["l"], 0.0, 0.0)
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), cfg["p1_grid"]["n"], cfg["p1_grid"]["i_f"])
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), s["n"], s["i_f"])
          for n, s in cfg["grids"].items()}
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])
    p1 = bowl.incident_field(pts, cfg["R"], cfg["l"], k1, cfg["p0"], g1.coords(0), g1.coords(1), g1.coords(2),
                             device="cuda", chunk=8192).cpu().numpy()
    return cfg, g1, gn, p1


@pytest.mark.parametrize("order", [1, 3])
def test_paper_scale_p2_sampled(ctx, order):
    """p2 on 256^3 (circulant 512^3, complex64) from the 4096-point bowl's p1 on 128^3."""
    cfg, g1, gn, p1 = paper_scale_inputs()
    say("case paper-scale p2 order=%d" % order)
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=P.NVP_C64, order=order)
    p2 = host(plan.execute_harmonic(2, [dev(p1, P.NVP_C64)]))
    plan.close()
    t = sample_targets(gn[2].n, (128, 128, 128), 24, 3)
    ref = oracle.harmonic(2, {1: (p1, g1)}, gn[2], F0, WATER, order, method="direct", targets=t)
    assert oracle.rel_l2(p2.ravel()[t], ref) < 1e-5


def test_paper_scale_p5_sampled_with_stand_ins(ctx):
    """p5 on 448 x 256^2 (circulant 896 x 512^2) from p1 and stand-ins for p2..p4 on their grids."""
    cfg, g1, gn, p1 = paper_scale_inputs()
    flds = {1: (p1, g1)}
    for m in range(2, 5):
        flds[m] = (fields.smooth_field(gn[m].n, 10 + m) * 10 ** (6 - m), gn[m])
    say("case paper-scale p5 stand-ins")
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=P.NVP_C64, order=3)
    p5 = host(plan.execute_harmonic(5, [dev(flds[m][0], P.NVP_C64) for m in range(1, 5)]))
    plan.close()
    t = sample_targets(gn[5].n, (128, 128, 128), 24, 5)
    ref = oracle.harmonic(5, flds, gn[5], F0, WATER, 3, method="direct", targets=t)
    assert oracle.rel_l2(p5.ravel()[t], ref) < 1e-5


def test_uniform_size_volume_potential_sampled(ctx):
    """The uniform baseline's operator: 640^3 at lambda_5/6 (circulant 1280^3, complex64)."""
    n = (640, 640, 640)
    h = oracle.spacing(5, F0, WATER["c0"])
    g = grid_of(n, h=h, origin=(0.15 - 320 * h, -320 * h, -320 * h))
    say("case uniform 640^3 vp")
    ax = [np.exp(-0.5 * ((np.arange(s) - 0.45 * s) / (0.2 * s)) ** 2) * np.exp(0.3j * np.arange(s)) for s in n]
    fx = [torch.from_numpy(a).to("cuda") for a in ax]
    f_dev = (fx[0][:, None, None] * fx[1][None, :, None] * fx[2][None, None, :]).to(torch.complex64).contiguous()
    k = oracle.wavenumber(5, F0, WATER)
    u = P.volume_potential(ctx, k, g, f_dev)
    t = sample_targets(n, (320, 320, 320), 12, 7)
    f_host = f_dev.to(torch.complex128).cpu().numpy()
    del f_dev
    ref = -oracle.conv_direct(f_host, h, k, targets=t)
    got = host(u).ravel()[t]
    del u
    torch.cuda.empty_cache()
    assert oracle.rel_l2(got, ref) < 1e-5


@pytest.mark.parametrize("n", [(716, 568, 568), (890, 735, 735)])
def test_largest_paper_meshes_volume_potential_sampled(ctx, n):
    """The largest meshes of the paper's own runs, complex64: H101's p5 box (716 x 568^2, circulant
    1536 x 1280^2) and H131's p5 reference domain of Section 5 (890 x 735^2, circulant 2048 x 1536^2)."""
    h = oracle.spacing(5, F0, WATER["c0"])
    c = tuple(v // 2 for v in n)
    g = grid_of(n, h=h, origin=tuple(-ci * h for ci in c))
    say("case largest mesh vp n=%s" % (n,))
    ax = [np.exp(-0.5 * ((np.arange(s) - 0.55 * s) / (0.25 * s)) ** 2) * np.exp(0.2j * np.arange(s)) for s in n]
    fx = [torch.from_numpy(a).to("cuda") for a in ax]
    f_dev = (fx[0][:, None, None] * fx[1][None, :, None] * fx[2][None, None, :]).to(torch.complex64).contiguous()
    k = oracle.wavenumber(5, F0, WATER)
    u = P.volume_potential(ctx, k, g, f_dev)
    t = sample_targets(n, c, 8, 9)
    got = u.reshape(-1)[torch.from_numpy(t).to("cuda")].to(torch.complex128).cpu().numpy()
    del u
    f_host = f_dev.to(torch.complex128).cpu().numpy()
    del f_dev
    torch.cuda.empty_cache()
    ref = -oracle.conv_direct(f_host, h, k, targets=t)
    assert oracle.rel_l2(got, ref) < 1e-5


# ------------------------------------------------------------------ error paths

def test_allocation_failures_keep_no_state(ctx, monkeypatch):
    """Forced device allocation failures (NVP_DEVICE_ALLOC_LIMIT): NVP_E_NOMEM, nothing held after,
    and the same calls succeed once the limit is lifted."""
    focus = (40e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (24, 20, 18), (12, 10, 9))
    gn = [oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (48, 40, 40), (24, 20, 20)) for n in (2, 3)]
    p1 = dev(fields.smooth_field(g1.n, 3) * 1e6, P.NVP_C64)
    f = dev(fields.random_field((20, 18, 33), 7), P.NVP_C64)
    g = grid_of((20, 18, 33))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("case forced allocation failures")  # a wavenumber no other test uses: the context's cache misses
    # limit 0: every allocation fails; 1 MiB: the plan's tables fit but its work buffers do not
    for limit in ("0", "1048576"):
        monkeypatch.setenv("NVP_DEVICE_ALLOC_LIMIT", limit)
        with pytest.raises(P.NvpError) as e:
            P.CascadePlan(ctx, WATER, F0, g1, gn, prec=P.NVP_C64, order=3)
        assert e.value.status == 2
    monkeypatch.setenv("NVP_DEVICE_ALLOC_LIMIT", "0")
    with pytest.raises(P.NvpError) as e:
        P.volume_potential(ctx, 9123.0 + 1j, g, f)
    assert e.value.status == 2
    monkeypatch.delenv("NVP_DEVICE_ALLOC_LIMIT")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (8 << 20)  # nothing new held (a cache may have been freed)
    plan = P.CascadePlan(ctx, WATER, F0, g1, gn, prec=P.NVP_C64, order=3)
    a = [t.clone() for t in plan.execute(p1)]
    b = plan.execute(p1)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b)) and all(bool(torch.isfinite(x).all()) for x in a)
    plan.close()
    u = P.volume_potential(ctx, 9123.0 + 1j, g, f)
    torch.cuda.synchronize()
    ref = -oracle.conv_direct(f.to(torch.complex128).cpu().numpy(), g.h, 9123.0 + 1j)
    assert oracle.rel_l2(host(u), ref) < 1e-5

def test_error_codes(ctx):
    g = grid_of((8, 8, 8))
    f = torch.zeros((8, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(P.NvpError) as e:
        P.volume_potential(ctx, 9000.0, g, f, out=f)  # aliasing
    assert e.value.status == 1
    with pytest.raises(P.NvpError) as e:
        P.CascadePlan(ctx, WATER, F0, g, [g], order=2)
    assert e.value.status == 4
    with pytest.raises(P.NvpError) as e:  # an axis beyond the longest transform (8192)
        P.volume_potential(ctx, 9000.0, grid_of((4097, 2, 2)), torch.zeros((4097, 2, 2), dtype=torch.complex64,
                                                                           device="cuda"))
    assert e.value.status == 4
    small = grid_of((3, 8, 8))
    with pytest.raises(P.NvpError) as e:
        P.CascadePlan(ctx, WATER, F0, small, [g], order=3)  # source axis shorter than the cubic stencil
    assert e.value.status == 1
    empty = oracle.Grid((0.0, 0.0, 0.0), 1e-4, (0, 4, 4))
    for call in (lambda: P.CascadePlan(ctx, WATER, F0, g, [empty]),
                 lambda: P.CascadePlan(ctx, WATER, F0, empty, [g]),
                 lambda: P.volume_potential(ctx, 9000.0, empty, torch.zeros((0, 4, 4), dtype=torch.complex64,
                                                                             device="cuda"))):
        with pytest.raises(P.NvpError) as e:
            call()
        assert e.value.status == 1


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_regrid_equals_a_fresh_plan(ctx, prec):
    """nvp_plan_regrid replaces one harmonic's grid (a guarded run's fallback to the full box): the
    cascade then equals, bit for bit, that of a plan made with the new grids, and matches the oracle;
    a refused regrid leaves the plan working as before."""
    focus, g1, gn = nested_grids()
    big = oracle.grid_from_counts(focus, gn[3].h, (30, 23, 20), (12, 10, 9))  # harmonic 3, larger box
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(7.5e-3, 15e-3, 128, 1)
    p1 = bowl.incident_field(pts, 7.5e-3, 15e-3, k1, 1e6, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    say("case regrid prec=%d" % prec)
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 6)], prec=prec, order=3)
    first = [t.clone() for t in plan.execute(dev(p1, prec))]  # spectra of the small boxes computed
    plan.regrid(3, big)
    got = plan.execute(dev(p1, prec))
    with pytest.raises(P.NvpError):
        plan.regrid(7, big)  # no harmonic 7: refused, plan unchanged
    again = plan.execute(dev(p1, prec))
    grids2 = {2: gn[2], 3: big, 4: gn[4], 5: gn[5]}
    fresh = P.CascadePlan(ctx, WATER, F0, g1, [grids2[n] for n in range(2, 6)], prec=prec, order=3)
    want = fresh.execute(dev(p1, prec))
    torch.cuda.synchronize()
    assert tuple(got[1].shape) == tuple(big.n)
    assert torch.equal(got[0], first[0])  # harmonic 2 untouched
    for a, b, c in zip(got, want, again):
        assert torch.equal(a, b) and torch.equal(a, c)
    ref = oracle.cascade(p1, g1, grids2, F0, WATER, 3, method="direct")
    for n in range(2, 6):
        assert oracle.rel_l2(host(got[n - 2]), ref[n]) < TOL[prec], n
    plan.close()
    fresh.close()


def test_context_outlives_its_plans():
    """The C ABI refuses to destroy a context a plan still uses (the plan's destroy call reaches
    it); the binding's Context.close() destroys the context's plans first."""
    c = P.Context(0)
    h = oracle.spacing(2, F0, WATER["c0"])
    g1 = oracle.grid_from_counts((15e-3, 0.0, 0.0), 2 * h, (10, 9, 8), (5, 4, 4))
    g2 = oracle.grid_from_counts((15e-3, 0.0, 0.0), h, (12, 11, 10), (6, 5, 5))
    plan = P.CascadePlan(c, WATER, F0, g1, [g2], prec=P.NVP_C64, order=3)
    assert P._native.lib().nvp_ctx_destroy(c.handle) == 5  # NVP_E_STATE, nothing freed
    p2 = plan.execute(torch.ones(tuple(g1.n), dtype=torch.complex64, device="cuda"))[0]
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(p2)).all()
    c.close()
    assert plan.handle is None and c.handle is None
    plan.close()  # a no-op now


@pytest.mark.parametrize("prec", [P.NVP_C128, P.NVP_C64])
def test_eight_harmonic_cascade_matches_oracle(ctx, prec):
    """The longest cascade the library takes, p2..p8 (up to seven lower fields per source term), each
    harmonic from the plan's own chained outputs, against the oracle's direct-sum cascade at every
    voxel.  In complex64 the source terms of p6..p8 run in the kernel with a wavefront per field; in
    complex128 they take the fused path."""
    focus = (15e-3, 0.0, 0.0)
    c0 = WATER["c0"]
    g1 = oracle.grid_from_counts(focus, oracle.spacing(1, F0, c0), (10, 9, 8), (5, 4, 4))
    gn = {n: oracle.grid_from_counts(focus, oracle.spacing(n, F0, c0), (8 + 2 * n, 12, 16), (4 + n, 6, 8))
          for n in range(2, 9)}
    say("case eight-harmonic cascade prec=%d" % prec)
    k1 = oracle.wavenumber(1, F0, WATER)
    pts = bowl.bowl_points(7.5e-3, 15e-3, 128, 1)
    p1 = bowl.incident_field(pts, 7.5e-3, 15e-3, k1, 1e6, g1.coords(0), g1.coords(1), g1.coords(2)).numpy()
    plan = P.CascadePlan(ctx, WATER, F0, g1, [gn[n] for n in range(2, 9)], prec=prec, order=3)
    try:
        outs = plan.execute(dev(p1, prec))
        ref = oracle.cascade(p1, g1, gn, F0, WATER, 3, method="direct")
        for n in range(2, 9):
            assert oracle.rel_l2(host(outs[n - 2]), ref[n]) < TOL[prec], n
    finally:
        plan.close()
