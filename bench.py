"""Benchmark of the nested-mesh volume-potential cascade on one MI355X.

Workload (paper-scale homogeneous run): bowl R = 7.5 cm, l = 15 cm, 1.1 MHz,
water, focal pressure 3.5 MPa, 4096 surface points; p1 on 128^3 at lambda_1/6;
harmonics 2..5 on nested grids (64 (n+2), 256, 256) at lambda_n/6 (circulants
(128 (n+2), 512, 512)), complex64, tricubic transfer.  One step = the whole
cascade p1 -> p2..p5: for each harmonic the FP64 kernel tabulation and kernel
spectrum, the transfer + source build, and the pruned circulant convolution.

Prints one JSON line.  `value` = voxels of p2..p5 per second of step time.
Also measured: the same cascade on the uniform 640^3 baseline grid (circulant
1280^3) and the focal-pressure difference between the two, per-kernel HIP
event times (roofline of the dominant kernel), and the FP64 oracle on a
bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "volume-potential voxels/s + % peak HBM; nested vs uniform time @1% focal err"
PEAK_HBM_GBS = 8000.0
ELEM = 8  # complex64 bytes


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """SHA-256 over the library's sources: HBM counter figures apply only to the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2011_03009_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "nvp.h"), "rb").read())
    return h.hexdigest()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_nested_cascade_paper_scale.md")


def counter_traffic(kind):
    """HBM bytes per launch of `kind` from the committed counter summary, or None when it is absent or
    was taken on other kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    i = text.find("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    d = json.loads(text[i + 7:j])
    if d.get("source_hash") != kernel_source_hash() or kind not in d.get("kinds", {}):
        return None
    k = d["kinds"][kind]
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def build_inputs(P, torch, cfg, device):
    from workload import bowl
    W = cfg["medium"]
    f0 = cfg["f0"]
    focus = (cfg["l"], 0.0, 0.0)
    g1 = P.grid_from_counts(focus, P.spacing(W, f0, 1), cfg["p1_grid"]["n"], cfg["p1_grid"]["i_f"])
    gn = [P.grid_from_counts(focus, P.spacing(W, f0, n), cfg["grids"][n]["n"], cfg["grids"][n]["i_f"])
          for n in range(2, cfg["n_harm"] + 1)]
    gu = [P.grid_from_counts(focus, P.spacing(W, f0, 5), cfg["uniform_grids"][n]["n"],
                             cfg["uniform_grids"][n]["i_f"]) for n in range(2, cfg["n_harm"] + 1)]
    k1 = P.wavenumber(W, f0, 1)
    import numpy as np
    ax = [g1.origin[a] + np.arange(g1.n[a]) * g1.h for a in range(3)]
    pts = bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])
    p1 = bowl.incident_field(pts, cfg["R"], cfg["l"], k1, cfg["p0"], ax[0], ax[1], ax[2], device=device,
                             chunk=8192).to(torch.complex64).contiguous()
    return g1, gn, gu, p1


def corrected_quadrature_bench(P, torch, cfg, g1, gn, p1, nested, order, stream):
    """The nested cascade under the corrected quadrature (its own context) against the paper's rule:
    per harmonic, the relative L2 and focal differences, and the step time under each rule."""
    c = P.Context(0, stream)
    try:
        P.set_quadrature(c, P.NVP_QUAD_CORRECTED)
        plan = P.CascadePlan(c, cfg["medium"], cfg["f0"], g1, gn, prec=P.NVP_C64, order=order)
        plan.set_kernel_cache(False)
        outs = [torch.empty(tuple(g.n), dtype=torch.complex64, device=p1.device) for g in gn]
        ms = time_steps(torch, plan, p1, outs, 5, 1, stream)
        rows = {}
        for i, (a, b) in enumerate(zip(outs, nested)):
            i_f = tuple(cfg["grids"][i + 2]["i_f"])
            rows[str(i + 2)] = {"rel_l2_paper_vs_corrected": float(torch.linalg.vector_norm(b - a) /
                                                                   torch.linalg.vector_norm(a)),
                                "focal_corrected_Pa": abs(complex(a[i_f].item())),
                                "focal_paper_Pa": abs(complex(b[i_f].item()))}
        plan.close()
        return {"ms_per_step": ms, "harmonics": rows,
                "note": "same workload and step as the headline figure, corrected lattice quadrature"}
    finally:
        c.close()


def full_cascade_bench(P, torch, ctx, cfg, g1, gn, p1, order, log):
    """The full truncated cascade (difference-frequency terms included) against the paper's one-way
    cascade on the nested workload: fixed-point sweeps, time, and the change of every harmonic."""
    from paper_2011_03009_amd import full_cascade as GF
    W = cfg["medium"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, sweeps, change, paper = GF.full_cascade(ctx, W, cfg["f0"], g1, gn, p1, order=order, tol=1e-6, log=log)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rows = {}
    ref = [p1] + paper
    for n in range(1, len(p) + 1):
        i_f = tuple(cfg["p1_grid"]["i_f"] if n == 1 else cfg["grids"][n]["i_f"])
        a_n, b_n = abs(complex(p[n - 1][i_f].item())), abs(complex(ref[n - 1][i_f].item()))
        rel = float(torch.linalg.vector_norm(p[n - 1] - ref[n - 1]) / torch.linalg.vector_norm(ref[n - 1]))
        rows[str(n)] = {"focal_full_Pa": a_n, "focal_paper_Pa": b_n, "rel_l2_change": rel}
    return {"sweeps": sweeps, "last_change": change, "seconds": dt, "tol": 1e-6, "harmonics": rows,
            "note": "sweep 0 is the paper's cascade; each sweep recomputes p1..p5 with sum- and "
                    "difference-frequency sources (complex64, kernel spectra rebuilt per potential)"}


def nsz(g):
    return int(g.n[0]) * int(g.n[1]) * int(g.n[2])


def alg_bytes(P, g1, gn, order_fields):
    """Algorithmic HBM bytes per launch kind for one cascade (complex64 passes, FP64 kernel)."""
    b = {k: 0.0 for k in P.nvp.TIMING_KINDS}
    grids = [g1] + list(gn)
    for i, g in enumerate(gn):
        n = i + 2
        N = [int(v) for v in g.n]
        M = [P.circulant_size(v) for v in N]
        H = [m // 2 + 1 for m in M]
        Ho = H[0] * H[1] * H[2]
        b["ktab"] += 16.0 * Ho  # tabulation fused into the z pass: FP64 octant written once
        b["kfft"] += 16.0 * Ho * 2 + 16.0 * Ho + 8.0 * Ho  # y pass r+w FP64; x pass reads FP64, writes complex64
        src = sum(nsz(grids[m - 1]) for m in range(1, n))
        b["src"] += ELEM * (src + N[0] * N[1] * N[2])  # native fields in, f_n out
        b["xfwd"] += ELEM * (N[0] * N[1] * N[2] + M[0] * N[1] * N[2])
        b["yfwd"] += ELEM * (M[0] * N[1] * N[2] + M[0] * M[1] * N[2])
        b["zconv"] += ELEM * (2 * M[0] * M[1] * N[2] + Ho)
        b["yinv"] += ELEM * (M[0] * M[1] * N[2] + M[0] * N[1] * N[2])
        b["xinv"] += ELEM * (M[0] * N[1] * N[2] + N[0] * N[1] * N[2])
    return b


def time_steps(torch, plan, p1, outs, steps, warmup, stream):
    for _ in range(warmup):
        plan.execute(p1, outs)
    torch.cuda.synchronize()
    plan.get_timing()  # drop warmup events
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.execute(p1, outs)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def per_harmonic_rates(P, torch, plan, p1, outs, g1, gn, order, stream, reps=5):
    """Each harmonic's convolution step alone (kernel spectrum cached): voxels/s and the fraction of
    8 TB/s its algorithmic bytes (transfer + source build and the five passes) move at."""
    fields = [p1] + list(outs)
    rows = {}
    for i, g in enumerate(gn):
        n = i + 2
        plan.execute_harmonic(n, fields[:n - 1], outs[i])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.execute_harmonic(n, fields[:n - 1], outs[i])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b = alg_bytes(P, g1, gn[:i + 1], order)
        conv = sum(b[k] for k in ("src", "xfwd", "yfwd", "zconv", "yinv", "xinv"))
        if i:  # alg_bytes sums over the grids given: keep harmonic n's share
            prev = alg_bytes(P, g1, gn[:i], order)
            conv -= sum(prev[k] for k in ("src", "xfwd", "yfwd", "zconv", "yinv", "xinv"))
        rows[str(n)] = {"grid": [int(v) for v in g.n], "ms": ms, "voxels_per_s": nsz(g) / (ms * 1e-3),
                        "alg_GBs": conv / (ms * 1e-3) / 1e9, "frac_hbm": conv / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    return rows


def copy_ceiling(torch, stream, gib=4, reps=5):
    """A device-to-device copy of `gib` GiB (read + write bytes over time): the HBM rate a plain
    streaming kernel reaches, beside the 8 TB/s datasheet peak."""
    src = torch.ones((gib << 30) // 8, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2.0 * src.numel() * 8 / (ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_copied": (gib << 30), "ms": ms, "GBs_read_plus_write": gbs, "frac_of_peak": gbs / PEAK_HBM_GBS}


def amplitude_order_sweep(P, torch, ctx, stream, pfs=(2.0e6, 3.5e6, 5.0e6), orders=(1, 3)):
    """The headline workload at the other focal pressures and with the paper's linear transfer: the
    nested step time and the focal error e_n against the uniform 640^3 run of the same input."""
    from workload import configs
    rows = []
    for pf in pfs:
        cfg = configs.paper_scale(P_f=pf)
        W = cfg["medium"]
        g1, gn, gu, p1 = build_inputs(P, torch, cfg, torch.device("cuda", 0))
        i1 = tuple(cfg["p1_grid"]["i_f"])
        p1f = abs(complex(p1[i1].item()))
        for order in orders:
            plan = P.CascadePlan(ctx, W, cfg["f0"], g1, gn, prec=P.NVP_C64, order=order)
            plan.set_kernel_cache(False)
            outs = [torch.empty(tuple(g.n), dtype=torch.complex64, device="cuda") for g in gn]
            ms = time_steps(torch, plan, p1, outs, 5, 2, stream)
            plan.close()
            plan_u = P.CascadePlan(ctx, W, cfg["f0"], g1, gu, prec=P.NVP_C64, order=order)
            plan_u.set_kernel_cache(False)
            outs_u = [torch.empty(tuple(g.n), dtype=torch.complex64, device="cuda") for g in gu]
            ms_u = time_steps(torch, plan_u, p1, outs_u, 2, 1, stream)
            plan_u.close()
            e = {}
            for i in range(len(gn)):
                a_n = complex(outs[i][tuple(cfg["grids"][i + 2]["i_f"])].item())
                b_n = complex(outs_u[i][tuple(cfg["uniform_grids"][i + 2]["i_f"])].item())
                e[str(i + 2)] = abs(a_n - b_n) / p1f
            rows.append({"P_f_MPa": pf / 1e6, "order": order, "ms_nested": ms, "ms_uniform": ms_u,
                         "ratio": ms_u / ms, "focal_err": e, "max_focal_err": max(e.values()),
                         "p1_focal_Pa": p1f})
            del outs, outs_u
            torch.cuda.empty_cache()
    return rows


def cpu_baseline(cfg, g1_p, gn_p, p1_dev, budget_s, order):
    """The FP64 oracle on a bounded sample: p2 at random voxels of its 256^3 grid.

    The oracle's steps as it runs them for one harmonic: transfer of p1 onto
    the 256^3 grid and the source term (whole grid, once), then the direct
    midpoint sum at each sampled voxel.  The sample size is chosen from a
    256-voxel probe (enough voxels to keep every host thread busy) so that
    the whole sample takes about budget_s seconds.
    """
    import numpy as np
    import oracle
    W = cfg["medium"]
    f0 = cfg["f0"]
    g1 = oracle.Grid(tuple(g1_p.origin), g1_p.h, tuple(g1_p.n))
    g2 = oracle.Grid(tuple(gn_p[0].origin), gn_p[0].h, tuple(gn_p[0].n))
    p1 = p1_dev.to("cpu").numpy().astype(np.complex128)
    k2 = oracle.wavenumber(2, f0, W)
    C2 = oracle.cascade_constant(2, f0, W)
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    f = oracle.source_term(2, {1: oracle.transfer(p1, g1, g2, order)})
    t_fixed = time.perf_counter() - t0
    probe = rng.integers(0, g2.size(), 256)
    t0 = time.perf_counter()
    C2 * oracle.conv_direct(f, g2.h, k2, targets=probe)
    per = (time.perf_counter() - t0) / 256
    n_t = int(max(256, min(200000, (budget_s - t_fixed) / max(per, 1e-6))))
    t = rng.integers(0, g2.size(), n_t)
    t0 = time.perf_counter()
    C2 * oracle.conv_direct(f, g2.h, k2, targets=t)
    t_sum = time.perf_counter() - t0
    dt = t_fixed + t_sum
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_t / dt, "unit": "voxels/s", "cores": cores, "kind": "oracle",
            "circulant_fft": cpu_method_baseline(cfg, g1_p, gn_p, p1_dev, order),
            "sample": "p2 at %d random voxels of the 256^3 grid: transfer (order %d) and source term of the whole "
                      "grid (%.1f s) plus the FP64 direct midpoint sum over all 16.8M source voxels per sampled "
                      "voxel (%.1f s)" % (n_t, order, t_fixed, t_sum)}


def cpu_method_baseline(cfg, g1_p, gn_p, p1_dev, order):
    """Part of the CPU-baseline leg: the paper's method on the host CPU, p2 on its 256^3 grid through
    the oracle's circulant FFT.

    Transfer of p1 and the source term, the FP64 kernel embedded in a 512^3 circulant, and
    three scipy.fft transforms, complex128, with the box's share of host threads.  The same
    work as one nested harmonic of the GPU step, kernel spectrum included.
    """
    import numpy as np
    import oracle
    workers = int(os.environ.get("OMP_NUM_THREADS", "16"))
    W = cfg["medium"]
    f0 = cfg["f0"]
    g1 = oracle.Grid(tuple(g1_p.origin), g1_p.h, tuple(g1_p.n))
    g2 = oracle.Grid(tuple(gn_p[0].origin), gn_p[0].h, tuple(gn_p[0].n))
    p1 = p1_dev.to("cpu").numpy().astype(np.complex128)
    M = tuple(int(2 * v) for v in g2.n)
    t0 = time.perf_counter()
    f = oracle.source_term(2, {1: oracle.transfer(p1, g1, g2, order)})
    oracle.cascade_constant(2, f0, W) * oracle.conv_circulant(f, g2.h, oracle.wavenumber(2, f0, W), M=M,
                                                              workers=workers)
    dt = time.perf_counter() - t0
    return {"value": g2.size() / dt, "unit": "voxels/s", "cores": workers, "kind": "oracle circulant FFT",
            "sample": "p2 on its %s grid, circulant %s, complex128 scipy.fft: transfer (order %d), source term, "
                      "kernel embedding and three transforms in %.1f s" % (list(g2.n), list(M), order, dt)}


def incident_bench(P, torch, ctx, cfg, g1, p1_ref, stream, reps):
    """The incident field p_1 (Section 3.2 monopole sum) by the HIP kernel on the cascade's p1 grid.

    Timed with HIP events on the context stream; the output is compared with
    the FP64 p1 input that the cascade ran on (generated by torch).
    """
    import numpy as np
    from workload import bowl
    W, f0 = cfg["medium"], cfg["f0"]
    k1 = P.wavenumber(W, f0, 1)
    pts = torch.from_numpy(bowl.bowl_points(cfg["R"], cfg["l"], cfg["n_points"], cfg["seed"])).to(p1_ref.device)
    s = bowl.rayleigh_scale(cfg["R"], cfg["l"], k1, cfg["p0"], cfg["n_points"])
    out = P.incident_field(ctx, k1, s, pts, g1, prec=P.NVP_C64)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        P.incident_field(ctx, k1, s, pts, g1, prec=P.NVP_C64, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ref = p1_ref.to(torch.complex128)
    diff = float(torch.linalg.vector_norm(out.to(torch.complex128) - ref) / torch.linalg.vector_norm(ref))
    vox = nsz(g1)
    return {"ms": ms, "voxels": vox, "points": int(cfg["n_points"]), "pairs_per_s": vox * cfg["n_points"] / (ms * 1e-3),
            "rel_l2_vs_fp64_input": diff, "dtype": "c64 (FP64 distances and phases, FP32 sin/cos/exp, FP64 sums)"}


def paper_workload_bench(P, torch, ctx, stream, reps, log):
    """The paper's own workload (its timing table): the H101 bowl (1.1 MHz, l 63.2 mm, R 32 mm)
    in water at 100 W radiated power, about 4096 points in Deserno's regular placement (as the
    paper), harmonics 2..5 at lambda_n / 6 on the rule-of-thumb nested boxes (post-focal
    d = 10.5 mm), linear transfer, complex64.

    p_1 is the GPU monopole sum on the reference window at lambda_1 / 6, scaled to 100 W by the
    disc-power integral; the cascade then recomputes its kernel spectra on every run.
    """
    import math
    from workload import bowl, configs
    W = configs.WATER
    f0, l, R, d, n_p, power = 1.1e6, 63.2e-3, 32e-3, 10.5e-3, 4096, 100.0
    focus = (l, 0.0, 0.0)
    dev = torch.device("cuda", 0)
    g1, _ = P.grid_from_box(focus, *P.rule_of_thumb_box(2, l, R, d), P.spacing(W, f0, 1))
    gn = [P.grid_from_box(focus, *P.rule_of_thumb_box(n, l, R, d), P.spacing(W, f0, n))[0] for n in range(2, 6)]
    k1 = P.wavenumber(W, f0, 1)
    pts = torch.from_numpy(bowl.bowl_points_deserno(R, l, n_p)).to(dev)
    n_p = int(pts.shape[0])
    s_raw = bowl.cap_area(R, l) / n_p  # the unnormalised field (A / n_p) sum_j G_k
    centre = (bowl.cap_height(R, l), 0.0, 0.0)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pw = P.radiated_power(ctx, k1, s_raw, pts, centre, R, W["rho0"], W["c0"], 256, 256)
    t_power = time.perf_counter() - t0
    s = s_raw * math.sqrt(power / pw)
    p1 = P.incident_field(ctx, k1, s, pts, g1, prec=P.NVP_C64)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    P.incident_field(ctx, k1, s, pts, g1, prec=P.NVP_C64, out=p1)
    b.record(stream)
    torch.cuda.synchronize()
    ms_p1 = a.elapsed_time(b)
    plan = P.CascadePlan(ctx, W, f0, g1, gn, prec=P.NVP_C64, order=1)
    plan.set_kernel_cache(False)
    outs = plan.execute(p1)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        plan.execute(p1, outs)
    b.record(stream)
    torch.cuda.synchronize()
    ms_cascade = a.elapsed_time(b) / reps
    per = []
    fields = [p1]
    for n in range(2, 6):
        a.record(stream)
        plan.execute_harmonic(n, fields, outs[n - 2])
        b.record(stream)
        torch.cuda.synchronize()
        per.append(a.elapsed_time(b))
        fields.append(outs[n - 2])
    i_f = [int(round((focus[ax] - g1.origin[ax]) / g1.h)) for ax in range(3)]
    focal = [abs(complex(p1[i_f[0], i_f[1], i_f[2]].item()))]
    for g, o in zip(gn, outs):
        j = [int(round((focus[ax] - g.origin[ax]) / g.h)) for ax in range(3)]
        focal.append(abs(complex(o[j[0], j[1], j[2]].item())))
    vox = [nsz(g) for g in gn]
    res = {"workload": "H101 in water, 100 W, %d points (Deserno's regular placement), p2..p5 on rule-of-thumb "
                       "boxes (d 10.5 mm) at lambda_n/6, linear transfer, complex64, kernel spectra recomputed" % n_p,
           "p1_grid": [int(v) for v in g1.n], "grids": [[int(v) for v in g.n] for g in gn],
           "circulants": [[P.circulant_size(int(v)) for v in g.n] for g in gn], "voxels": vox,
           "radiated_power_W_before_scaling": pw, "power_integral_s": t_power, "p1_ms": ms_p1,
           "cascade_ms": ms_cascade, "harmonic_ms": per, "total_ms": ms_p1 + ms_cascade + t_power * 1e3,
           "voxels_per_s": sum(vox) / (ms_cascade * 1e-3), "focal_pressure_Pa": focal,
           "plan_device_bytes": plan.workspace_bytes(),
           "paper_cpu_total_s": 4991.0, "paper_cpu_note": "1h23m11s on 2x 14-core Xeon E5-2690 v4 (context)"}
    plan.close()
    return res


def batch_bench(P, torch, ctx, W, steps, log):
    """The batched workload: 64 seeded transducers, harmonic boxes from the trained box predictor.

    Every transducer's p_1 grid covers its reference window; p_2..p_n live on
    the predicted boxes (uneven grids).  Kernel spectra are cached after the
    first run, so a timed run is the transfer + source builds and the
    convolutions of every harmonic of every transducer.
    """
    from paper_2011_03009_amd import boxpred as BP
    from paper_2011_03009_amd import train_boxnet as TB
    Ts = TB.transducers(64, 0)
    net, _ = BP.load_net(ctx)
    inc = TB.make_incident(ctx)
    probs, p1s = [], []
    for T in Ts:
        fr = BP.predict_fractions(net, T, ctx)
        geo = BP.Geometry(T, W)
        g1 = geo.g1()
        probs.append(dict(med=W, f0=T.f0, g1=g1, grids=[geo.grid(n, fr[n]) for n in range(2, T.n_harm + 1)]))
        p1s.append(inc(T, g1))
    net.close()
    vox = sum(nsz(g) for p in probs for g in p["grids"])
    sizes = [nsz(g) for p in probs for g in p["grids"]]
    b = P.Batch(ctx, probs, prec=P.NVP_C64, order=3)
    outs = b.outputs()
    stream = torch.cuda.current_stream()

    def timed(k):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            b.execute(p1s, outs)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    res = {"transducers": len(Ts), "harmonic_grids": len(sizes), "voxels": vox,
           "smallest_grid": min(sizes), "largest_grid": max(sizes)}
    b.set_graph(False)
    b.execute(p1s, outs)  # kernel spectra and twiddles
    torch.cuda.synchronize()
    res["eager_ms"] = timed(steps)
    b.set_graph(True, 4)
    b.execute(p1s, outs)
    torch.cuda.synchronize()
    res["graph_ms"] = timed(steps)
    t0 = time.perf_counter()
    b.autotune(None, reps=2)
    res["autotune_s"] = time.perf_counter() - t0
    b.set_graph(True, 4)
    b.execute(p1s, outs)
    torch.cuda.synchronize()
    res["tuned_graph_ms"] = timed(steps)
    b.set_graph(False)
    res["tuned_eager_ms"] = timed(steps)
    # multi-task launches: each pass of each harmonic level as one launch per transform length
    b.set_grouped(True)
    b.set_graph(True, 1)
    b.execute(p1s, outs)
    torch.cuda.synchronize()
    res["grouped_graph_ms"] = timed(steps)
    b.set_graph(False)
    res["grouped_eager_ms"] = timed(steps)
    best = min(res["eager_ms"], res["graph_ms"], res["tuned_graph_ms"], res["tuned_eager_ms"],
               res["grouped_graph_ms"], res["grouped_eager_ms"])
    res["voxels_per_s"] = vox / (best * 1e-3)
    # the algorithmic bytes of the timed work (spectra cached: transfer + source builds and the five
    # passes of every harmonic of every transducer) over the best time, against 8 TB/s
    conv = 0.0
    for p in probs:
        ab = alg_bytes(P, p["g1"], p["grids"], 3)
        conv += sum(ab[k] for k in ("src", "xfwd", "yfwd", "zconv", "yinv", "xinv"))
    res["alg_bytes"] = conv
    res["alg_GBs"] = conv / (best * 1e-3) / 1e9
    res["frac_hbm"] = res["alg_GBs"] / PEAK_HBM_GBS
    b.close()
    log("bench: batched %s" % res)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's H101 workload")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", type=int, default=3, choices=[1, 3])
    ap.add_argument("--pf", type=float, default=3.5e6, help="focal pressure (Pa)")
    ap.add_argument("--no-uniform", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the focal-pressure and transfer-order sweep")
    ap.add_argument("--corrected-quadrature", action="store_true",
                    help="also run the nested cascade under the corrected quadrature and report how far the "
                         "paper's rule is from it")
    ap.add_argument("--full-cascade", action="store_true",
                    help="also solve the full truncated cascade (with the difference-frequency terms the paper "
                         "drops) on the nested workload and report how far it moves the paper's harmonics")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--calib", action="store_true",
                    help="only copy 1 GiB device-to-device 3 times (a known-size reference for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; every configuration fits one MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2011_03009_amd as P
    from workload import configs

    if a.calib:
        src = torch.ones(1 << 27, dtype=torch.complex64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": src.numel() * 8, "copies": 3}))
        return

    cfg = configs.paper_scale(P_f=a.pf)
    W = cfg["medium"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    log("bench: building inputs")
    g1, gn, gu, p1 = build_inputs(P, torch, cfg, dev)
    ctx = P.Context(0, stream)
    voxels = sum(nsz(g) for g in gn)

    # nested cascade, full step (kernel spectra recomputed every step)
    plan = P.CascadePlan(ctx, W, cfg["f0"], g1, gn, prec=P.NVP_C64, order=a.order)
    plan.set_kernel_cache(False)
    outs = [torch.empty(tuple(g.n), dtype=torch.complex64, device=dev) for g in gn]
    log("bench: nested cascade, %d warmup + %d steps" % (a.warmup, a.steps))
    # the step: kernel spectra on the plan's second stream, overlapped with the convolutions
    ms = time_steps(torch, plan, p1, outs, a.steps, a.warmup, stream)
    # per-kernel HIP-event times: every launch in line on the plan's stream
    plan.set_timing(True)
    ms_seq = time_steps(torch, plan, p1, outs, a.steps, 1, stream)
    timing = plan.get_timing()
    plan.set_timing(False)
    # conv-only rate: kernel spectra cached
    plan.set_kernel_cache(True)
    ms_conv = time_steps(torch, plan, p1, outs, a.steps, 1, stream)
    ctx.sync()
    nested = [o.clone() for o in outs]
    per_harmonic = per_harmonic_rates(P, torch, plan, p1, outs, g1, gn, a.order, stream)

    # roofline of the dominant kernel kind
    ab = alg_bytes(P, g1, gn, a.order)
    per_kind = {}
    for k, (t_ms, cnt) in timing.items():
        if cnt:
            per_kind[k] = {"ms_per_step": t_ms / a.steps, "launches_per_step": cnt / a.steps,
                           "alg_GBs": ab[k] * a.steps / (t_ms * 1e-3) / 1e9}
    dom = max(per_kind, key=lambda k: per_kind[k]["ms_per_step"])
    achieved = per_kind[dom]["alg_GBs"]
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": counter_traffic(dom),
            "alg_bytes_per_launch": ab[dom] / max(1.0, per_kind[dom]["launches_per_step"]),
            "avg_launch_ms": per_kind[dom]["ms_per_step"] / max(1.0, per_kind[dom]["launches_per_step"])}
    conv_kinds = ("src", "xfwd", "yfwd", "zconv", "yinv", "xinv")
    conv_ms = sum(per_kind[k]["ms_per_step"] for k in conv_kinds if k in per_kind)
    conv_gbs = sum(ab[k] for k in conv_kinds) / (conv_ms * 1e-3) / 1e9

    result = {
        "metric": METRIC, "value": voxels / (ms * 1e-3), "unit": "voxels/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": "paper-scale nested cascade: bowl R 7.5 cm, l 15 cm, 1.1 MHz, water, P_f %.2g MPa, "
                               "4096 points; p1 128^3; p2..p5 on (64(n+2),256,256) at lambda_n/6; complex64; "
                               "transfer order %d; kernel spectra recomputed every step" % (a.pf / 1e6, a.order),
                   "voxels_per_step": voxels, "grids": [list(map(int, g.n)) for g in gn],
                   "circulants": [[P.circulant_size(int(v)) for v in g.n] for g in gn]},
        "roofline": roof,
        "sequential": {"ms_per_step": ms_seq, "note": "every launch in line on one stream (the per-kernel timing run)"},
        "conv_only": {"ms_per_step": ms_conv, "voxels_per_s": voxels / (ms_conv * 1e-3),
                      "five_pass_alg_GBs": conv_gbs, "five_pass_frac": conv_gbs / PEAK_HBM_GBS},
        "per_kernel": per_kind,
        "per_harmonic": per_harmonic,
        "copy_ceiling": copy_ceiling(torch, stream),
    }
    del plan

    log("bench: incident field p1 (%d points on 128^3)" % cfg["n_points"])
    result["incident_field"] = incident_bench(P, torch, ctx, cfg, g1, p1, stream, 5)
    log("bench: incident %s" % result["incident_field"])

    if not a.no_paper:
        log("bench: the paper's H101 workload")
        try:
            result["paper_workload"] = paper_workload_bench(P, torch, ctx, stream, 2, log)
        except Exception as exc:  # recorded, so that the rest of the benchmark still reports
            result["paper_workload"] = {"error": repr(exc)}
        log("bench: paper workload %s" % result["paper_workload"])

    if not a.no_uniform:
        log("bench: uniform 640^3 cascade")
        plan_u = P.CascadePlan(ctx, W, cfg["f0"], g1, gu, prec=P.NVP_C64, order=a.order)
        plan_u.set_kernel_cache(False)
        outs_u = [torch.empty(tuple(g.n), dtype=torch.complex64, device=dev) for g in gu]
        ms_u = time_steps(torch, plan_u, p1, outs_u, 3, 1, stream)
        plan_u.set_kernel_cache(True)
        ms_u_conv = time_steps(torch, plan_u, p1, outs_u, 3, 1, stream)
        ctx.sync()
        i1 = cfg["p1_grid"]["i_f"]
        p1f = abs(complex(p1[i1].item()))
        errs = {}
        for i in range(len(gn)):
            a_n = complex(nested[i][tuple(cfg["grids"][i + 2]["i_f"])].item())
            b_n = complex(outs_u[i][tuple(cfg["uniform_grids"][i + 2]["i_f"])].item())
            errs[str(i + 2)] = {"e_n": abs(a_n - b_n) / p1f, "nested": abs(a_n), "uniform": abs(b_n)}
        result["nested_vs_uniform"] = {
            "t_nested_ms": ms, "t_uniform_ms": ms_u, "ratio": ms_u / ms,
            "conv_only_ratio": ms_u_conv / ms_conv, "t_uniform_conv_ms": ms_u_conv,
            "uniform_voxels": sum(nsz(g) for g in gu), "focal_err": errs,
            "max_focal_err": max(e["e_n"] for e in errs.values()), "gate": 0.01,
            "p1_focal_Pa": p1f}
        del plan_u, outs_u
        torch.cuda.empty_cache()

    if not a.no_sweep:
        log("bench: focal pressures 2 / 3.5 / 5 MPa and transfer orders 1 / 3 against the uniform run")
        result["amplitude_order_sweep"] = amplitude_order_sweep(P, torch, ctx, stream)

    if a.corrected_quadrature:
        log("bench: nested cascade under the corrected quadrature")
        result["corrected_quadrature"] = corrected_quadrature_bench(P, torch, cfg, g1, gn, p1, nested, a.order,
                                                                    stream)
        log("bench: corrected quadrature %s" % result["corrected_quadrature"])

    if a.full_cascade:
        log("bench: full cascade with the difference-frequency terms")
        result["full_cascade"] = full_cascade_bench(P, torch, ctx, cfg, g1, gn, p1, a.order, log)
        log("bench: full cascade %s" % result["full_cascade"])

    if not a.no_batch:
        log("bench: batched transducers")
        result["batched"] = batch_bench(P, torch, ctx, W, 5, log)

    if not a.no_cpu:
        log("bench: oracle CPU baseline (direct sum, and the circulant FFT of p2)")
        result["cpu_baseline"] = cpu_baseline(cfg, g1, gn, p1, a.cpu_budget, a.order)
        log("bench: cpu baseline %s" % result["cpu_baseline"])
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
