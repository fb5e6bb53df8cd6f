"""The truncation-convergence study of Section 5 at the paper's scale.

The protocol of Section 5 (the domain study behind the table of domain
fractions):
- The reference domain is D_2 of equation "domain", [l - L, l + d] x
  [-R, R]^2 with L = sqrt(l^2 - R^2) - eps and eps = 0.1 mm, meshed once at
  lambda_5 / 6 with the focus on a voxel centre (for H131 with d = 9.8 mm:
  900 x 732 x 732 voxels); every harmonic's reference solution p_n^r is
  computed on that one mesh, by the cascade of eqs. harm2-harm5.
- For harmonic n and a threshold Q0, the integration domain is the smallest
  cuboid outside which Q = log10(|f_n| / max |f_n|) < Q0, with the part
  beyond the focus kept whole (the post-focal length is never shrunk).
- The error is measured along the x axis relative to the first harmonic,
  ||p_n - p_n^r|| / ||p_1^r||, by the midpoint rule on the reference mesh's
  axis voxels.
- A domain's size is given as fractions of the reference domain's:
  fraction_x = L' / L (pre-focal lengths), fraction_yz = w' / w (widths),
  and the whole x extent (L' + d) / (L + d) (the paper's plots put "the
  fraction of the total domain in the x-direction" on their axis).

Where the paper is silent the study runs each reading side by side, so that
the one that reproduces the printed table can be named:
- lower harmonics: the source f_n of a truncated p_n is built from the
  reference solutions of the lower harmonics ("ref"), or from lower harmonics
  computed on their own domains of the same Q0 ("trunc");
- the truncated p_n on the axis: the potential of the cut source evaluated
  along the whole axis ("everywhere"), or p_n taken as zero on the part of the
  axis outside its domain, where the nested method never computes it
  ("inside").

Every numeric step runs in the library (incident field and its power, the
cascade, source terms, localisation boxes, and the volume potential of the
source restricted to a box, scaled by C_n); this module chooses the boxes and
reduces the axis norms of the results for the report.
"""

import math

import numpy as np
import torch

from . import nvp

# Transducers of the paper's Table of transducers (f0, focal length l, outer radius R).
H131 = dict(f0=1.1e6, l=35e-3, R=16.5e-3)
H101 = dict(f0=1.1e6, l=63.2e-3, R=32e-3)
# Post-focal distance d of H131's reference domain: the paper's mesh of 901 x 732 x 732 voxels
# at lambda_5 / 6 has an x extent of L + d with L = sqrt(l^2 - R^2).
H131_D = 9.8e-3
EPS = 1.0e-4  # the paper's displacement of the reference domain from the bowl (0.1 mm)
Q0_LADDER = tuple(-0.125 * i for i in range(1, 65))
TARGET = 0.01


def cap_height(T):
    return T["l"] - math.sqrt(T["l"] ** 2 - T["R"] ** 2)


def normalised_incident(ctx, T, med, power, points, n_r=256, n_theta=256, reading="abs2"):
    """Scale of the bowl's monopole sum (points: float64 CUDA tensor [n, 3] on the cap) that makes it
    radiate `power` watts through the rim-plane disc: the paper's (A / n) sum G times sqrt(P0 / P).

    reading: how the garbled power integral of Section 3.2 is read.  "abs2" (the library's
    nvp_radiated_power): 1/(2 rho0 c0) int |p|^2 r dr dtheta.  The two alternatives, for the
    domain study's comparison of readings: "sq", the printed p^2 taken literally (complex),
    |1/(2 rho0 c0) int p^2 r dr dtheta|; "abs2_nor", |p|^2 without the area element r.  These
    two sum the library's field at the same midpoint nodes on the host."""
    k1 = nvp.wavenumber(med, T["f0"], 1)
    area = 2.0 * math.pi * T["l"] * cap_height(T)
    s = area / points.shape[0]
    centre = (cap_height(T), 0.0, 0.0)
    if reading == "abs2":
        pw = nvp.radiated_power(ctx, k1, s, points, centre, T["R"], med["rho0"], med["c0"], n_r, n_theta)
    else:
        dr, dth = T["R"] / n_r, 2.0 * math.pi / n_theta
        r = (np.arange(n_r) + 0.5) * dr
        th = (np.arange(n_theta) + 0.5) * dth
        R_, TH = np.meshgrid(r, th, indexing="ij")
        tg = np.stack([np.full(R_.size, centre[0]), (R_ * np.cos(TH)).ravel(), (R_ * np.sin(TH)).ravel()], axis=1)
        p = nvp.incident_at(ctx, k1, s, points, torch.from_numpy(tg).to("cuda"), prec=nvp.NVP_C128)
        p = p.cpu().numpy().reshape(n_r, n_theta)
        if reading == "sq":
            pw = abs(np.sum(p * p * R_)) * dr * dth / (2.0 * med["rho0"] * med["c0"])
        elif reading == "abs2_nor":
            pw = float(np.sum(np.abs(p) ** 2)) * dr * dth / (2.0 * med["rho0"] * med["c0"])
        else:
            raise ValueError("unknown power reading %r" % reading)
    return s * math.sqrt(power / pw)


def reference_mesh(T, med, d, n_max=5, eps=EPS):
    """The one mesh of the reference domain D_2 at lambda_{n_max} / 6, and the focal voxel."""
    l, R = T["l"], T["R"]
    L = math.sqrt(l * l - R * R) - eps
    lo, hi = (l - L, -R, -R), (l + d, R, R)
    h = nvp.spacing(med, T["f0"], n_max)
    g, i_f = nvp.grid_from_box((l, 0.0, 0.0), lo, hi, h)
    return g, tuple(int(v) for v in i_f), L


def domain_box(qbox, i_f, n):
    """The truncated integration domain for a localisation box: its pre-focal start and width, with
    everything beyond the focus along x kept (inclusive voxel indices lo_x, lo_y, lo_z, hi_x, hi_y, hi_z)."""
    return (min(int(qbox[0]), i_f[0]), int(qbox[1]), int(qbox[2]), int(n[0]) - 1, int(qbox[4]), int(qbox[5]))


def fractions(box, i_f, n):
    """(fraction_x, fraction_yz, extent_x): fraction_x = L' / L by voxel edges (the pre-focal lengths),
    fraction_yz = w' / w (the wider of y and z), extent_x = (L' + d) / (L + d) (the whole x extents,
    the post-focal part being the same)."""
    fx = (i_f[0] - box[0] + 0.5) / (i_f[0] + 0.5)
    fyz = max((box[4] - box[1] + 1) / n[1], (box[5] - box[2] + 1) / n[2])
    ex = (box[3] - box[0] + 1) / n[0]
    return fx, fyz, ex


def crossing(fr, err, target=TARGET):
    """The fraction at which the error curve (errors at increasing fractions) last falls below the
    target, read off by linear interpolation of log(error) between the two bracketing boxes."""
    ok = err < target
    i = len(ok)
    while i > 0 and ok[i - 1]:
        i -= 1
    if i == len(ok):
        return float("nan")
    if i == 0:
        return float(fr[0])
    a, b = math.log(err[i - 1]), math.log(max(err[i], 1e-300))
    t = (a - math.log(target)) / (a - b) if a != b else 1.0
    return float(fr[i - 1] + t * (fr[i] - fr[i - 1]))


def read_off(fr, err, q0, step=1.0, target=TARGET):
    """The fractions at which the error curve crosses the target, read as off a plot of it: only the
    thresholds on whole multiples of `step` (the paper's figures show its convergence at whole
    values of Q0), the smallest box from which on every larger one meets the target, and a straight
    line in error between it and the next smaller box."""
    idx = [i for i, q in enumerate(q0) if abs(q / step - round(q / step)) < 1e-9]
    fr, err = np.asarray(fr)[idx], np.asarray(err)[idx]
    ok = err < target
    i = len(ok)
    while i > 0 and ok[i - 1]:
        i -= 1
    if i == len(ok):
        return tuple(float("nan") for _ in range(fr.shape[1]))
    if i == 0:
        return tuple(float(v) for v in fr[0])
    t = (err[i - 1] - target) / (err[i - 1] - err[i]) if err[i - 1] != err[i] else 1.0
    return tuple(float(v) for v in fr[i - 1] + t * (fr[i] - fr[i - 1]))


def study(ctx, T, med, power, d, points, n_max=5, q0=Q0_LADDER, order=1, readings=("ref",), power_reading="abs2",
          log=None):
    """Axis errors of every ladder domain of every harmonic, per reading of the lower harmonics.

    Returns {reading: [per-harmonic record]}; each record holds the ladder's boxes, fractions and the
    two axis errors ("everywhere", "inside") and, per error, the smallest ladder domain from which on
    every larger one meets 1% and the interpolated 1% crossing."""
    g, i_f, L = reference_mesh(T, med, d, n_max)
    N = [int(v) for v in g.n]
    s = normalised_incident(ctx, T, med, power, points, reading=power_reading)
    k1 = nvp.wavenumber(med, T["f0"], 1)
    p1 = nvp.incident_field(ctx, k1, s, points, g)
    if log:
        log("reference mesh %s at %.2f um, focus voxel %s" % (N, g.h * 1e6, i_f))
    plan = nvp.CascadePlan(ctx, med, T["f0"], g, [g] * (n_max - 1), prec=nvp.NVP_C64, order=order)
    try:
        ref = [p1] + [t for t in plan.execute(p1)]
        axis = lambda t: t[:, i_f[1], i_f[2]].to(torch.complex128).cpu().numpy()  # noqa: E731
        ref_axis = [axis(t) for t in ref]
        norm1 = float(np.linalg.norm(ref_axis[0]))
        # the ladder's domains of every harmonic, from the localisation boxes of its reference source
        boxes = {}
        for n in range(2, n_max + 1):
            f_ref = plan.source_term(n, ref[:n - 1])
            qb = [b for i in range(0, len(q0), 32) for b in nvp.qbox(ctx, f_ref, q0[i:i + 32])]
            boxes[n] = [domain_box(b, i_f, N) for b in qb]
            del f_ref
        out = {}
        for reading in readings:
            errs = {n: np.zeros((len(q0), 2)) for n in range(2, n_max + 1)}

            def measure(n, j, p):
                a = axis(p)
                box = boxes[n][j]
                inside = np.zeros_like(a)
                inside[box[0]:box[3] + 1] = a[box[0]:box[3] + 1]
                errs[n][j, 0] = np.linalg.norm(a - ref_axis[n - 1]) / norm1
                errs[n][j, 1] = np.linalg.norm(inside - ref_axis[n - 1]) / norm1

            if reading == "ref":  # the truncated p_n from the reference lower harmonics
                for n in range(2, n_max + 1):
                    k, C = nvp.wavenumber(med, T["f0"], n), nvp.cascade_constant(med, T["f0"], n)
                    f = plan.source_term(n, ref[:n - 1])
                    for j in range(len(q0)):
                        measure(n, j, nvp.volume_potential_box(ctx, k, g, f, boxes[n][j], C))
                    del f
            elif reading == "trunc":  # every harmonic of the chain on its own domain of the same Q0
                for j in range(len(q0)):
                    chain = [p1]
                    for n in range(2, n_max + 1):
                        k, C = nvp.wavenumber(med, T["f0"], n), nvp.cascade_constant(med, T["f0"], n)
                        f = plan.source_term(n, chain)
                        p = nvp.volume_potential_box(ctx, k, g, f, boxes[n][j], C)
                        del f
                        measure(n, j, p)
                        chain.append(p)
                    del chain
            else:
                raise ValueError("reading must be 'ref' or 'trunc'")
            recs = []
            for n in range(2, n_max + 1):
                fr = np.array([fractions(b, i_f, N) for b in boxes[n]])
                rec = dict(n=n, q0=np.asarray(q0), boxes=boxes[n], fractions=fr, err=errs[n],
                           rel_norm=float(np.linalg.norm(ref_axis[n - 1])) / norm1)
                for e, name in ((0, "everywhere"), (1, "inside")):
                    ok = errs[n][:, e] < TARGET
                    i = len(ok)
                    while i > 0 and ok[i - 1]:
                        i -= 1
                    need = fr[i] if i < len(ok) else np.ones(3)
                    rec[name] = dict(ladder=tuple(float(v) for v in need),
                                     crossing=tuple(crossing(fr[:, c], errs[n][:, e]) for c in range(3)),
                                     read_off=read_off(fr, errs[n][:, e], q0))
                recs.append(rec)
                if log:
                    log("%s p%d: 1%% at L'/L %.2f, w'/w %.2f, extent %.2f (error everywhere on the axis); "
                        "%.2f, %.2f, %.2f (zero outside the domain); ||p%d|| / ||p1|| = %.3g" % (
                            reading, n, *rec["everywhere"]["ladder"], *rec["inside"]["ladder"], n, rec["rel_norm"]))
            out[reading] = recs
        return dict(mesh=N, h=g.h, i_f=i_f, L=L, readings=out)
    finally:
        plan.close()


def table(ctx, configs, n_points=4096, readings=("ref", "trunc"), power_reading="abs2", log=None):
    """Per configuration (name, transducer, medium, power, d): the study's fractions per reading, and
    every harmonic's error curve (thresholds, fractions, both axis errors)."""
    from workload import bowl
    rows = []
    for name, T, med, power, d in configs:
        pts = torch.from_numpy(bowl.bowl_points_deserno(T["R"], T["l"], n_points)).to("cuda")
        res = study(ctx, T, med, power, d, pts, readings=readings, power_reading=power_reading, log=log)
        row = dict(name=name, mesh=res["mesh"], h=res["h"], power_W=power, power_reading=power_reading)
        for reading, recs in res["readings"].items():
            for e in ("everywhere", "inside"):
                row["%s/%s" % (reading, e)] = [r[e] for r in recs]
            row["%s/rel_norms" % reading] = [r["rel_norm"] for r in recs]
            row["%s/curves" % reading] = [dict(q0=r["q0"], fractions=r["fractions"], err=r["err"]) for r in recs]
        rows.append(row)
        torch.cuda.empty_cache()
    return rows


# The paper's three configurations of the domain table (Section 5).
def paper_configs(water):
    from workload import configs
    W, Lv = water, configs.LIVER
    return [("H131 water 100W", H131, W, 100.0, H131_D), ("H131 water 150W", H131, W, 150.0, H131_D),
            ("H131 liver 100W", H131, Lv, 100.0, H131_D)]


def main():
    import argparse
    import json
    import time
    from workload import configs
    ap = argparse.ArgumentParser(description="Section 5 domain study on the paper's H131 configurations")
    ap.add_argument("--out", default="truncation_study.json")
    ap.add_argument("--water", choices=("build", "table"), default="build",
                    help="water constants: the build's c 1487 / rho 998, or the paper's table c 1480 / rho 1000")
    ap.add_argument("--readings", default="ref,trunc")
    ap.add_argument("--only", default="", help="comma-separated configuration names")
    ap.add_argument("--power-reading", choices=("abs2", "sq", "abs2_nor"), default="abs2")
    ap.add_argument("--power-scale", type=float, default=1.0, help="multiplies every configuration's power")
    a = ap.parse_args()
    water = dict(configs.WATER) if a.water == "build" else dict(configs.WATER, c0=1480.0, rho0=1000.0)
    cfgs = [(nm, T, med, pw * a.power_scale, d) for nm, T, med, pw, d in paper_configs(water)
            if not a.only or nm in a.only.split(",")]
    t0 = time.time()
    with nvp.Context(0) as ctx:
        rows = table(ctx, cfgs, readings=tuple(a.readings.split(",")), power_reading=a.power_reading,
                     log=lambda m: print(m, flush=True))
    out = dict(water=water, seconds=time.time() - t0, rows=rows)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1, default=lambda v: v.tolist() if hasattr(v, "tolist") else float(v))
    print("wrote %s in %.0f s" % (a.out, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
