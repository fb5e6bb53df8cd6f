"""The truncation-convergence study of Section 5 at the paper's scale.

For one transducer and medium, every harmonic p_2..p_n is first computed on
the reference domain (equation "domain": [l - L, l + d] x [-R, R]^2, each
harmonic at its own lambda_n / 6); these are the reference solutions p_n^r.
Then, for each harmonic, the source f_n (built from the reference lower
harmonics) is cut to the localisation boxes {Q >= Q0} of Section 5
(Q = log10(|f| / max |f|)) for a ladder of thresholds, the volume potential
of each cut source is taken, and its error is measured as the paper does,
along the x axis and relative to the first harmonic:

    error = || p_n - p_n^r || / || p_1^r ||   (discrete L2 over the axis voxels).

The fractions of the reference domain that a box needs for an error below 1%
are the study's result (the paper's table of domain sizes); the paper reads
them off its convergence plots.  The incident field is the GPU monopole sum,
normalised to the prescribed radiated power.

Every numeric step runs in the library (incident field, power, cascade plan,
source terms, localisation boxes, volume potentials); this module chooses the
boxes, masks the sources and reduces the axis norms.
"""

import math

import numpy as np
import torch

from . import boxpred, nvp

# Transducers of the paper's Table of transducers (f0, focal length l, outer radius R).
H131 = dict(f0=1.1e6, l=35e-3, R=16.5e-3)
H101 = dict(f0=1.1e6, l=63.2e-3, R=32e-3)
# Post-focal distance d of H131's reference domain: the paper's mesh of 901 x 732 x 732 voxels
# at lambda_5 / 6 has an x extent of L + d with L = sqrt(l^2 - R^2).
H131_D = 9.8e-3
Q0_LADDER = tuple(-0.25 * i for i in range(1, 33))
TARGET = 0.01


def cap_height(T):
    return T["l"] - math.sqrt(T["l"] ** 2 - T["R"] ** 2)


def normalised_incident(ctx, T, med, power, points, n_r=256, n_theta=256):
    """Scale of the bowl's monopole sum (points: float64 CUDA tensor [n, 3] on the cap) that makes it
    radiate `power` watts through the rim-plane disc: the paper's (A / n) sum G times sqrt(P0 / P)."""
    k1 = nvp.wavenumber(med, T["f0"], 1)
    area = 2.0 * math.pi * T["l"] * cap_height(T)
    s = area / points.shape[0]
    centre = (cap_height(T), 0.0, 0.0)
    pw = nvp.radiated_power(ctx, k1, s, points, centre, T["R"], med["rho0"], med["c0"], n_r, n_theta)
    return s * math.sqrt(power / pw)


def study(ctx, T, med, power, d, points, n_max=5, q0=Q0_LADDER, order=1, log=None):
    """Axis errors of every ladder box of every harmonic; returns a list of per-harmonic records.

    points: the bowl's source points (float64 CUDA tensor [n, 3]); d: post-focal distance of the
    reference domain; order: transfer order (the paper's is linear)."""
    lam1 = med["c0"] / T["f0"]
    tr = boxpred.Transducer(R=T["R"], l=T["l"], f0=T["f0"], p0=0.0, n_harm=n_max)
    geo = boxpred.Geometry(tr, med, window=(1e9, d / lam1, 1e9))
    g1 = geo.g1()
    grids = [geo.grid(n) for n in range(2, n_max + 1)]
    pts = points
    s = normalised_incident(ctx, T, med, power, pts)
    k1 = nvp.wavenumber(med, T["f0"], 1)
    p1 = nvp.incident_field(ctx, k1, s, pts, g1)
    plan = nvp.CascadePlan(ctx, med, T["f0"], g1, grids, prec=nvp.NVP_C64, order=order)
    fields = [p1]
    out = []
    try:
        for n in range(2, n_max + 1):
            g = grids[n - 2]
            pre, _, hy, hz = geo.half_counts(n, (1.0, 1.0, 1.0))
            xs = g.origin[0] + np.arange(int(g.n[0])) * g.h
            axis_pts = torch.tensor(np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1), device="cuda")
            p1_axis = nvp.incident_at(ctx, k1, s, pts, axis_pts, prec=nvp.NVP_C128)
            norm1 = float(torch.linalg.vector_norm(p1_axis))
            f = plan.source_term(n, fields)
            k, C = nvp.wavenumber(med, T["f0"], n), nvp.cascade_constant(med, T["f0"], n)
            # p_n = C_n sum K f = -C_n u, with u the raw operator's output
            ref = -C * nvp.volume_potential(ctx, k, g, f)[:, hy, hz].to(torch.complex128)
            boxes = nvp.qbox(ctx, f, q0)
            errs, fracs, sizes = [], [], []
            for b in boxes:
                sizes.append(((b[3] - b[0] + 1) / g.n[0], max((b[4] - b[1] + 1) / g.n[1], (b[5] - b[2] + 1) / g.n[2])))
                fm = torch.zeros_like(f)
                sl = (slice(b[0], b[3] + 1), slice(b[1], b[4] + 1), slice(b[2], b[5] + 1))
                fm[sl] = f[sl]
                u = -C * nvp.volume_potential(ctx, k, g, fm)[:, hy, hz].to(torch.complex128)
                errs.append(float(torch.linalg.vector_norm(u - ref)) / norm1)
                fracs.append(geo.fractions_of(n, b))
            errs, fracs = np.asarray(errs), np.asarray(fracs)
            # the smallest ladder box from which on every larger box meets the target
            ok = errs < TARGET
            i = len(ok)
            while i > 0 and ok[i - 1]:
                i -= 1
            need = fracs[i] if i < len(ok) else np.ones(3)
            size = sizes[i] if i < len(ok) else (1.0, 1.0)
            # need_x / need_yz: pre-focal length and half-width as fractions of the reference
            # domain's; size_x / size_yz: the box's whole x extent and width as fractions of the
            # reference domain's (the paper's L' = fraction_x L, w' = fraction_yz w)
            rec = dict(n=n, grid=[int(v) for v in g.n], q0=np.asarray(q0), err=errs, fractions=fracs,
                       need_x=float(need[0]), need_yz=float(max(need[1], need[2])),
                       size_x=float(size[0]), size_yz=float(size[1]),
                       rel_norm=float(torch.linalg.vector_norm(ref)) / norm1)
            out.append(rec)
            if log:
                log("p%d on %s, < 1%% axis error: extent x %.2f, y/z %.2f (pre-focal %.2f, half-width %.2f) of the "
                    "reference domain; ||p%d|| / ||p1|| = %.3g" % (n, rec["grid"], rec["size_x"], rec["size_yz"],
                                                                  rec["need_x"], rec["need_yz"], n, rec["rel_norm"]))
            if n < n_max:
                fields.append(plan.execute_harmonic(n, fields))
    finally:
        plan.close()
    return out


def table(ctx, configs, n_points=4096, log=None):
    """Rows (name, per-harmonic (x, y/z) fractions) for a list of (name, transducer, medium, power, d).

    The bowl carries about n_points monopoles in Deserno's regular placement, as in the paper."""
    from workload import bowl
    rows = []
    for name, T, med, power, d in configs:
        pts = torch.from_numpy(bowl.bowl_points_deserno(T["R"], T["l"], n_points)).to("cuda")
        recs = study(ctx, T, med, power, d, pts, log=log)
        rows.append(dict(name=name, extent=[(r["size_x"], r["size_yz"]) for r in recs],
                         prefocal=[(r["need_x"], r["need_yz"]) for r in recs],
                         rel_norms=[r["rel_norm"] for r in recs], grids=[r["grid"] for r in recs]))
    return rows
