"""The inhomogeneous example of Section 7: H131 at 50 W in water with a 2 cm layer of kidney
centred on the focus (kidney density taken equal to water's, as the paper does).

Every harmonic solves the volume integral equation of the inhomogeneous medium,
    p_n - V_kb[(k_n(x)^2 - kb_n^2) p_n] = rhs_n,
with the water wavenumber kb_n as background: p_1 with the incident field of the
bowl (normalised to the radiated power in water) on the right, p_n (n >= 2) with
C_n(x) V_kb[f_n], f_n = sum_m p_m p_{n-m} transferred onto p_n's grid and C_n(x)
the cascade constant of the medium at x.  Each harmonic lives on its own
lambda_n / 6 grid of the reference domain.  The homogeneous water cascade is
run beside it for comparison.

The library does the numerics (incident field, power, source terms, volume
potentials scaled by C_n, the slab's rescaling of the right-hand side, the
BiCGStab solves); this module lays out the layer on the grids.  In complex128
the solves reach a true relative residual of 1e-6 and below; in complex64 the
rounding of the FP32 operator stalls them near 5e-6.
"""

import time

import numpy as np
import torch

from . import boxpred, nvp
from .truncation_study import H131, H131_D, normalised_incident

# Kidney as the paper's table of media gives it, with water's density (Section 7).
KIDNEY_TABLE = dict(c0=1570.0, beta=4.7, alpha0_db=10.0, eta=1.0)


def _slab_range(g, lo, hi):
    """x-index range [a, b) of the voxel centres with lo <= x < hi."""
    x = g.origin[0] + np.arange(int(g.n[0])) * g.h
    idx = np.nonzero((x >= lo) & (x < hi))[0]
    return (int(idx[0]), int(idx[-1]) + 1) if idx.size else (0, 0)


def slab(ctx, water, points, power=50.0, width=20e-3, n_max=3, order=1, tol=1e-6, prec=nvp.NVP_C64,
         max_iter=400, log=None):
    T = H131
    kidney = dict(water, **KIDNEY_TABLE)
    lam1 = water["c0"] / T["f0"]
    tr = boxpred.Transducer(R=T["R"], l=T["l"], f0=T["f0"], p0=0.0, n_harm=n_max)
    geo = boxpred.Geometry(tr, water, window=(1e9, H131_D / lam1, 1e9))
    g1 = geo.g1()
    grids = [geo.grid(n) for n in range(2, n_max + 1)]
    lo, hi = T["l"] - width / 2, T["l"] + width / 2
    s = normalised_incident(ctx, T, water, power, points)
    k1 = nvp.wavenumber(water, T["f0"], 1)
    p_inc = nvp.incident_field(ctx, k1, s, points, g1, prec=prec)
    plan = nvp.CascadePlan(ctx, water, T["f0"], g1, grids, prec=prec, order=order)
    hom = plan.execute(p_inc)  # the homogeneous water cascade
    torch.cuda.synchronize()
    rows = []
    fields = []
    try:
        for n in range(1, n_max + 1):
            g = g1 if n == 1 else grids[n - 2]
            kb, kk = nvp.wavenumber(water, T["f0"], n), nvp.wavenumber(kidney, T["f0"], n)
            a, b = _slab_range(g, lo, hi)
            q = torch.zeros(tuple(g.n), dtype=p_inc.dtype, device="cuda")
            q[a:b] = complex(kk * kk - kb * kb)
            t0 = time.perf_counter()
            if n == 1:
                rhs = p_inc
            else:
                f = plan.source_term(n, fields)
                cw, ck = nvp.cascade_constant(water, T["f0"], n), nvp.cascade_constant(kidney, T["f0"], n)
                rhs = nvp.volume_potential_box(ctx, kb, g, f, None, cw)  # C_n(water) V[f]
                del f
                if b > a:  # the layer's x-slab (contiguous rows) carries the kidney's C_n
                    nvp.field_lin3(ctx, rhs[a:b], None, rhs[a:b], None, ck / cw, 0.0)
            p, it, rr = nvp.vie_solve(ctx, kb, g, q, rhs, tol=tol, max_iter=max_iter)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            fields.append(p)
            i_f = [int(round((c - o) / g.h)) for c, o in zip((T["l"], 0.0, 0.0), g.origin)]
            ref = p_inc if n == 1 else hom[n - 2]
            axis = p[:, i_f[1], i_f[2]].abs()
            axis_w = ref[:, i_f[1], i_f[2]].abs()
            row = dict(n=n, grid=[int(v) for v in g.n], iterations=it, relres=rr, seconds=dt,
                       focal_slab=float(axis[i_f[0]]), focal_water=float(axis_w[i_f[0]]),
                       axis_max_slab=float(axis.max()), axis_max_water=float(axis_w.max()),
                       peak_x_slab=float(g.origin[0] + int(axis.argmax()) * g.h),
                       peak_x_water=float(g.origin[0] + int(axis_w.argmax()) * g.h))
            rows.append(row)
            if log:
                log("p%d on %s: %d BiCGStab iterations (residual %.1e) in %.2f s; |p| at the focus %.4g Pa "
                    "(water %.4g); on-axis peak %.4g Pa at x = %.2f mm (water %.4g at %.2f mm)"
                    % (n, row["grid"], it, rr, dt, row["focal_slab"], row["focal_water"], row["axis_max_slab"],
                       row["peak_x_slab"] * 1e3, row["axis_max_water"], row["peak_x_water"] * 1e3))
    finally:
        plan.close()
    return rows


def main():
    import argparse
    import json
    from workload import bowl, configs
    ap = argparse.ArgumentParser(description="Section 7's kidney-layer example (H131, 50 W, 2 cm layer)")
    ap.add_argument("--prec", choices=("c64", "c128"), default="c128")
    ap.add_argument("--n-max", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--out", default="slab_study.json")
    a = ap.parse_args()
    T = H131
    pts = torch.from_numpy(bowl.bowl_points_deserno(T["R"], T["l"], 4096)).to("cuda")
    prec = nvp.NVP_C128 if a.prec == "c128" else nvp.NVP_C64
    with nvp.Context(0) as ctx:
        rows = slab(ctx, configs.WATER, pts, n_max=a.n_max, tol=a.tol, prec=prec, max_iter=a.max_iter,
                    log=lambda m: print(m, flush=True))
    with open(a.out, "w") as fh:
        json.dump(dict(prec=a.prec, tol=a.tol, rows=rows), fh, indent=1)


if __name__ == "__main__":
    main()
