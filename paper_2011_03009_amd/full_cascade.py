"""The harmonic cascade with the difference-frequency terms that the paper drops.

Equation "cascade_1" of Section 2 gives harmonic n the source
S_n + D_n, S_n = sum_{m<n} p_m p_{n-m} (kept by the paper's "cascade_2") and
D_n = 2 sum_{m=n+1}^{N} p_m conj(p_{m-n}) (dropped there, p_1 included, since it
carries energy from the higher harmonics back down).  With N harmonics kept,
the truncated system is solved by fixed-point sweeps: sweep 0 is the paper's
cascade; each later sweep recomputes p_1, ..., p_N in order from the newest
values,

    p_n = [n = 1] p_inc + C_n sum_j K_{k_n}(x_i - x_j) (S_n + D_n)(x_j),

until no harmonic changes by more than `tol` (relative L2).  Lower harmonics
are transferred onto p_n's grid as in Section 6; a higher harmonic is zero
outside its own box (zero outside the hull of its voxel centres).

The library does the numerics: S_n by the plan's source build, D_n by
nvp_difference_term, C_n times the convolution by nvp_volume_potential_box,
p_inc added by nvp_field_lin3 and the change of each harmonic by
nvp_field_diff_norms.  This module only orders the calls.
"""

import torch

from . import nvp


def full_cascade(ctx, med, f0, g1, grids, p_inc, order=1, tol=1e-6, max_sweeps=30, log=None):
    """Returns ([p_1, ..., p_N], sweeps, last relative change, [paper's p_2, ..., p_N]).

    p_inc: the incident field on g1 (complex64 or complex128 CUDA tensor); grids: grids of
    p_2..p_N.  The plan and the volume potentials use the context's quadrature rule."""
    prec = nvp.prec_of(p_inc.dtype)
    g = [nvp.grid(g1)] + [nvp.grid(x) for x in grids]
    N = len(g)
    plan = nvp.CascadePlan(ctx, med, f0, g1, grids, prec=prec, order=order)
    try:
        paper = plan.execute(p_inc)
        p = [p_inc.clone()] + [t.clone() for t in paper]
        change, sweeps = float("inf"), 0
        while change > tol and sweeps < max_sweeps:
            sweeps += 1
            change = 0.0
            for n in range(1, N + 1):
                gn = g[n - 1]
                if n >= 2:
                    f = plan.source_term(n, p[:n - 1])
                else:
                    f = torch.zeros(tuple(gn.n), dtype=p_inc.dtype, device=p_inc.device)
                for m in range(n + 1, N + 1):
                    nvp.difference_term(ctx, gn, f, g[m - 1], p[m - 1], True, g[m - n - 1], p[m - n - 1],
                                        m - n > n, order, 2.0)
                new = nvp.volume_potential_box(ctx, nvp.wavenumber(med, f0, n), gn, f, None,
                                               nvp.cascade_constant(med, f0, n))
                del f
                if n == 1:
                    nvp.field_lin3(ctx, new, new, p_inc, None, 1.0, 0.0)
                dd, nn = nvp.field_diff_norms(ctx, new, p[n - 1])
                change = max(change, (dd / nn) ** 0.5 if nn > 0 else 0.0)
                p[n - 1] = new
            if log:
                log("sweep %d: largest relative change %.2e" % (sweeps, change))
        return p, sweeps, change, paper
    finally:
        plan.close()
