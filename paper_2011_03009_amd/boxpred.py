"""Learned truncation boxes: convergence sweeps, training data, guarded prediction.

The paper chooses each harmonic's integration domain by a rule of thumb
(Section 5): boxes whose pre-focal length and width are fixed fractions of a
reference domain, after observing in truncation-convergence tests that the
fractions needed for 1% error differ between transducers and media.  Here a
small network predicts those fractions per transducer and harmonic instead:

* A sweep runs the plain method on the reference domain of one transducer and
  truncates the source of every harmonic to the localisation boxes
  {Q >= Q0} of Section 5 for a ladder of thresholds Q0; the smallest box
  beyond which the focal value of p_n stays within the error target is the
  label (x: fraction of the pre-focal length, y and z: fractions of the
  half-width; the post-focal distance is kept whole, as in the paper).
* The network (nvp_boxnet) is trained on the sweeps with a pinball loss of a
  high quantile, which biases it towards boxes that are too large rather than
  too small.
* A prediction is used through a guard: after computing p_n on the predicted
  box, the focal value with the source cut to the box and to a box shrunk by
  a factor is compared (one more step of the same convergence sweep); when
  they differ by more than the guard tolerance, p_n is recomputed on the full
  reference box.

All computation runs in the library (cascade plans, source terms, box
reductions, truncated potentials, the network); this module is host logic.
The incident field is the caller's input: every function that needs p_1 takes
a callable incident(transducer, grid) returning it as a complex64 CUDA tensor.
"""

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import nvp

# Reference window in first-harmonic wavelengths: pre-focal length, post-focal
# distance and lateral half-width (each also capped by the transducer's own
# reference domain [l - L, l + d] x [-R, R]^2 with L = sqrt(l^2 - R^2) - eps).
WINDOW = (10.0, 2.0, 4.0)
# Thresholds Q0 of the sweep, from the tightest box to the loosest.
Q0_LADDER = tuple(-0.25 * i for i in range(1, 25))
MIN_HALF = 2  # smallest half-width in voxels (a grid keeps >= 5 voxels per axis for cubic transfer)
EPS = 0.01  # error target of the focal value of each harmonic
# Guard: largest relative change of the focal value between a box and the box
# shrunk by 0.8 that is accepted without falling back to the window.  On 2000
# sweeps of the batched workload's transducers no ladder box within this
# tolerance missed the 1% target.
GUARD_DELTA = 0.01
GUARD_SHRINK = 0.8


@dataclass
class Transducer:
    R: float      # aperture radius (m)
    l: float      # focal length (m)
    f0: float     # frequency (Hz)
    p0: float     # surface pressure (Pa)
    n_harm: int   # harmonics computed

    def features(self, n):
        return [self.R, self.l, self.f0, self.p0, float(n)]


class Geometry:
    """Reference window and voxel boxes of one transducer (focus at (l, 0, 0), axis along x)."""

    def __init__(self, T, med, window=WINDOW):
        self.T, self.med = T, med
        lam1 = med["c0"] / T.f0
        # eps: half a wavelength, so that p_1's grid with its margin stays clear of the bowl's rim
        self.L = min(math.sqrt(T.l * T.l - T.R * T.R) - 0.5 * lam1, window[0] * lam1)
        self.d = window[1] * lam1
        self.w = min(T.R, window[2] * lam1)
        self.focus = (T.l, 0.0, 0.0)

    def h(self, n):
        return nvp.spacing(self.med, self.T.f0, n)

    def half_counts(self, n, frac):
        """(pre, post, half_y, half_z) voxel counts of the box with fractions frac on harmonic n's lattice."""
        h = self.h(n)
        pre = max(MIN_HALF, math.ceil(frac[0] * self.L / h - 1e-9))
        post = max(MIN_HALF, math.ceil(self.d / h - 1e-9))
        hy = max(MIN_HALF, math.ceil(frac[1] * self.w / h - 1e-9))
        hz = max(MIN_HALF, math.ceil(frac[2] * self.w / h - 1e-9))
        return pre, post, hy, hz

    def grid(self, n, frac=(1.0, 1.0, 1.0)):
        pre, post, hy, hz = self.half_counts(n, frac)
        return nvp.grid_from_counts(self.focus, self.h(n), (pre + post + 1, 2 * hy + 1, 2 * hz + 1), (pre, hy, hz))

    def g1(self, margin=2):
        """p_1's grid at lambda_1/6, covering the whole window with a margin for the transfer stencils."""
        pre, post, hy, hz = self.half_counts(1, (1.0, 1.0, 1.0))
        pre, post, hy, hz = pre + margin, post + margin, hy + margin, hz + margin
        return nvp.grid_from_counts(self.focus, self.h(1), (pre + post + 1, 2 * hy + 1, 2 * hz + 1), (pre, hy, hz))

    def sub_box(self, n, frac, within):
        """Voxel box (lo xyz, hi xyz) of fractions frac inside the box of fractions `within` (same lattice)."""
        pre, _, hy, hz = self.half_counts(n, frac)
        wpre, wpost, why, whz = self.half_counts(n, within)
        pre, hy, hz = min(pre, wpre), min(hy, why), min(hz, whz)
        return [wpre - pre, why - hy, whz - hz, wpre + wpost, why + hy, whz + hz]

    def fractions_of(self, n, box, frac=(1.0, 1.0, 1.0)):
        """Fractions of the smallest window box that holds a voxel box of the grid with fractions frac."""
        h = self.h(n)
        pre, _, hy, hz = self.half_counts(n, frac)
        fx = max(0, pre - int(box[0])) * h / self.L
        fy = max(hy - int(box[1]), int(box[4]) - hy, 0) * h / self.w
        fz = max(hz - int(box[2]), int(box[5]) - hz, 0) * h / self.w
        return (min(1.0, fx), min(1.0, fy), min(1.0, fz))


def voxels(g):
    return int(g.n[0]) * int(g.n[1]) * int(g.n[2])


def _focal_index(geo, n, frac):
    pre, _, hy, hz = geo.half_counts(n, frac)
    return (pre, hy, hz)


# ------------------------------------------------------------------ sweeps

def sweep(ctx, T, med, incident, n_max=5, q0=Q0_LADDER, shrink=GUARD_SHRINK, order=3):
    """Truncation-convergence sweep of harmonics 2..n_max of one transducer.

    For each harmonic n and each threshold of the ladder: the fractions of the
    window box that holds the localisation box {Q >= Q0} of f_n, the relative
    change err of the focal value of p_n when the source is cut to that box
    (against the whole window), and the guard statistic delta: the relative
    change between that box and the box shrunk by `shrink`.  Lower harmonics
    are the window (reference) solutions.
    """
    geo = Geometry(T, med)
    g1 = geo.g1()
    full = [geo.grid(n) for n in range(2, n_max + 1)]
    plan = nvp.CascadePlan(ctx, med, T.f0, g1, full, prec=nvp.NVP_C64, order=order)
    fields = [incident(T, g1)]
    recs = []
    try:
        for n in range(2, n_max + 1):
            g = full[n - 2]
            f = plan.source_term(n, fields)
            qb = nvp.qbox(ctx, f, q0)
            fr = [geo.fractions_of(n, b) for b in qb]
            cand = [geo.sub_box(n, c, (1.0, 1.0, 1.0)) for c in fr]
            small = [geo.sub_box(n, tuple(shrink * v for v in c), (1.0, 1.0, 1.0)) for c in fr]
            whole = [0, 0, 0, int(g.n[0]) - 1, int(g.n[1]) - 1, int(g.n[2]) - 1]
            k = nvp.wavenumber(med, T.f0, n)
            t = _focal_index(geo, n, (1.0, 1.0, 1.0))
            u = nvp.box_potential(ctx, k, g, f, t, cand + [whole])
            us = nvp.box_potential(ctx, k, g, f, t, small)
            err = np.abs(u[:-1] - u[-1]) / abs(u[-1])
            delta = np.abs(u[:-1] - us) / np.abs(u[:-1])
            recs.append(dict(n=n, fractions=np.asarray(fr), err=err, delta=delta, q0=np.asarray(q0)))
            if n < n_max:
                fields.append(plan.execute_harmonic(n, fields))
    finally:
        plan.close()
    return recs


def label(rec, eps=EPS, delta_max=GUARD_DELTA):
    """Fractions of the smallest ladder box from which on every larger box keeps err <= eps and passes
    the guard (delta <= delta_max); the whole window when there is none."""
    err, delta = rec["err"], rec["delta"]
    for i in range(len(err)):
        if np.all(err[i:] <= eps) and np.all(delta[i:] <= delta_max):
            return tuple(float(v) for v in rec["fractions"][i])
    return (1.0, 1.0, 1.0)


def dataset(records, eps=EPS, delta_max=GUARD_DELTA):
    """(x [S][5], t [S][3]) float32 arrays from [(Transducer, sweep records)]."""
    xs, ts = [], []
    for T, recs in records:
        for r in recs:
            xs.append(T.features(r["n"]))
            ts.append(label(r, eps, delta_max))
    return np.asarray(xs, dtype=np.float32), np.asarray(ts, dtype=np.float32)


def guard_safety(records, eps=EPS, delta_max=GUARD_DELTA):
    """Share of the sweeps' ladder boxes that pass the guard yet miss the error target (the guard's
    false-pass rate on these sweeps), and the number of boxes that pass it."""
    err = np.concatenate([r["err"] for _, rs in records for r in rs])
    delta = np.concatenate([r["delta"] for _, rs in records for r in rs])
    ok = delta <= delta_max
    return float(np.mean(err[ok] > eps)) if ok.any() else 0.0, int(ok.sum())


# ------------------------------------------------------------------ training

def train(ctx, x, t, init_params, mean, std, steps=3000, lr=3e-3, tau=0.9, log=None):
    """Full-batch Adam on the pinball loss; returns the trained nvp.BoxNet and the loss history."""
    net = nvp.BoxNet(ctx, max(1, x.shape[0]))
    net.set_params(init_params)
    net.set_norm(mean, std)
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(ctx.device)
    td = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).to(ctx.device)
    hist = []
    for s in range(steps):
        rate = lr * (0.1 ** (s / max(1, steps)))  # exponential decay to lr / 10
        want = s % 100 == 0 or s == steps - 1
        L = net.train_step(xd, td, tau, rate, want_loss=want)
        if want:
            hist.append((s, L))
            if log:
                log("train step %d loss %.5f" % (s, L))
    return net, hist


def predict_fractions(net, T, ctx):
    """Monotone fractions {n: (fx, fy, fz)} for harmonics 2..n_harm, clipped to [0, 1].

    Each harmonic's box is kept inside the previous one's, so that every
    transferred lower harmonic is known on the whole box it is needed on.
    """
    x = torch.tensor([T.features(n) for n in range(2, T.n_harm + 1)], dtype=torch.float32, device=ctx.device)
    y = net.predict(x).cpu().numpy().astype(np.float64)
    out, prev = {}, (1.0, 1.0, 1.0)
    for i, n in enumerate(range(2, T.n_harm + 1)):
        f = tuple(float(min(max(v, 0.0), p)) for v, p in zip(y[i], prev))
        out[n] = f
        prev = f
    return out


def rule_of_thumb_fractions(T):
    """The paper's rule: length and width of D_n scaled by lambda_n / lambda_2 = 2 / n."""
    return {n: (min(1.0, 2.0 / n),) * 3 for n in range(2, T.n_harm + 1)}


# ------------------------------------------------------------------ guarded nested run

def run_boxes(ctx, T, med, incident, fractions, guard=None, shrink=GUARD_SHRINK, order=3):
    """Nested cascade of T on the boxes `fractions`; with a guard, fall back to the full box per harmonic.

    Returns focal values {n: complex}, the voxels of every grid computed
    (fallbacks count both), the harmonics that fell back, and the wall time
    of the cascade (plans, kernels, guards; p_1 excluded).
    """
    geo = Geometry(T, med)
    g1 = geo.g1()
    frac = dict(fractions)
    p1 = incident(T, g1)
    torch.cuda.synchronize(ctx.device)
    t0 = time.perf_counter()
    grids = [geo.grid(n, frac[n]) for n in range(2, T.n_harm + 1)]
    plan = nvp.CascadePlan(ctx, med, T.f0, g1, grids, prec=nvp.NVP_C64, order=order)
    fields, focal, fallbacks, vox = [p1], {}, [], 0
    try:
        for n in range(2, T.n_harm + 1):
            p = plan.execute_harmonic(n, fields)
            vox += voxels(grids[n - 2])
            if guard is not None and frac[n] != (1.0, 1.0, 1.0):
                f = plan.source_term(n, fields)
                g = grids[n - 2]
                whole = [0, 0, 0, int(g.n[0]) - 1, int(g.n[1]) - 1, int(g.n[2]) - 1]
                small = geo.sub_box(n, tuple(shrink * v for v in frac[n]), frac[n])
                u = nvp.box_potential(ctx, nvp.wavenumber(med, T.f0, n), g, f, _focal_index(geo, n, frac[n]),
                                      [whole, small])
                if abs(u[0] - u[1]) > guard * abs(u[0]):
                    # fall back to the full box for this harmonic only: the plan is re-laid
                    # out for its grid, the kernel spectra of the others are kept
                    fallbacks.append(n)
                    frac[n] = (1.0, 1.0, 1.0)
                    grids[n - 2] = geo.grid(n)
                    plan.regrid(n, grids[n - 2])
                    p = plan.execute_harmonic(n, fields)
                    vox += voxels(grids[n - 2])
            fields.append(p)
            i_f = _focal_index(geo, n, frac[n])
            focal[n] = complex(p[i_f].item())
        torch.cuda.synchronize(ctx.device)
    finally:
        plan.close()
    return dict(focal=focal, voxels=vox, fallbacks=fallbacks, ms=1e3 * (time.perf_counter() - t0),
                fractions=frac)


def evaluate(ctx, transducers, med, incident, net=None, guard=GUARD_DELTA, log=None):
    """Full box vs rule of thumb vs the network (with guard) on each transducer.

    Errors are |p_n(focus) - p_n^ref(focus)| / |p_n^ref(focus)| against the
    full reference box.  Returns per-transducer rows and totals.
    """
    rows = []
    for i, T in enumerate(transducers):
        ref = run_boxes(ctx, T, med, incident, {n: (1.0, 1.0, 1.0) for n in range(2, T.n_harm + 1)})
        row = dict(T=T, full=ref)
        runs = [("rule", rule_of_thumb_fractions(T), None)]
        if net is not None:
            runs.append(("net", predict_fractions(net, T, ctx), guard))
        for name, fr, gd in runs:
            r = run_boxes(ctx, T, med, incident, fr, guard=gd)
            r["err"] = {n: abs(r["focal"][n] - ref["focal"][n]) / abs(ref["focal"][n]) for n in ref["focal"]}
            row[name] = r
        rows.append(row)
        if log:
            msg = "eval %d/%d full %d vox" % (i + 1, len(transducers), ref["voxels"])
            for name in ("rule", "net"):
                if name in row:
                    msg += " | %s %d vox max err %.2e fb %s" % (name, row[name]["voxels"],
                                                              max(row[name]["err"].values()),
                                                              row[name]["fallbacks"])
            log(msg)
    tot = {"full": dict(voxels=sum(r["full"]["voxels"] for r in rows), ms=sum(r["full"]["ms"] for r in rows))}
    for name in ("rule", "net"):
        if rows and name in rows[0]:
            errs = [e for r in rows for e in r[name]["err"].values()]
            tot[name] = dict(voxels=sum(r[name]["voxels"] for r in rows), ms=sum(r[name]["ms"] for r in rows),
                             max_err=max(errs), n_over_1pct=int(sum(e > 0.01 for e in errs)),
                             fallbacks=sum(len(r[name]["fallbacks"]) for r in rows),
                             harmonics=len(errs))
            tot[name]["voxel_gain"] = tot["full"]["voxels"] / tot[name]["voxels"]
            tot[name]["time_gain"] = tot["full"]["ms"] / tot[name]["ms"]
    return rows, tot


# ------------------------------------------------------------------ trained weights

DATA = __file__.rsplit("/", 1)[0] + "/data"


def save_net(net, path, meta):
    """Parameters (float32 .npy) and a JSON description beside them."""
    import json
    np.save(path + ".npy", net.get_params())
    with open(path + ".json", "w") as fh:
        json.dump(meta, fh, indent=1, default=float)


def load_net(ctx, path=DATA + "/boxnet_window", max_batch=64):
    """A BoxNet with the stored parameters and input standardisation."""
    import json
    meta = json.load(open(path + ".json"))
    net = nvp.BoxNet(ctx, max_batch)
    net.set_params(np.load(path + ".npy", allow_pickle=False))
    net.set_norm(meta["norm_mean"], meta["norm_std"])
    return net, meta
