"""Train the box predictor on convergence sweeps and evaluate it against the full box and the rule of thumb.

  python -m paper_2011_03009_amd.train_boxnet --transducers 500 --eval 64 --out boxnet_out

Training transducers are drawn from the batched workload's ranges with one
seed, the held-out ones with another; p_1 is the Rayleigh integral of a
seeded equal-area point set on each bowl (synthetic stand-ins for measured
transducers), summed on the GPU by the library's incident-field kernel.  Writes dataset.npz, boxnet_window.npy/.json (the trained network) and summary.json to --out.
"""

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2011_03009_amd import boxpred as BP  # noqa: E402
from paper_2011_03009_amd import nvp  # noqa: E402
from workload import bowl, configs, learn as WL  # noqa: E402

MED = configs.WATER


def make_incident(ctx, n_points=4096, seed=0):
    """p_1 of a transducer on a grid: the library's monopole sum (nvp_incident_field) over a seeded
    equal-area point set on the bowl, scaled to the Rayleigh integral of surface pressure p0."""
    def incident(T, g):
        k1 = nvp.wavenumber(MED, T.f0, 1)
        pts = torch.from_numpy(bowl.bowl_points(T.R, T.l, n_points, seed)).to("cuda")
        return nvp.incident_field(ctx, k1, bowl.rayleigh_scale(T.R, T.l, k1, T.p0, n_points), pts, g)
    return incident


def transducers(count, seed):
    return [BP.Transducer(**d) for d in configs.batch_transducers(count, seed)]


def log(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--transducers", type=int, default=500)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--eval-seed", type=int, default=0)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--sweep-only", action="store_true")
    ap.add_argument("--tau", type=float, default=0.9)
    ap.add_argument("--guard", type=float, default=BP.GUARD_DELTA)
    ap.add_argument("--eps", type=float, default=BP.EPS)
    ap.add_argument("--out", default="boxnet_out")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    with nvp.Context(0) as ctx:
        inc = make_incident(ctx)
        t0 = time.time()
        recs = []
        for i, T in enumerate(transducers(a.transducers, a.seed)):
            recs.append((T, BP.sweep(ctx, T, MED, inc, n_max=5)))
            if (i + 1) % 25 == 0:
                log("sweeps %d/%d (%.0f s)" % (i + 1, a.transducers, time.time() - t0))
        x, t = BP.dataset(recs, a.eps, a.guard)
        false_pass, n_pass = BP.guard_safety(recs, a.eps, a.guard)
        log("guard: %d ladder boxes pass, %.4f of them miss the target" % (n_pass, false_pass))
        t_sweep = time.time() - t0
        np.savez(os.path.join(a.out, "dataset.npz"), x=x, t=t,
                 fractions=np.stack([r["fractions"] for _, rs in recs for r in rs]),
                 err=np.stack([r["err"] for _, rs in recs for r in rs]),
                 delta=np.stack([r["delta"] for _, rs in recs for r in rs]))
        log("dataset %d sweeps in %.1f s; label means %s" % (x.shape[0], t_sweep, t.mean(axis=0)))
        if a.sweep_only:
            return
        mean, std = WL.input_norm()
        t1 = time.time()
        net, hist = BP.train(ctx, x, t, WL.boxnet_init(a.seed), mean, std, steps=a.steps, tau=a.tau, log=log)
        t_train = time.time() - t1
        BP.save_net(net, os.path.join(a.out, "boxnet_window"),
                    dict(window=BP.WINDOW, eps=a.eps, guard=a.guard, shrink=BP.GUARD_SHRINK, tau=a.tau,
                         steps=a.steps, sweeps=int(x.shape[0]), transducers=a.transducers, seed=a.seed,
                         norm_mean=mean.tolist(), norm_std=std.tolist(), final_loss=hist[-1][1]))
        y = net.predict(torch.from_numpy(x).cuda()).cpu().numpy()
        cover = float(np.mean(np.all(y >= t - 1e-6, axis=1)))
        log("trained in %.1f s; final loss %.5f; training samples fully covered %.3f" % (t_train, hist[-1][1], cover))
        rows, tot = BP.evaluate(ctx, transducers(a.eval, a.eval_seed), MED, inc, net=net, guard=a.guard, log=log)
        net.close()
    per_n = {}
    for r in rows:
        for n, e in r["net"]["err"].items():
            per_n.setdefault(n, []).append(e)
    summary = dict(sweeps=int(x.shape[0]), transducers=a.transducers, sweep_s=t_sweep, train_s=t_train,
                   guard_false_pass=false_pass, guard_passing_boxes=n_pass,
                   steps=a.steps, tau=a.tau, guard=a.guard, eps=a.eps, final_loss=hist[-1][1],
                   train_coverage=cover, eval=tot,
                   net_max_err_per_harmonic={str(n): max(v) for n, v in per_n.items()})
    with open(os.path.join(a.out, "summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1, default=float)
    log(json.dumps(summary, default=float))


if __name__ == "__main__":
    main()
