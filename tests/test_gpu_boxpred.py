"""The learned box predictor on the GPU: what it gains over the method without it.

Every error here is measured against the plain method on the full reference
window (the conservative box), at the focus, per harmonic.
"""

import sys

import numpy as np
import pytest

from workload import configs, learn as WL

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")
BP = pytest.importorskip("paper_2011_03009_amd.boxpred")
TB = pytest.importorskip("paper_2011_03009_amd.train_boxnet")

MED = configs.WATER


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.sync()
    c.close()


def test_stored_network_beats_full_box_within_target(ctx):
    """The network trained on 2000 sweeps, on 8 held-out transducers: at most 1% focal error on every
    harmonic (after the guard) and at least 1.5x fewer voxels than the full box.  (The rule of thumb's
    row is reported only: applied to the clipped window rather than to the paper's reference domain
    it is no fair baseline.)"""
    net, meta = BP.load_net(ctx)
    assert meta["sweeps"] >= 2000
    Ts = TB.transducers(8, 0)
    say("case stored boxnet on 8 held-out transducers")
    rows, tot = BP.evaluate(ctx, Ts, MED, TB.make_incident(ctx), net=net, log=say)
    net.close()
    say("totals", tot)
    assert tot["net"]["max_err"] <= 0.01
    assert tot["net"]["voxel_gain"] >= 1.5


def test_sweep_train_predict_end_to_end(ctx):
    """Sweeps of 30 transducers -> labels -> GPU training -> guarded prediction on 4 others."""
    inc = TB.make_incident(ctx, n_points=2048)
    say("case boxnet end-to-end: sweeps")
    recs = [(T, BP.sweep(ctx, T, MED, inc)) for T in TB.transducers(30, 7)]
    fp, n_pass = BP.guard_safety(recs)
    x, t = BP.dataset(recs)
    assert x.shape == (120, 5) and np.all((t >= 0) & (t <= 1))
    # the second harmonic needs (nearly) the whole window, the fifth a small part of it
    n = x[:, 4]
    assert t[n == 2].mean() > 0.8 and np.prod(t[n == 5], axis=1).mean() < 0.5
    mean, std = WL.input_norm()
    say("case boxnet end-to-end: training")
    net, hist = BP.train(ctx, x, t, WL.boxnet_init(0), mean, std, steps=1500)
    assert hist[-1][1] < 0.25 * hist[0][1]
    say("case boxnet end-to-end: evaluation")
    rows, tot = BP.evaluate(ctx, TB.transducers(4, 8), MED, inc, net=net, log=say)
    net.close()
    say("guard false-pass %.4f over %d boxes; totals %s" % (fp, n_pass, tot))
    assert tot["net"]["max_err"] <= 0.01
    assert tot["net"]["voxel_gain"] > 1.0
