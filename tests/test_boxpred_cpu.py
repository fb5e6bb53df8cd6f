"""Host logic of the learned truncation boxes (CPU only)."""

import numpy as np

import paper_2011_03009_amd.boxpred as BP
from workload import configs

MED = configs.WATER


def _geos(count=12, seed=3):
    return [BP.Geometry(BP.Transducer(**d), MED) for d in configs.batch_transducers(count, seed)]


def test_window_grids_hold_the_focus_at_their_focal_index():
    for geo in _geos():
        for n in range(1, 6):
            g = geo.g1() if n == 1 else geo.grid(n, (0.4, 0.7, 0.2))
            pre, _, hy, hz = geo.half_counts(n, (1.0, 1.0, 1.0) if n == 1 else (0.4, 0.7, 0.2))
            if n == 1:
                pre, hy, hz = pre + 2, hy + 2, hz + 2
            for a, i in enumerate((pre, hy, hz)):
                assert abs(g.origin[a] + i * g.h - geo.focus[a]) < 1e-12
            # window limits: pre-focal length L, lateral half-width w, both within the bowl's domain
            assert geo.L <= np.sqrt(geo.T.l ** 2 - geo.T.R ** 2) and geo.w <= geo.T.R


def test_fractions_and_boxes_round_trip():
    rng = np.random.default_rng(0)
    for geo in _geos():
        for n in range(2, 6):
            N = [int(v) for v in geo.grid(n).n]
            for _ in range(40):
                lo = [int(rng.integers(0, N[a])) for a in range(3)]
                hi = [int(rng.integers(lo[a], N[a])) for a in range(3)]
                fr = geo.fractions_of(n, lo + hi)
                sb = geo.sub_box(n, fr, (1.0, 1.0, 1.0))
                assert all(0 <= sb[a] <= lo[a] and hi[a] <= sb[3 + a] < N[a] for a in range(3))
                # the box of a fraction triple is the grid of that triple placed in the window
                g = geo.grid(n, fr)
                assert [sb[3 + a] - sb[a] + 1 for a in range(3)] == [int(v) for v in g.n]


def test_label_takes_the_smallest_converged_guard_passing_box():
    fr = np.array([[0.125 * (i + 1)] * 3 for i in range(6)])
    rec = dict(fractions=fr, err=np.array([0.5, 0.02, 0.004, 0.011, 0.003, 0.001]),
               delta=np.array([0.3, 0.05, 0.002, 0.004, 0.001, 0.0]))
    # index 3 misses eps, so the label starts after it
    assert BP.label(rec, eps=0.01, delta_max=0.01) == (0.625,) * 3
    rec["err"][3] = 0.009
    assert BP.label(rec, eps=0.01, delta_max=0.01) == (0.375,) * 3
    rec["delta"][2] = 0.02
    assert BP.label(rec, eps=0.01, delta_max=0.01) == (0.5,) * 3
    rec["err"][-1] = 0.02
    assert BP.label(rec, eps=0.01, delta_max=0.01) == (1.0, 1.0, 1.0)
    recs = [(None, [rec])]
    fp, n_pass = BP.guard_safety(recs, eps=0.01, delta_max=0.01)
    assert n_pass == 3 and abs(fp - 1.0 / 3.0) < 1e-15


def test_rule_of_thumb_fractions():
    T = BP.Transducer(0.03, 0.1, 1e6, 1e6, 5)
    assert BP.rule_of_thumb_fractions(T) == {2: (1.0,) * 3, 3: (2 / 3,) * 3, 4: (0.5,) * 3, 5: (0.4,) * 3}
