"""Pins of the oracle's truncation-box tools and box-predictor network (CPU only)."""

import math

import numpy as np

import oracle
import oracle.learn as OL
from workload import fields, learn as WL


# ---------------------------------------------------------------- localisation boxes

def test_qbox_of_gaussian_matches_closed_form():
    """|f| = exp(-r^2 / 2s^2) about a voxel: Q >= Q0 iff r^2 <= -2 s^2 Q0 ln 10, so the half-width is known."""
    n = (41, 33, 29)
    c = (17, 15, 12)
    s = (4.3, 2.9, 3.7)
    ax = [np.arange(m, dtype=np.float64) for m in n]
    r2 = sum(((a - c[i]) / s[i]) ** 2 for i, a in enumerate(np.meshgrid(*ax, indexing="ij")))
    f = (np.exp(-0.5 * r2) * np.exp(0.3j)).astype(np.complex128)
    q0 = [-0.37, -1.13, -2.71]
    got = OL.qbox(f, q0)
    for i, q in enumerate(q0):
        for a in range(3):
            half = math.floor(s[a] * math.sqrt(-2.0 * q * math.log(10.0)))
            assert got[i, a] == max(c[a] - half, 0)
            assert got[i, 3 + a] == min(c[a] + half, n[a] - 1)


def test_qbox_matches_log10_definition_by_brute_force():
    f = fields.smooth_field((13, 11, 9), seed=3) + 1e-3 * fields.random_field((13, 11, 9), seed=4)
    Q = np.log10(np.abs(f) / np.abs(f).max())
    q0 = [-0.2, -0.5, -1.0, -2.0, 0.0]
    got = OL.qbox(f, q0)
    for i, q in enumerate(q0):
        if np.min(np.abs(Q - q)) < 1e-9:
            continue  # a tie at the threshold: the squared comparison decides it
        pts = [(x, y, z) for x in range(13) for y in range(11) for z in range(9) if Q[x, y, z] >= q]
        ref = [min(p[a] for p in pts) for a in range(3)] + [max(p[a] for p in pts) for a in range(3)]
        assert list(got[i]) == ref
    # Q0 = 0 keeps the maximum only
    i = int(np.argmax(np.abs(f)))
    m = np.unravel_index(i, f.shape)
    assert list(got[4]) == [m[0], m[1], m[2], m[0], m[1], m[2]]


# ---------------------------------------------------------------- truncated potentials

def test_box_potential_full_box_is_volume_potential_and_partitions_add():
    n = (9, 8, 7)
    f = fields.random_field(n, seed=11)
    h, k = 1.0e-4, complex(9000.0, 3.0)
    t = (4, 3, 5)
    full = OL.box_potential(f, h, k, t, [[0, 0, 0, 8, 7, 6]])[0]
    ref = oracle.volume_potential(f, h, k)[t]
    assert abs(full - ref) <= 1e-13 * abs(ref)
    # the potential is additive over a partition of the grid into boxes
    parts = [[0, 0, 0, 3, 7, 6], [4, 0, 0, 8, 2, 6], [4, 3, 0, 8, 7, 3], [4, 3, 4, 8, 7, 6]]
    tot = OL.box_potential(f, h, k, t, parts).sum()
    assert abs(tot - full) <= 1e-13 * abs(full)
    # an empty box contributes nothing
    assert OL.box_potential(f, h, k, t, [[3, 0, 0, 2, 7, 6]])[0] == 0


# ---------------------------------------------------------------- network

def _net(seed=0, B=7):
    p = WL.boxnet_init(seed).astype(np.float64)
    p += 0.05 * np.random.default_rng(seed + 1).standard_normal(p.size)  # non-zero biases
    mean, std = WL.input_norm()
    x, t = WL.boxnet_batch(B, seed + 2)
    return p, mean.astype(np.float64), std.astype(np.float64), x.astype(np.float64), t.astype(np.float64)


def test_boxnet_layout_and_forward_by_hand():
    p, mean, std, x, _ = _net()
    assert p.size == OL.BOXNET_PARAMS == WL.N_PARAMS == 8899
    y, _ = OL.boxnet_forward(p, mean, std, x)
    # the same network written out sample by sample with explicit index loops
    o = 0
    layers = []
    for (no, ni) in WL.SHAPES:
        W = [[p[o + i * ni + j] for j in range(ni)] for i in range(no)]
        o += no * ni
        b = [p[o + i] for i in range(no)]
        o += no
        layers.append((W, b))
    for s in range(x.shape[0]):
        a = [(x[s, j] - mean[j]) / std[j] for j in range(5)]
        for li, (W, b) in enumerate(layers):
            z = [b[i] + sum(W[i][j] * a[j] for j in range(len(a))) for i in range(len(b))]
            a = z if li == 3 else [math.tanh(v) for v in z]
        assert np.allclose(a, y[s], rtol=1e-13, atol=1e-13)


def test_boxnet_gradients_match_finite_differences():
    p, mean, std, x, t = _net(seed=5, B=6)
    y, _ = OL.boxnet_forward(p, mean, std, x)
    t = y + np.where(np.arange(y.size).reshape(y.shape) % 2 == 0, 0.3, -0.4)  # far from the loss kink
    tau = 0.8
    g, L = OL.boxnet_grads(p, mean, std, x, t, tau)
    assert abs(L - OL.pinball_loss(y, t, tau)) < 1e-15
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(8899, 60, replace=False), [0, 319, 320, 383, 384, 8895, 8896, 8898]])
    eps = 1e-6
    for q in idx:
        pp = p.copy()
        pp[q] += eps
        pm = p.copy()
        pm[q] -= eps
        fd = (OL.pinball_loss(OL.boxnet_forward(pp, mean, std, x)[0], t, tau) -
              OL.pinball_loss(OL.boxnet_forward(pm, mean, std, x)[0], t, tau)) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-7 * max(1e-3, abs(g).max())


def test_pinball_loss_special_cases():
    rng = np.random.default_rng(1)
    y, t = rng.standard_normal((5, 3)), rng.standard_normal((5, 3))
    # tau = 1/2: half the mean absolute error
    assert abs(OL.pinball_loss(y, t, 0.5) - 0.5 * np.mean(np.abs(t - y))) < 1e-15
    # all targets above the predictions: tau times the mean gap
    assert abs(OL.pinball_loss(t - 5.0, t, 0.9) - 0.9 * 5.0) < 1e-12


def test_adam_first_step_closed_form():
    """With zero moments, the bias-corrected first step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p, g = rng.standard_normal(50), rng.standard_normal(50)
    z = np.zeros(50)
    p1, m, v = OL.adam_step(p, g, z, z, 1, 1e-2)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
