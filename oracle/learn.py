"""ORACLE — test infrastructure only.

Plain FP64 CPU versions of the truncation-box tools and of the box-predictor
network, for the parity tests of the HIP library (which shares no code with
this module).

* qbox, box_potential: the localisation measure Q(x) = log10(|f| / max |f|) and
  the truncated integration domains of the paper's Section 5 convergence tests;
  the truncated potential is the midpoint sum of Section 3.1 restricted to a
  box (through the pinned direct sum of core.conv_direct).
* boxnet_*: a 5-64-64-64-3 tanh MLP with a pinball (quantile) loss and Adam.
  The paper has no learned component; these are the textbook definitions
  (quantile loss rho_tau(u) = u (tau - [u < 0]); Adam with bias-corrected
  moments), pinned by finite differences and closed-form special cases.
"""

import math

import numpy as np

from .core import conv_direct

# ---------------------------------------------------------------- truncation boxes (Section 5)


def qbox(f, q0):
    """Smallest voxel boxes outside which Q < q0, for each threshold: int64 [len(q0)][6] (lo xyz, hi xyz).

    A voxel is inside when |f|^2 >= 10^(2 q0) max |f|^2: the squares of the
    FP64 parts and their sum are formed as written (exact for complex64 input),
    10^(2 q0) by the C library's pow (math.pow), so the integer decision is the
    same one the library takes.
    """
    f = np.asarray(f)
    re = np.real(f).astype(np.float64)
    im = np.imag(f).astype(np.float64)
    m2 = re * re + im * im
    mx = m2.max()
    out = np.zeros((len(q0), 6), dtype=np.int64)
    for i, q in enumerate(q0):
        inside = m2 >= math.pow(10.0, 2.0 * float(q)) * mx
        idx = np.nonzero(inside)
        for a in range(3):
            out[i, a] = idx[a].min()
            out[i, 3 + a] = idx[a].max()
    return out


def box_potential(f, h, k, target, boxes):
    """-sum over voxels j of each box of K(x_t - x_j) f_j (eq. quad restricted to the box)."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape
    t = int(np.ravel_multi_index(tuple(int(v) for v in target), n))
    out = np.zeros(len(boxes), dtype=np.complex128)
    for i, b in enumerate(np.asarray(boxes, dtype=np.int64).reshape(-1, 6)):
        if np.any(b[3:] < b[:3]):
            continue
        g = np.zeros_like(f)
        sl = tuple(slice(int(b[a]), int(b[3 + a]) + 1) for a in range(3))
        g[sl] = f[sl]
        out[i] = -conv_direct(g, h, k, targets=np.array([t], dtype=np.int64))[0]
    return out


# ---------------------------------------------------------------- box-predictor MLP

BOXNET_SHAPES = ((64, 5), (64, 64), (64, 64), (3, 64))
BOXNET_PARAMS = sum(o * i + o for o, i in BOXNET_SHAPES)
ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def boxnet_unpack(params):
    """[(W, b)] per layer from the flat layout W1 b1 W2 b2 W3 b3 W4 b4 (W row-major [out][in])."""
    p = np.asarray(params, dtype=np.float64).reshape(-1)
    assert p.size == BOXNET_PARAMS
    layers, o = [], 0
    for (no, ni) in BOXNET_SHAPES:
        W = p[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = p[o:o + no]
        o += no
        layers.append((W, b))
    return layers


def boxnet_forward(params, mean, std, x):
    """y [B][3] and the activations (a0, h1, h2, h3) of the forward pass."""
    x = np.asarray(x, dtype=np.float64)
    a0 = (x - np.asarray(mean, dtype=np.float64)) / np.asarray(std, dtype=np.float64)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = boxnet_unpack(params)
    h1 = np.tanh(a0 @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    h3 = np.tanh(h2 @ W3.T + b3)
    y = h3 @ W4.T + b4
    return y, (a0, h1, h2, h3)


def pinball_loss(y, t, tau):
    """(1 / (3B)) sum of rho_tau(t - y) over samples and outputs."""
    u = np.asarray(t, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return float(np.sum(u * (tau - (u < 0.0))) / u.size)


def boxnet_grads(params, mean, std, x, t, tau):
    """(dL/dparams in the flat layout, L) by back-propagation."""
    y, (a0, h1, h2, h3) = boxnet_forward(params, mean, std, x)
    (W1, _), (W2, _), (W3, _), (W4, _) = boxnet_unpack(params)
    u = np.asarray(t, dtype=np.float64) - y
    d4 = -(tau - (u < 0.0)) / u.size
    d3 = (d4 @ W4) * (1.0 - h3 * h3)
    d2 = (d3 @ W3) * (1.0 - h2 * h2)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)
    parts = []
    for d, a in ((d1, a0), (d2, h1), (d3, h2), (d4, h3)):
        parts.append((d.T @ a).reshape(-1))
        parts.append(d.sum(axis=0))
    return np.concatenate(parts), pinball_loss(y, t, tau)


def adam_step(params, grad, m, v, step, lr, b1=ADAM_BETA1, b2=ADAM_BETA2, eps=ADAM_EPS):
    """One Adam update (step counts from 1): returns new (params, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
