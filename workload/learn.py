"""Seeded inputs of the box predictor: initial network weights and stand-in batches.

These are random draws only (no arithmetic of the method): the initial
weights are passed to the library and to the oracle alike.
"""

import numpy as np

SHAPES = ((64, 5), (64, 64), (64, 64), (3, 64))
N_PARAMS = sum(o * i + o for o, i in SHAPES)


def boxnet_init(seed):
    """Flat float32 parameters W1 b1 ... W4 b4: Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for (no, ni) in SHAPES:
        a = np.sqrt(6.0 / (ni + no))
        parts.append(rng.uniform(-a, a, size=no * ni))
        parts.append(np.zeros(no))
    return np.concatenate(parts).astype(np.float32)


def boxnet_batch(B, seed):
    """Stand-in inputs (aperture m, focal length m, frequency Hz, pressure Pa, harmonic) and targets in [0, 1]."""
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(0.02, 0.08, B), rng.uniform(0.04, 0.16, B), rng.uniform(0.5e6, 1.5e6, B),
                  rng.uniform(0.2e6, 1.5e6, B), rng.integers(2, 6, B).astype(np.float64)], axis=1)
    t = rng.uniform(0.0, 1.0, (B, 3))
    return x.astype(np.float32), t.astype(np.float32)


def input_norm():
    """Fixed input standardisation of the predictor: the centres and half-ranges of the sampled ranges."""
    mean = np.array([0.05, 0.10, 1.0e6, 0.85e6, 3.5], dtype=np.float32)
    std = np.array([0.03, 0.06, 0.5e6, 0.65e6, 1.5], dtype=np.float32)
    return mean, std
