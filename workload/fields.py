"""Seeded synthetic complex fields used as sources and as stand-in harmonics."""

import numpy as np


def random_field(shape, seed, dtype=np.complex128):
    """Independent standard-normal real and imaginary parts (the harshest case for FFT parity)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return a.astype(dtype)


def smooth_field(shape, seed, n_blobs=4, dtype=np.complex128):
    """Sum of a few complex Gaussian blobs with seeded centres, widths and phases.

    Coordinates are voxel indices; widths are 8-30% of each extent, so the
    field is smooth on the grid and varies over several voxels.
    """
    rng = np.random.default_rng(seed)
    idx = [np.arange(n, dtype=np.float64) for n in shape]
    out = np.zeros(shape, dtype=np.complex128)
    for _ in range(n_blobs):
        acc = np.ones(shape, dtype=np.float64)
        for ax, n in enumerate(shape):
            c = rng.uniform(0.2, 0.8) * (n - 1)
            w = rng.uniform(0.08, 0.3) * max(n, 1)
            g = np.exp(-0.5 * ((idx[ax] - c) / w) ** 2)
            sh = [1] * len(shape)
            sh[ax] = n
            acc = acc * g.reshape(sh)
        amp = rng.uniform(0.5, 2.0) * np.exp(1j * rng.uniform(0, 2 * np.pi))
        out += amp * acc
    return out.astype(dtype)
