"""ORACLE — test infrastructure only (see the package docstring).

The volume integral equation of an inhomogeneous medium (Section 7, the
equations of the harmonics in an inhomogeneous domain), discretised with the
midpoint-rule kernel of the volume potential (Section 3.1, equation "quad"):

    p_i - sum_j K_kb(x_i - x_j) q_j p_j = rhs_i,    q = k(x)^2 - kb^2,

written out as the dense matrix I - K diag(q) and solved directly (FP64).
Tiny grids only (the matrix has N^2 entries).

Pins (tests/test_oracle_pins.py): with no contrast the solution is the
right-hand side; as the contrast is scaled by eps -> 0 the solution follows
the Born series rhs + eps V[q rhs] + eps^2 V[q V[q rhs]] + ..., with V the
direct-sum volume potential (pinned to its own closed forms).
"""

import numpy as np

from .core import kernel_offsets
from .quadrature import corrected_weights


def dense_operator(k, h, n, rule="ball"):
    """The N x N matrix of sum_j K_k(x_i - x_j) f_j on a grid of n voxels (C order).

    rule "corrected": the kernel of oracle/quadrature.py (self value replaced,
    the face weight added at the offsets of length one)."""
    K = kernel_offsets(k, h, n)
    if rule == "corrected":
        w_self, w_face = corrected_weights(k, h)
        K[0, 0, 0] = w_self
        for off in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            if all(off[a] < n[a] for a in range(3)):
                K[off] += w_face
    elif rule != "ball":
        raise ValueError("rule must be 'ball' or 'corrected'")
    idx = np.indices(n).reshape(3, -1).T
    d = np.abs(idx[:, None, :] - idx[None, :, :])
    return K[d[..., 0], d[..., 1], d[..., 2]]


def vie_solve(q, rhs, h, kb, rule="ball"):
    """p with p - V_kb[q p] = rhs on the grid of q's shape (dense FP64 solve)."""
    n = q.shape
    A = np.eye(q.size, dtype=np.complex128) - dense_operator(kb, h, n, rule) * q.reshape(-1)[None, :]
    return np.linalg.solve(A, rhs.reshape(-1)).reshape(n)
