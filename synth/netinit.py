"""Seeded initial parameters of the filter-weight network.

A random draw only (none of the method's arithmetic): weight matrices of the
hidden layers from N(0, 2/fan_in) (He initialisation), biases zero, and the
output layer zero so that the untrained network adds nothing to the Fourier
weights.  Layout: W1 (64 x 128), b1, W2 (128 x 128), b2, W3 (128 x 128), b3,
W4 (128 x 512), b4, each row-major, concatenated.
"""

from __future__ import annotations

import math

import numpy as np

N_IN, HIDDEN, N_OUT = 64, 128, 512


def layer_shapes(n_in: int = N_IN, hidden: int = HIDDEN, n_out: int = N_OUT):
    return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out),
            (n_out,)]


def init_params(seed: int, shapes=None) -> np.ndarray:
    shapes = layer_shapes() if shapes is None else shapes
    n_out = shapes[-1][0]
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes:
        if len(s) == 1 or s[1] == n_out:
            parts.append(np.zeros(s))
        else:
            parts.append(rng.standard_normal(s) * math.sqrt(2.0 / s[0]))
    return np.concatenate([p.ravel() for p in parts])
