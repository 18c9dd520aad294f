"""Seeded inputs of the surrogate network: initial weights and the scaled
feature vector of a (device parameters, circuit angles) sample.

Only random draws and fixed rescaling happen here; the network's arithmetic
(forward, gradients, optimiser) lives with each consumer.

Parameter vector of one member, flattened in this order (row-major weights,
``W[out][in]``, so that ``z_o = sum_i W[o][i] a_i + b_o``)::

    W1 (256 x 24), b1 (256), W2 (256 x 256), b2 (256),
    W3 (256 x 256), b3 (256), W4 (10 x 256), b4 (10)       -> 140554 values
"""
from __future__ import annotations

import math

import numpy as np

from .circuits import SEED_BASE

LAYERS = (24, 256, 256, 256, 10)
N_MEMBERS = 4


def n_params(layers=LAYERS) -> int:
    return sum(o * i + o for i, o in zip(layers[:-1], layers[1:]))


def init_member(seed: int, layers=LAYERS) -> np.ndarray:
    """One member's initial parameters: weights and biases ~ U(-1/sqrt(fan_in),
    +1/sqrt(fan_in)) (the usual default for dense layers), float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(layers[:-1], layers[1:]):
        a = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-a, a, o * i))
        parts.append(rng.uniform(-a, a, o))
    return np.concatenate(parts).astype(np.float32)


def init_ensemble(seed: int = SEED_BASE + 5, members: int = N_MEMBERS, layers=LAYERS) -> np.ndarray:
    """``[members, n_params]`` float32, member m drawn with seed + m."""
    return np.stack([init_member(seed + m, layers) for m in range(members)])


# ranges of the 8 device parameters (see c5_draw_samples); p1, p2 are drawn
# log-uniformly and scaled on the log axis
_DEV_LO = np.array([20.0, 10.0, math.log(1e-4), math.log(1e-4), 0.02, 0.2, 0.0, 0.0])
_DEV_HI = np.array([200.0, 200.0, math.log(1e-2), math.log(1e-2), 0.1, 0.8, 0.02, 0.1])


def c5_features(dev: np.ndarray, angles: np.ndarray) -> np.ndarray:
    """``[count, 24]`` float32 network inputs in [0, 1]: device parameters
    scaled by their drawing ranges (T2 by [10, 200] us, the error rates on the
    log axis), then the 16 angles divided by 2 pi."""
    dev = np.atleast_2d(np.asarray(dev, dtype=np.float64)).copy()
    dev[:, 2:4] = np.log(dev[:, 2:4])
    d = (dev - _DEV_LO) / (_DEV_HI - _DEV_LO)
    a = np.atleast_2d(angles) / (2 * math.pi)
    return np.concatenate([d, a], axis=1).astype(np.float32)
