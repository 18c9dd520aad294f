"""FP64 reference of the surrogate MLP ensemble -- TEST INFRASTRUCTURE.

The surrogate is not in the paper; the network and its number formats are
those of the learned-surrogate extension of the emulator (an ensemble of MLPs
mapping 8 device parameters and 16 circuit angles of the paper's
hardware-efficient ansatz to the 10 read-outs <Z_i>).

Network of one member: 24 -> 256 -> 256 -> 256 -> 10, GELU after each hidden
layer, linear output; loss = mean squared error over the batch and the 10
outputs.  Parameter layout: row-major ``W[out][in]`` then ``b`` per layer, in
layer order (140554 values).

Mixed precision (``mixed=True``): the operands of every matrix product are
rounded to bfloat16 (round to nearest, ties to even) and the products are
exact here (FP64) -- the GPU accumulates them in FP32.  Rounded are: the
input, every weight matrix, every hidden activation after GELU, and every
back-propagated pre-activation gradient (which then feeds the weight, bias
and input gradients alike).  Biases, pre-activations, the loss and the
optimiser state stay at full precision.  ``mixed=False`` is plain FP64.

Pins (tests/test_mlp_oracle.py): bf16 rounding against hand-computed values
and an independent bit-level rounding of float32; GELU against x * Phi(x)
from the normal CDF; gradients against central finite differences; Adam
against its closed form under a constant gradient; the weight layout against
a one-hot network; the spread against numpy's population std.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = (24, 256, 256, 256, 10)


def bf16(x):
    """Nearest bfloat16 value (8 significant bits, ties to even), as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                        # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def gelu(z):
    """GELU(z) = z * Phi(z) = z/2 * (1 + erf(z / sqrt 2))."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d GELU / dz = Phi(z) + z * phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(theta, layers=LAYERS):
    """Flat parameter vector -> [(W, b), ...] (views, float64)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for i, o in zip(layers[:-1], layers[1:]):
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    assert off == theta.size, (off, theta.size)
    return out


def pack(parts):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in parts])


def forward(theta, X, mixed=True, layers=LAYERS):
    """Outputs [B, 10] and the cache for backward."""
    r = bf16 if mixed else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(theta, layers)
    A = [r(X)]
    Z = []
    for li, (W, b) in enumerate(layers):
        z = A[-1] @ r(W).T + b
        Z.append(z)
        if li + 1 < len(layers):
            A.append(r(gelu(z)))
    return Z[-1], (A, Z, layers, r)


def loss_and_grad(theta, X, Y, mixed=True, layers=LAYERS):
    """MSE loss and its gradient with respect to the flat parameters."""
    out, (A, Z, layers, r) = forward(theta, X, mixed, layers)
    B = X.shape[0]
    diff = out - Y
    loss = float(np.mean(diff * diff))
    G = 2.0 * diff / diff.size
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        D = r(G)
        grads[li] = (D.T @ A[li], D.sum(axis=0))
        if li > 0:
            G = (D @ r(W)) * gelu_grad(Z[li - 1])
    assert B == Y.shape[0]
    return loss, pack(grads)


def adam(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1) with bias correction; returns new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def ensemble(thetas, X, mixed=True, layers=LAYERS):
    """Mean over members [B, 10] and spread [B]: the largest, over the 10
    outputs, population standard deviation across members."""
    P = np.stack([forward(t, X, mixed, layers)[0] for t in thetas])
    mean = P.mean(axis=0)
    spread = np.sqrt(((P - mean) ** 2).mean(axis=0)).max(axis=1)
    return mean, spread, P

