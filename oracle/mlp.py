"""Plain FP64 oracle of the learned closure network (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module; it shares no code with the GPU library.

The closure of the fluid model (section IV: the electron flux and energy flux
of eqs. (12)-(13), here predicted instead of taken from drift-diffusion
coefficients) is a multilayer perceptron with 5 inputs, three hidden layers
of 64 tanh units and 2 linear outputs: 8,834 parameters.  Loss: mean squared
error over samples and outputs.  Optimiser: Adam (Kingma and Ba, 2015).

Parameter vector layout (float, row-major, W[i, j] maps input i to output j):
    W1 (5 x 64), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 64), b3 (64),
    W4 (64 x 2), b4 (2)

The GPU computes in BF16 with FP32 accumulation.  With emulate=True the
oracle rounds to BF16 at exactly the points where the GPU does (inputs,
weights, hidden activations after tanh, back-propagated pre-activation
gradients; biases, accumulations and outputs stay unrounded); the rounding
goes through FP32 first, as the GPU's values are FP32 before they are
narrowed.  With emulate=False everything is FP64 (the reference for finite
differences).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 5, 64, 2
SHAPES = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,),
          (N_HID, N_OUT), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)   # 8834


def bf16(x):
    """Round to the nearest BF16 value, ties to even, via FP32 (finite inputs)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    """Split a flat parameter vector into [W1, b1, W2, b2, W3, b3, W4, b4]."""
    t = np.asarray(theta, dtype=np.float64)
    if t.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(t[o:o + k].reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed: int = 0):
    """Glorot-uniform weights, zero biases (seeded; the GPU trains from the
    same vector)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts).astype(np.float32).astype(np.float64)


def forward(theta, x, emulate: bool = True):
    """Returns (y, [a0, a1, a2, a3]): outputs and the layer inputs (a0 = the
    input, a1..a3 the hidden activations), as the backward pass uses them."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    a = [r(x)]
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z = a[-1] @ r(W) + b
        a.append(r(np.tanh(z)))
    y = a[-1] @ r(W4) + b4
    return y, a


def loss(theta, x, t, emulate: bool = False):
    y, _ = forward(theta, x, emulate)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(theta, x, t, emulate: bool = True, hidden=None):
    """Gradient of the mean squared error with respect to theta (flat), and the loss.

    hidden (optional): the three hidden activations [a1, a2, a3] to use in
    place of the oracle's own forward pass (the layer inputs a parity check
    shares with the GPU); the output layer and the whole backward pass are
    then computed here from them."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    if hidden is None:
        y, a = forward(theta, x, emulate)
    else:
        a = [r(x)] + [np.asarray(h, dtype=np.float64) for h in hidden]
        y = a[3] @ r(W4) + b4
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    dz = r(2.0 * (y - t) / (n * N_OUT))          # d loss / d output pre-activation
    grads = []
    Ws = [W1, W2, W3, W4]
    for layer in (3, 2, 1, 0):
        grads.append((a[layer].T @ dz, dz.sum(axis=0)))
        if layer == 0:
            break
        da = dz @ r(Ws[layer]).T                 # d loss / d activation of the layer below
        dz = r(da * (1.0 - a[layer] ** 2))       # tanh' = 1 - tanh^2 at the stored activation
    gW4, gb4 = grads[0]
    gW3, gb3 = grads[1]
    gW2, gb2 = grads[2]
    gW1, gb1 = grads[3]
    return pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4]), float(np.mean((y - t) ** 2))


def adam(theta, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
