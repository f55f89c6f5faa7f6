"""Closure network kernels (BF16 matrix cores) against the FP64 oracle.

Forward: each layer is checked from the GPU's own previous-layer activations
(shared inputs), so differences come only from FP32 accumulation (the
oracle sums in FP64): hidden activations equal the oracle's BF16 rounding
except where the two pre-activations round differently, and then differ by
at most the accumulation bound, the GPU tanh error (6.6e-7) and half an ulp
on each side (rare);
outputs within 4e-6 x sum |a w| (64-term FP32 accumulation bound
64 * 2^-24 ~ 3.8e-6).
Gradient: every element within its FP32-accumulation and BF16-flip bound of
the oracle's emulated backward taken from the GPU's own hidden activations
(test_gradient_elementwise_parity, bound derived there); end to end (each
side with its own forward) norm-wise within 5e-3, bitwise repeatable.
Adam: one step within a few FP32 ulp of the parameter and of the step.
"""
import numpy as np
import pytest

from oracle import mlp as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _net(theta):
    from paper_2202_03215_amd.mlp import ClosureNet
    return ClosureNet(theta, max_batch=1 << 14)


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = O.init_params(seed)
    W1, b1, W2, b2, W3, b3, W4, b4 = O.unpack(th)
    parts = [W1 * 1.5, rng.normal(0, 0.2, 64), W2, rng.normal(0, 0.2, 64), W3, rng.normal(0, 0.2, 64),
             W4 * 3.0, rng.normal(0, 0.5, 2)]
    return O.pack(parts).astype(np.float32).astype(np.float64)


def _ulp(v):
    """BF16 unit in the last place of |v| (v a BF16 value; 2^-133 at zero)."""
    e = np.frexp(np.abs(v))[1] - 1
    return np.where(v == 0, 2.0 ** -133, np.ldexp(1.0, np.maximum(e, -126) - 7))


def _check_layer(g, o, S):
    """GPU activation g = bf16(tanh_gpu(z_gpu)), oracle o = bf16(tanh(z)),
    with |z_gpu - z| <= 4e-6 S (FP32 accumulation of 64 terms) and the GPU's
    tanh, 1 - 2 r with r = 1/(1 + 2^(2 z log2 e)) on the hardware exp2 and
    reciprocal (one ulp each) and one fused multiply-add, within
    2 r (2^-23 + 2^-24 + 2^-23) + 2^-24 <= 6.6e-7 absolute:
    |g - o| <= 4e-6 S + 6.6e-7 + ulp(g)/2 + ulp(o)/2.  Returns the number of
    elements that differ."""
    d = g != o
    if d.any():
        lim = 4e-6 * S[d] + 6.6e-7 + 0.5 * (_ulp(g[d]) + _ulp(o[d]))
        assert np.all(np.abs(g[d] - o[d]) <= lim), np.max(np.abs(g[d] - o[d]) / lim)
    return int(d.sum())


@pytest.mark.parametrize("n", [1, 17, 1000, 4099, 1 << 20])   # 1 << 20: the fluid bench's 256 x 4096 faces
def test_forward_layerwise_parity(torch_cuda, n):
    from paper_2202_03215_amd.mlp import bf16_bits_to_float
    torch = torch_cuda
    th = _theta(n)
    rng = np.random.default_rng(100 + n)
    x = rng.normal(0.0, 1.0, size=(n, 5)).astype(np.float32)
    net = _net(th)
    y, h = net.forward(torch.from_numpy(x), hidden=True)
    y = y.cpu().numpy().astype(np.float64)
    hs = [bf16_bits_to_float(h[k]) for k in range(3)]
    W1, b1, W2, b2, W3, b3, W4, b4 = O.unpack(th)
    prev = O.bf16(x.astype(np.float64))
    flips = 0
    for k, (W, b) in enumerate(((W1, b1), (W2, b2), (W3, b3))):
        ref = O.bf16(np.tanh(prev @ O.bf16(W) + b))
        S = np.abs(prev) @ np.abs(O.bf16(W)) + np.abs(b)
        flips += _check_layer(hs[k], ref, S)
        prev = hs[k]                                # next layer from the GPU's activations
    assert flips <= max(2, 1e-3 * 3 * 64 * n), flips
    yo = prev @ O.bf16(W4) + b4
    bound = 4e-6 * (np.abs(prev) @ np.abs(O.bf16(W4)) + np.abs(b4)) + 1e-30
    assert np.all(np.abs(y - yo) <= bound), np.abs(y - yo).max()
    # end to end against the oracle's own emulated forward
    ye, _ = O.forward(th, x.astype(np.float64), emulate=True)
    assert np.abs(y - ye).max() <= 2e-2 * max(1.0, np.abs(ye).max())


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 1.5, size=(n, 5))
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1] + 0.3 * x[:, 4], x[:, 2] ** 2 - x[:, 3] * x[:, 4]], axis=1)
    return x.astype(np.float32), t.astype(np.float32)


def _abs_scales(th, x, hidden, t, y):
    """Magnitude scale of every gradient element: the backward pass with the
    absolute value of every factor (|dz| through |W| and 1 - a^2 >= 0), so
    that S = sum over samples of |a| |dz| bounds the sum of the absolute
    terms each gradient element adds up, at every level."""
    W1, b1, W2, b2, W3, b3, W4, b4 = O.unpack(th)
    n = x.shape[0]
    a = [O.bf16(x)] + list(hidden)
    D = np.abs(2.0 * (y - t) / (n * 2))
    Ws = [W1, W2, W3, W4]
    out = []
    for layer in (3, 2, 1, 0):
        out.append((np.abs(a[layer]).T @ D, D.sum(axis=0)))
        if layer == 0:
            break
        D = (D @ np.abs(O.bf16(Ws[layer])).T) * (1.0 - a[layer] ** 2)
    (sW4, sb4), (sW3, sb3), (sW2, sb2), (sW1, sb1) = out
    return O.pack([sW1, sb1, sW2, sb2, sW3, sb3, sW4, sb4])


@pytest.mark.parametrize("n", [5, 33, 3000, 16384])
def test_gradient_elementwise_parity(torch_cuda, n):
    """Every gradient element against the oracle's emulated backward pass
    taken from the GPU's own hidden activations (the shared layer inputs).
    What is left to differ: FP32 accumulation (the output layer over 64
    terms, the back-propagated sums over 64, each weight gradient over n
    samples: at most (n + 192) 2^-24 S for the element's absolute scale S),
    and the rounding of a back-propagated gradient to BF16 when the GPU's
    FP32 value and the oracle's FP64 value fall on the two sides of a
    rounding point: one BF16 ulp (at most 2^-7 of its magnitude) on that
    term, at any of the four levels (output and three hidden layers), so
    at most 4 2^-7 S in all.  Bound: |dg| <= (4 2^-7 + (n + 192) 2^-24) S.
    Such flips need the two values within the FP32 accumulation error of a
    rounding point, so they are rare: at least 99 % of the elements must
    also lie within (n + 192) 2^-24 S + 2^-9 |g|."""
    from paper_2202_03215_amd.mlp import bf16_bits_to_float
    torch = torch_cuda
    th = _theta(11 + n)
    x, t = _data(n, 100 + n)
    net = _net(th)
    y, h = net.forward(torch.from_numpy(x), hidden=True)
    hidden = [bf16_bits_to_float(h[k]) for k in range(3)]
    g, _ = net.grad_loss(torch.from_numpy(x), torch.from_numpy(t))
    g = g.cpu().numpy().astype(np.float64)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    go, _ = O.backward(th, x64, t64, emulate=True, hidden=hidden)
    W4, b4 = O.unpack(th)[6:8]
    yo = hidden[2] @ O.bf16(W4) + b4
    S = _abs_scales(th, x64, hidden, t64, yo)
    d = np.abs(g - go)
    acc = (n + 192) * 2.0 ** -24
    bound = (4 * 2.0 ** -7 + acc) * S + 1e-30
    ratio = d / np.maximum(S, 1e-300)
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    o = 0
    for name, blk in zip(names, O.unpack(ratio)):
        print(f"n={n} {name}: max |dg|/S {blk.max():.3e}, 99.9% {np.quantile(blk, 0.999):.3e}")
        o += blk.size
    assert np.all(d <= bound), float((d / bound).max())
    tight = d <= acc * S + 2.0 ** -9 * np.abs(go) + 1e-30
    assert tight.mean() >= 0.99, tight.mean()


@pytest.mark.parametrize("n", [5, 33, 3000])
def test_gradient_parity_and_determinism(torch_cuda, n):
    torch = torch_cuda
    th = _theta(7 + n)
    x, t = _data(n, n)
    net = _net(th)
    g1, l1 = net.grad_loss(torch.from_numpy(x), torch.from_numpy(t))
    g1 = g1.cpu().numpy().astype(np.float64)
    l1 = float(l1.cpu().numpy()[0])
    g2, l2 = net.grad_loss(torch.from_numpy(x), torch.from_numpy(t))
    assert np.array_equal(g1, g2.cpu().numpy().astype(np.float64))    # fixed-order reductions
    go, lo = O.backward(th, x.astype(np.float64), t.astype(np.float64), emulate=True)
    assert abs(l1 - lo) <= 1e-4 * lo
    err = np.linalg.norm(g1 - go) / np.linalg.norm(go)
    assert err <= 5e-3, err
    # every parameter block carries gradient (layout of the flat vector)
    parts = O.unpack(g1)
    for p, q in zip(parts, O.unpack(go)):
        assert np.linalg.norm(p - q) <= 2e-2 * np.linalg.norm(q) + 1e-12


def test_adam_step_parity(torch_cuda):
    torch = torch_cuda
    th = _theta(3)
    x, t = _data(512, 1)
    net = _net(th)
    net.grad_loss(torch.from_numpy(x), torch.from_numpy(t))
    g = net.grad.cpu().numpy().astype(np.float64)
    net.adam(lr=1e-3)
    got = net.params()
    ref, m, v = O.adam(th, np.zeros_like(th), np.zeros_like(th), g, 1, lr=1e-3)
    # FP32: the step lr m/(sqrt(v) + eps) to a few ulp of lr, the subtraction to half an ulp of theta
    assert np.all(np.abs(got - ref) <= 2.0 ** -24 * (4 * np.abs(ref) + 8 * 1e-3))
    assert np.allclose(net.m.cpu().numpy(), m, rtol=1e-6, atol=1e-30)


def test_training_on_gpu_reduces_loss(torch_cuda):
    torch = torch_cuda
    x, t = _data(8192, 2)
    net = _net(O.init_params(0))
    losses = net.train(torch.from_numpy(x), torch.from_numpy(t), steps=400, lr=3e-3, batch=2048)
    assert losses[-20:].mean() < 0.1 * losses[:5].mean(), (losses[:5], losses[-20:])
    # the trained network generalises to fresh samples of the same target
    xv, tv = _data(2048, 9)
    yv = net.forward(torch.from_numpy(xv)).cpu().numpy()
    assert np.mean((yv - tv) ** 2) < 0.15 * np.mean((tv - tv.mean(0)) ** 2)
