"""Pins of the closure-network oracle (oracle/mlp.py) against things other
than itself: central finite differences of the FP64 loss, torch's own
bfloat16 conversion, closed forms of tiny networks and of one Adam step."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 8834
    th = mlp.init_params(1)
    assert th.size == 8834
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.01171875, 3.0e38, -2.5e-38]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(mlp.bf16(x32), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    th = mlp.init_params(3) + rng.normal(0.0, 0.05, mlp.N_PARAMS)
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=(9, 2))
    g, _ = mlp.backward(th, x, t, emulate=False)
    h = 1e-6
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 120, replace=False),
                          [0, 319, 320, 383, 384, 8831, 8832, 8833]])
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(th + e, x, t) - mlp.loss(th - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_closed_form_zero_weights_and_single_path():
    # zero weights: every hidden unit is tanh(bias) and the output is
    # W4^T tanh(b3) + b4
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.zeros(s) for s in mlp.SHAPES]
    b3[:] = 0.5
    W4[:, 0] = 1.0 / 64
    b4[1] = -2.0
    th = mlp.pack([W1, b1, W2, b2, W3, b3, W4, b4])
    y, _ = mlp.forward(th, np.ones((3, 5)), emulate=False)
    assert np.allclose(y[:, 0], np.tanh(0.5), rtol=0, atol=1e-15)
    assert np.all(y[:, 1] == -2.0)
    # one path: input 0 -> unit 0 -> unit 0 -> unit 0 -> output 1
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.zeros(s) for s in mlp.SHAPES]
    W1[0, 0] = 0.7
    W2[0, 0] = 1.3
    W3[0, 0] = -0.4
    W4[0, 1] = 2.0
    th = mlp.pack([W1, b1, W2, b2, W3, b3, W4, b4])
    x = np.array([[0.9, 5, 5, 5, 5]])
    y, _ = mlp.forward(th, x, emulate=False)
    expect = 2.0 * np.tanh(-0.4 * np.tanh(1.3 * np.tanh(0.7 * 0.9)))
    assert y[0, 0] == 0.0 and abs(y[0, 1] - expect) < 1e-15


def test_emulation_changes_only_at_bf16_level():
    rng = np.random.default_rng(2)
    th = mlp.init_params(5)
    x = rng.normal(size=(64, 5))
    y64, _ = mlp.forward(th, x, emulate=False)
    y16, a = mlp.forward(th, x, emulate=True)
    for act in a:
        assert np.array_equal(act, mlp.bf16(act))          # stored activations are BF16 values
    assert np.abs(y16 - y64).max() < 0.05 * np.abs(y64).max()
    assert np.abs(y16 - y64).max() > 0.0


def test_adam_first_step_closed_form():
    # from m = v = 0 the bias-corrected first step is -lr g / (|g| + eps)
    g = np.array([3.0, -0.25, 1e-3, 0.0])
    th, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps the step at -lr sign(g) (up to eps) for every step
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for k in range(1, 6):
        th, m, v = mlp.adam(th, m, v, g, k, lr=0.01)
    assert np.allclose(th[:3], -0.05 * np.sign(g[:3]), rtol=2e-5)   # eps/|g| <= 1e-5


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, size=(256, 5))
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2 - x[:, 3] * x[:, 4]], axis=1)
    th = mlp.init_params(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, x, t)
    for k in range(1, 201):
        g, _ = mlp.backward(th, x, t, emulate=True)
        th, m, v = mlp.adam(th, m, v, g, k, lr=3e-3)
    assert mlp.loss(th, x, t) < 0.2 * l0
