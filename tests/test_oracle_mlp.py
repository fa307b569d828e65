"""Pins for the surrogate-network oracle: bfloat16 rounding against hand
cases and torch's own conversion, GELU against the normal CDF's textbook
values and its odd-part identity, the analytic backward against central
finite differences, Adam against its closed form under a constant gradient,
and the hull test and features on hand cases."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_2101_06318_amd import workloads


def test_param_count():
    assert mlp.N_PARAMS == 34179
    assert mlp.OFFSETS[0] == (0, 640, 768)
    assert mlp.OFFSETS[3][2] == mlp.N_PARAMS


def test_bf16_round_hand_cases():
    one = np.float32(1.0)
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -8, 1.0),                       # exact tie -> even (1.0)
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),       # exact tie -> even (up)
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),   # just above the tie
        (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),
        (2.0 ** -130, 2.0 ** -130),                   # subnormal, exact
        (0.0, 0.0),
    ]
    for a, r in cases:
        assert mlp.bf16_round(np.array([a], np.float32))[0] == np.float32(r), a
    big = mlp.bf16_round(np.array([3.4028235e38, -3.4028235e38], np.float32))
    assert np.isposinf(big[0]) and np.isneginf(big[1])
    assert np.isnan(mlp.bf16_round(np.array([np.nan], np.float32))[0])
    assert one == 1.0


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    a = np.concatenate([
        rng.standard_normal(50000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 50000).astype(np.float32),
        rng.integers(0, 2 ** 32, 50000, dtype=np.uint64).astype(np.uint32).view(np.float32),
    ])
    a = a[np.isfinite(a)]
    ref = torch.from_numpy(a.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(a).view(np.uint32), ref.view(np.uint32))


def test_gelu_values():
    assert mlp.gelu64(np.array(0.0)) == 0.0
    assert mlp.gelu_grad64(np.array(0.0)) == 0.5
    # Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(mlp.gelu64(np.array(1.0)) - 0.8413447460685429) < 1e-15
    # Phi(-2) = 0.022750131948179195
    assert abs(mlp.gelu64(np.array(-2.0)) - (-2.0 * 0.022750131948179195)) < 1e-15
    x = np.linspace(-6, 6, 241)
    # odd part: x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x)) = x
    assert np.allclose(mlp.gelu64(x) - mlp.gelu64(-x), x, rtol=0, atol=1e-14)
    h = 1e-6
    fd = (mlp.gelu64(x + h) - mlp.gelu64(x - h)) / (2 * h)
    assert np.allclose(fd, mlp.gelu_grad64(x), rtol=0, atol=1e-8)
    # tails: GELU(x) -> x and -> 0
    assert abs(mlp.gelu64(np.array(10.0)) - 10.0) < 1e-15
    assert abs(mlp.gelu64(np.array(-10.0))) < 1e-20


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_zero_weights_give_output_bias(prec):
    theta = np.zeros(mlp.N_PARAMS)
    b4 = np.array([0.25, -1.5, 3.0])
    theta[mlp.OFFSETS[3][1]:] = b4
    x = np.random.default_rng(1).standard_normal((7, 5))
    y, _ = mlp.Net(prec).forward(theta, x)
    assert np.array_equal(np.asarray(y, np.float64), np.tile(b4, (7, 1)))


def _theta(seed):
    return workloads.mlp_init(seed).astype(np.float64)


def test_backward_matches_finite_differences():
    net = mlp.Net("f64")
    rng = np.random.default_rng(2)
    theta = _theta(3)
    theta[mlp.OFFSETS[0][1]:mlp.OFFSETS[0][2]] += 0.3 * rng.standard_normal(128)
    x = rng.standard_normal((6, 5))
    dy = rng.standard_normal((6, 3))

    def L(th):
        y, _ = net.forward(th, x)
        return float(np.sum(y * dy))

    _, cache = net.forward(theta, x)
    g = net.backward(theta, cache, dy)
    picks = []
    for (w0, b0, e) in mlp.OFFSETS:
        picks += list(rng.integers(w0, b0, 12)) + list(rng.integers(b0, e, 4))
    for i in picks:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])
    # a random direction through all parameters at once
    d = rng.standard_normal(mlp.N_PARAMS)
    h = 1e-6
    fd = (L(theta + h * d) - L(theta - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * abs(g @ d)


def test_mse_gradient():
    net = mlp.Net("f64")
    y = np.array([[1.0, 2.0, 3.0]])
    t = np.array([[0.0, 2.0, 5.0]])
    loss, dy = net.mse(y, t)
    assert loss == (1.0 + 0.0 + 4.0) / 3.0
    assert np.allclose(dy, [[2.0 / 3.0, 0.0, -4.0 / 3.0]], rtol=0, atol=1e-16)


def test_bf16_form_rounds_matmul_inputs():
    """A change of an input below half a bf16 unit is invisible to the bf16
    form and visible to the f64 form; the two forms agree to the bf16 bound."""
    rng = np.random.default_rng(4)
    theta = _theta(5)
    x = mlp.bf16_round(rng.standard_normal((32, 5)).astype(np.float32))
    x2 = x * np.float32(1.0 + 2.0 ** -10)        # below half a bf16 ulp
    f, b = mlp.Net("f64"), mlp.Net("bf16")
    y64, _ = f.forward(theta, x.astype(np.float64))
    y64b, _ = f.forward(theta, x2.astype(np.float64))
    yb, _ = b.forward(theta, x)
    yb2, _ = b.forward(theta, x2)
    assert np.array_equal(yb, yb2)
    assert not np.array_equal(y64, y64b)
    # every rounding is at most 2^-9 relative; four layers, GELU slope <= 1.13
    err = np.max(np.abs(yb - y64)) / np.max(np.abs(y64))
    assert 1e-6 < err < 3e-2, err


def test_bf16_backward_close_to_f64():
    rng = np.random.default_rng(6)
    theta = _theta(7)
    x = rng.standard_normal((64, 5))
    dy = rng.standard_normal((64, 3))
    f, b = mlp.Net("f64"), mlp.Net("bf16")
    _, c64 = f.forward(theta, x)
    _, cb = b.forward(theta, x.astype(np.float32))
    g64 = f.backward(theta, c64, dy)
    gb = b.backward(theta, cb, dy.astype(np.float32))
    for (w0, b0, e) in mlp.OFFSETS:
        for s, t in ((w0, b0), (b0, e)):
            ref = g64[s:t]
            err = np.max(np.abs(gb[s:t] - ref)) / np.max(np.abs(ref))
            assert err < 3e-2, (s, err)


def test_adam_closed_form_under_constant_gradient():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves each parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    th = rng.standard_normal(100)
    g = rng.standard_normal(100)
    g[:3] = [0.0, 1e-12, -5.0]
    m = np.zeros(100)
    v = np.zeros(100)
    t0 = th.copy()
    for t in range(1, 6):
        th, m, v = mlp.adam(th, m, v, g, t, lr=1e-3)
    step = 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(th, t0 - 5 * step, rtol=0, atol=1e-12)
    assert th[0] == t0[0]


def test_training_loss_decreases_on_a_fixed_batch():
    net = mlp.Net("f64")
    rng = np.random.default_rng(9)
    theta = _theta(10)
    x = rng.standard_normal((128, 5))
    t = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], np.tanh(x[:, 3] - x[:, 4])], axis=1)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    losses = []
    for step in range(1, 41):
        y, cache = net.forward(theta, x)
        loss, dy = net.mse(y, t)
        losses.append(loss)
        theta, m, v = mlp.adam(theta, m, v, net.backward(theta, cache, dy), step, lr=1e-3)
    assert all(b < a for a, b in zip(losses, losses[1:])), losses
    assert losses[-1] < 0.7 * losses[0]


def test_hull_fallback_hand_cases():
    lo = np.array([-1, -1, -1, -1, -1], np.float32)
    hi = np.array([1, 1, 1, 1, 1], np.float32)
    x = np.array([[0, 0, 0, 0, 0],
                  [1, -1, 1, -1, 1],            # on the boundary: inside
                  [0, 0, 1.0001, 0, 0],
                  [-2, 0, 0, 0, 0],
                  [0, 0, 0, 0, np.nan]], np.float32)
    assert mlp.hull_fallback(x, lo, hi).tolist() == [0, 0, 1, 1, 1]


def test_features_and_tendencies():
    M = np.array([[math.e, math.e ** 2, 1.0]])
    x = mlp.features(M, 2.0, 1, np.zeros(5), np.ones(5))
    assert np.allclose(x, [[1.0, 2.0, 0.0, 2.0, 1.0]], rtol=0, atol=1e-6)
    x = mlp.features(M, 2.0, 1, np.array([1, 0, 0, 0, 0]), np.array([2, 1, 1, 4, 1]))
    assert np.allclose(x, [[0.0, 2.0, 0.0, 0.5, 1.0]], rtol=0, atol=1e-6)
    assert np.allclose(mlp.tendencies([[2.0, 4.0, 8.0]], [[1.0, 4.0, 16.0]], 0.5),
                       [[-1.0, 0.0, 2.0]])


def test_apply_hand_case():
    M = np.array([[1.0, 2.0, 4.0], [8.0, 8.0, 8.0]])
    y = np.array([[1.0, 0.0, -1.0], [5.0, 5.0, 5.0]], np.float32)
    out = mlp.apply(M, y, np.array([0, 1], np.uint8), 0.5, [0.0, 1.0, 0.0], [2.0, 1.0, 0.5])
    # T = (2, 1, -0.5); M (1 + 0.5 T) = (2, 3, 3); the second cell falls back
    assert np.array_equal(out, [[2.0, 3.0, 3.0], [8.0, 8.0, 8.0]])
    assert np.array_equal(mlp.apply(M, y, None, 0.0, [0, 0, 0], [1, 1, 1]), M)
