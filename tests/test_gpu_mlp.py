"""Moment surrogate on the matrix cores (sdm_mlp_*, sdm_hull_check) against
the bf16-emulated oracle network.  Tolerance: the GPU and the oracle round
the same matmul inputs to bf16, so they differ only by the float32
accumulation order and GELU's last bits (an occasional one-ulp bf16 flip of
an activation); every tensor must agree to 1e-2 of its largest magnitude
and elementwise to 1e-2 relative plus 1e-3 of that magnitude."""
import numpy as np
import pytest

from oracle import mlp
from paper_2101_06318_amd import workloads
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

TOL = 1e-2


@pytest.fixture(scope="module")
def sdm():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(sdm):
    c = sdm.Context(1024, 16, 1)
    yield c
    c.close()


def _sync():
    import torch
    torch.cuda.synchronize()


def _close(got, ref, what):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = max(np.max(np.abs(ref)), 1e-30)
    err = np.abs(got - ref)
    assert np.max(err) <= TOL * scale, (what, np.max(err) / scale)
    assert np.all(err <= TOL * np.abs(ref) + 1e-3 * scale), (what, np.max(err / (np.abs(ref) + scale)))


def _theta(seed=7):
    th = workloads.mlp_init(seed)
    rng = np.random.default_rng(seed)
    for (w0, b0, e) in mlp.OFFSETS:          # non-trivial biases
        th[b0:e] += rng.uniform(-0.5, 0.5, e - b0).astype(np.float32)
    return th


def _x(B, seed=1):
    return np.random.default_rng(seed).standard_normal((B, 5)).astype(np.float32)


@pytest.mark.parametrize("B", [1, 15, 16, 17, 100, 1000, 4101, 40000, 70001, 300001])
def test_forward_matches_bf16_oracle(sdm, ctx, B):
    import torch
    th = _theta()
    net = sdm.Mlp(ctx, th)
    x = _x(B)
    xd = dev(x)
    y = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
    y2 = torch.zeros_like(y)
    cache = sdm.Mlp.cache_for(B)
    ctx.mlp_forward(y, xd, net)
    ctx.mlp_forward(y2, xd, net, cache=cache)
    _sync()
    ref, _ = mlp.Net("bf16").forward(th, x)
    _close(host(y), ref, "y")
    # inference and training launch shapes compute the same sums
    assert np.array_equal(host(y), host(y2))



def test_training_cache_same_in_both_forward_kernels(sdm, ctx):
    """A batch above the split kernel's size goes through the one-wave-per-tile
    kernel; its training cache of the first 16384 samples must equal
    those the split kernel saves for those samples alone (the same sums)."""
    import torch
    th = _theta(5)
    net = sdm.Mlp(ctx, th)
    B_big, B_small = 300001, 16384
    xd = dev(_x(B_big, 9))
    y = torch.zeros((B_big, 3), dtype=torch.float32, device="cuda")
    c_big = sdm.Mlp.cache_for(B_big)
    c_small = sdm.Mlp.cache_for(B_small)
    ctx.mlp_forward(y, xd, net, cache=c_big)
    y_small = torch.zeros((B_small, 3), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(y_small, xd[:B_small].contiguous(), net, cache=c_small)
    _sync()
    n = c_small.numel()
    assert np.array_equal(host(c_big[:n]), host(c_small))
    assert np.array_equal(host(y[:B_small]), host(y_small))

def test_zero_weights_give_output_bias(sdm, ctx):
    import torch
    th = np.zeros(mlp.N_PARAMS, np.float32)
    th[mlp.OFFSETS[3][1]:] = [0.25, -1.5, 3.0]
    net = sdm.Mlp(ctx, th)
    y = torch.zeros((37, 3), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(y, dev(_x(37)), net)
    _sync()
    assert np.array_equal(host(y), np.tile(np.float32([0.25, -1.5, 3.0]), (37, 1)))


@pytest.mark.parametrize("B", [1, 17, 64, 100, 4096, 9000])
def test_backward_matches_bf16_oracle(sdm, ctx, B):
    import torch
    th = _theta(11)
    net = sdm.Mlp(ctx, th)
    x = _x(B, 2)
    dy = np.random.default_rng(3).standard_normal((B, 3)).astype(np.float32)
    xd = dev(x)
    y = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
    cache = sdm.Mlp.cache_for(B)
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(y, xd, net, cache=cache)
    ctx.mlp_backward(grad, dev(dy), xd, cache, net)
    g1 = host(grad).copy()
    ctx.mlp_backward(grad, dev(dy), xd, cache, net)
    _sync()
    assert np.array_equal(g1, host(grad)), "backward is not deterministic"
    b = mlp.Net("bf16")
    _, c = b.forward(th, x)
    ref = b.backward(th, c, dy)
    for l, (w0, b0, e) in enumerate(mlp.OFFSETS):
        _close(g1[w0:b0], ref[w0:b0], "dW%d" % (l + 1))
        _close(g1[b0:e], ref[b0:e], "db%d" % (l + 1))


def test_mse_matches_oracle(sdm, ctx):
    import torch
    rng = np.random.default_rng(4)
    B = 3001
    y = rng.standard_normal((B, 3)).astype(np.float32)
    t = rng.standard_normal((B, 3)).astype(np.float32)
    dy = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_mse(dy, loss, dev(y), dev(t))
    _sync()
    ref_loss, ref_dy = mlp.Net("bf16").mse(y, t)
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-5 * ref_loss
    assert np.allclose(host(dy), ref_dy, rtol=1e-6, atol=0)


def test_adam_matches_oracle_and_repacks(sdm, ctx):
    import torch
    th = _theta(12)
    net = sdm.Mlp(ctx, th)
    rng = np.random.default_rng(5)
    m = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    th64, m64, v64 = th.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for t in range(1, 4):
        g = (rng.standard_normal(mlp.N_PARAMS) * 10.0 ** rng.uniform(-4, 0, mlp.N_PARAMS)).astype(np.float32)
        ctx.mlp_adam(net, m, v, dev(g), t, lr=1e-3)
        th64, m64, v64 = mlp.adam(th64, m64, v64, g.astype(np.float64), t, lr=1e-3)
    _sync()
    got = host(net.params)
    assert np.allclose(got, th64, rtol=0, atol=1e-6 * 3)
    # float32 moments vs float64: terms of size <= 0.1 |g| <= 0.1, rounding ~1e-8 each
    assert np.allclose(host(m), m64, rtol=1e-5, atol=1e-7)
    assert np.allclose(host(v), v64, rtol=1e-5, atol=1e-9)
    # the packed copy follows the masters: the same bits as a fresh pack,
    # the transposed fragments of the backward pass included
    fresh = sdm.Mlp(ctx, got)
    _sync()
    assert np.array_equal(host(net.packed), host(fresh.packed))
    x = dev(_x(77))
    y1 = torch.zeros((77, 3), dtype=torch.float32, device="cuda")
    y2 = torch.zeros_like(y1)
    ctx.mlp_forward(y1, x, net)
    ctx.mlp_forward(y2, x, fresh)
    _sync()
    assert np.array_equal(host(y1), host(y2))


def test_training_on_a_fixed_batch(sdm, ctx):
    """Forward, MSE, backward and Adam on the GPU: the loss falls at every
    step and follows the bf16 oracle's training curve."""
    import torch
    th = _theta(13)
    net = sdm.Mlp(ctx, th)
    B = 512
    rng = np.random.default_rng(6)
    x = rng.standard_normal((B, 5)).astype(np.float32)
    tgt = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], np.tanh(x[:, 3] - x[:, 4])], 1).astype(np.float32)
    xd, td = dev(x), dev(tgt)
    y = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
    dy = torch.zeros_like(y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cache = sdm.Mlp.cache_for(B)
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    b = mlp.Net("bf16")
    th_o, m_o, v_o = th.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    gl, ol = [], []
    for t in range(1, 21):
        ctx.mlp_forward(y, xd, net, cache=cache)
        ctx.mlp_mse(dy, loss, y, td)
        ctx.mlp_backward(grad, dy, xd, cache, net)
        ctx.mlp_adam(net, m, v, grad, t, lr=2e-3)
        _sync()
        gl.append(float(host(loss)[0]))
        yo, co = b.forward(th_o.astype(np.float32), x)
        lo, dyo = b.mse(yo, tgt)
        ol.append(lo)
        th_o, m_o, v_o = mlp.adam(th_o, m_o, v_o, b.backward(th_o.astype(np.float32), co, dyo), t, lr=2e-3)
    assert all(q < p for p, q in zip(gl, gl[1:])), gl
    assert np.allclose(gl, ol, rtol=2e-2), (gl, ol)


def test_hull_check(sdm, ctx):
    import torch
    rng = np.random.default_rng(7)
    B = 5000
    x = rng.standard_normal((B, 5)).astype(np.float32) * 1.3
    x[7, 2] = np.nan
    lo = np.float32([-2, -2.5, -2, -3, -2])
    hi = np.float32([2, 2, 2.5, 3, 2])
    x[8] = lo
    x[9] = hi
    fb = torch.full((B,), 7, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(8, dtype=torch.int64, device="cuda")
    ctx.hull_check(fb, dev(x), lo, hi, counters=cnt)
    _sync()
    ref = mlp.hull_fallback(x, lo, hi)
    assert np.array_equal(host(fb), ref)
    assert ref[7] == 1 and ref[8] == 0 and ref[9] == 0
    assert int(host(cnt)[sdm.CNT_FALLBACK]) == int(ref.sum()) > 0


def test_features_and_apply(sdm, ctx):
    import torch
    rng = np.random.default_rng(8)
    n = 3000
    M = np.stack([10 ** rng.uniform(6, 9, n), 10 ** rng.uniform(-6, -3, n),
                  10 ** rng.uniform(-20, -14, n)], 1)
    mean = np.float32([18.0, -10.0, -40.0, 2.0, 0.5])
    std = np.float32([2.0, 1.5, 3.0, 3.0, 0.5])
    x = torch.zeros((n, 5), dtype=torch.float32, device="cuda")
    Md = dev(M)
    ctx.mlp_features(x, Md, 2.0, 1, mean, std)
    y = rng.standard_normal((n, 3)).astype(np.float32)
    fb = (rng.random(n) < 0.1).astype(np.uint8)
    tm, ts = np.float32([-1e-4, 0.0, 2e-4]), np.float32([1e-4, 1e-9, 3e-4])
    ctx.mlp_apply(Md, dev(y), 2.0, tm, ts, fallback=dev(fb))
    _sync()
    ref_x = mlp.features(M, 2.0, 1, mean, std)
    assert np.allclose(host(x), ref_x, rtol=2e-7, atol=2e-7)
    assert np.array_equal(host(Md), mlp.apply(M, y, fb, 2.0, tm, ts))
