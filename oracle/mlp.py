"""Oracle for the moment-tendency surrogate network (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module; the product library never does.

The paper (arXiv:2101.06318, Sec. 5, outlook) motivates replacing the
particle-based coagulation of a cell by a learned model of its bulk
moments, since a coupled fluid solver needs only statistical moments of the
spectrum.  The surrogate here maps the features of one cell,
x = (log M0, log M1, log M2, dt, kernel id) standardised, to the three
relative moment tendencies (M_k(t + dt) - M_k(t)) / (M_k(t) dt),
standardised.  Architecture: 5 -> 128 -> 128 -> 128 -> 3, exact-erf GELU
after each hidden layer, linear output, mean-squared-error loss, Adam.

Parameters are one flat vector in the order W1, b1, W2, b2, W3, b3, W4, b4,
each W row-major [out][in] (layer computes z = W a + b).

Two forms of the same network:

* ``Net(precision="f64")``: float64 everywhere, no rounding (form i).
* ``Net(precision="bf16")``: bf16-emulated (form ii).  Weights are the
  float32 masters rounded to bfloat16 (round to nearest even); every matmul
  input (x, activations, back-propagated errors) is rounded to bfloat16;
  each matmul's sum of exact bf16 x bf16 products is formed in float64 and
  rounded once to float32 (one fixed order: exact sum, then one rounding);
  bias adds, GELU, its derivative and the bias-gradient sums are float32.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf as _erf

LAYERS = (5, 128, 128, 128, 3)
N_IN, N_HID, N_OUT = 5, 128, 3


def _offsets():
    off, o = [], 0
    for i in range(4):
        fi, fo = LAYERS[i], LAYERS[i + 1]
        off.append((o, o + fo * fi, o + fo * fi + fo))
        o += fo * fi + fo
    return off, o


OFFSETS, N_PARAMS = _offsets()          # (W start, b start, end) per layer; 34179


def split(theta):
    """Views (W_l [out][in], b_l [out]) of a flat parameter vector."""
    out = []
    for i, (w0, b0, e) in enumerate(OFFSETS):
        fi, fo = LAYERS[i], LAYERS[i + 1]
        out.append((theta[w0:b0].reshape(fo, fi), theta[b0:e]))
    return out


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  NaN stays NaN; values beyond the bf16 range become +-inf."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(nan, (u | 0x00400000) & 0xFFFF0000, r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a.shape)


def gelu64(z):
    """GELU with the exact normal CDF: z * Phi(z), Phi(z) = (1 + erf(z/sqrt 2))/2."""
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad64(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


class Net:
    """Forward and backward of the surrogate MLP in one of the two forms."""

    def __init__(self, precision="f64"):
        assert precision in ("f64", "bf16")
        self.p = precision

    # rounding hooks of the two forms
    def _in(self, a):
        """A matmul input."""
        if self.p == "f64":
            return np.asarray(a, np.float64)
        return bf16_round(np.asarray(a, np.float32)).astype(np.float64)

    def _acc(self, s):
        """A matmul result (exact products summed in float64)."""
        return s if self.p == "f64" else s.astype(np.float32)

    def _f(self, a):
        """An elementwise result (bias add, GELU, its derivative)."""
        return a if self.p == "f64" else np.asarray(a, np.float64).astype(np.float32)

    def weights(self, theta):
        if self.p == "f64":
            return [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in split(theta)]
        t32 = np.asarray(theta, np.float32)
        return [(bf16_round(W).astype(np.float64), b.astype(np.float32)) for W, b in split(t32)]

    def forward(self, theta, x):
        """x [B][5] -> (y [B][3], cache).  cache keeps the layer inputs (as the
        matmuls saw them) and the pre-activations of the hidden layers."""
        Wb = self.weights(theta)
        a = np.asarray(x, np.float64 if self.p == "f64" else np.float32)
        ins, zs = [], []
        for l, (W, b) in enumerate(Wb):
            ai = self._in(a)
            ins.append(ai)
            z = self._f(self._acc(ai @ W.T) + b)
            if l < 3:
                zs.append(z)
                a = self._f(gelu64(np.asarray(z, np.float64)))
            else:
                a = z
        return a, dict(ins=ins, zs=zs, Wb=Wb)

    def backward(self, theta, cache, dy):
        """dL/dy [B][3] -> flat gradient (same layout as theta)."""
        Wb, ins, zs = cache["Wb"], cache["ins"], cache["zs"]
        g = np.zeros(N_PARAMS, np.float64)
        dz = np.asarray(dy, np.float64 if self.p == "f64" else np.float32)
        for l in range(3, -1, -1):
            W, _ = Wb[l]
            w0, b0, e = OFFSETS[l]
            dzi = self._in(dz)
            g[w0:b0] = self._acc(dzi.T @ ins[l]).reshape(-1)
            g[b0:e] = self._f(np.sum(np.asarray(dz, np.float64), axis=0))
            if l > 0:
                dh = self._acc(dzi @ W)
                dz = self._f(dh * self._f(gelu_grad64(np.asarray(zs[l - 1], np.float64))))
        return g

    def mse(self, y, t):
        """Mean over all B*3 outputs of (y - t)^2 and its gradient wrt y."""
        y = np.asarray(y, np.float64)
        d = y - np.asarray(t, np.float64)
        n = d.size
        return float(np.sum(d * d) / n), self._f(2.0 * d / n)


def adam(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns new
    (theta, m, v).  float64 arithmetic."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def hull_fallback(x, lo, hi):
    """1 where any feature of a row lies outside [lo, hi] (or is NaN), else 0."""
    x = np.asarray(x, np.float32)
    inside = (x >= np.asarray(lo, np.float32)) & (x <= np.asarray(hi, np.float32))
    return (~np.all(inside, axis=1)).astype(np.uint8)


def features(M, dt, kernel_id, mean, std):
    """Standardised features of cells with moments M [n][3] (float64):
    ((log M0, log M1, log M2, dt, kernel id) - mean) / std in float64 with
    mean and std given as float32 values, rounded to float32."""
    M = np.asarray(M, np.float64)
    raw = np.stack([np.log(M[:, 0]), np.log(M[:, 1]), np.log(M[:, 2]),
                    np.full(len(M), float(dt)), np.full(len(M), float(kernel_id))], axis=1)
    mean = np.asarray(mean, np.float32).astype(np.float64)
    std = np.asarray(std, np.float32).astype(np.float64)
    return ((raw - mean) / std).astype(np.float32)


def tendencies(M0, M1, dt):
    """Relative moment tendencies (M1_k - M0_k) / (M0_k dt)."""
    M0 = np.asarray(M0, np.float64)
    return (np.asarray(M1, np.float64) - M0) / (M0 * dt)


def apply(M, y, fallback, dt, mean, std):
    """Surrogate update of the moments: T = y std + mean (de-standardised
    relative tendency), M_k <- M_k (1 + dt T_k) for cells that do not fall
    back; float64, evaluated in that order."""
    M = np.array(M, np.float64, copy=True)
    y = np.asarray(y, np.float32).astype(np.float64)
    tend = y * np.asarray(std, np.float32).astype(np.float64) + np.asarray(mean, np.float32).astype(np.float64)
    new = M * (1.0 + float(dt) * tend)
    keep = np.ones(len(M), bool) if fallback is None else (np.asarray(fallback) == 0)
    M[keep] = new[keep]
    return M
