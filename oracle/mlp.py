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


def ood_fallback(x, lo, hi, occ=None, glo=None, ginv=None):
    """Joint out-of-distribution test: the per-feature box (hull_fallback)
    and, given an occupancy grid occ [G][G][G] over the first three
    features, 1 where the row's cell holds no training input.  Cell index
    k_i = floor((x_i - glo_i) * ginv_i) in float32 (subtraction, then
    product), clamped to [0, G - 1]."""
    x = np.asarray(x, np.float32)
    out = hull_fallback(x, lo, hi)
    if occ is None:
        return out
    occ = np.asarray(occ)
    G = occ.shape[0]
    t = (x[:, :3] - np.asarray(glo, np.float32)) * np.asarray(ginv, np.float32)
    t = np.nan_to_num(t, nan=0.0)           # NaN rows fall back through the box test
    k = np.clip(np.floor(t).astype(np.int64), 0, G - 1)
    empty = occ[k[:, 0], k[:, 1], k[:, 2]] == 0
    return np.where(out == 1, 1, empty.astype(np.uint8)).astype(np.uint8)


def occupancy(x, lo, hi, G):
    """Occupancy grid of standardised training inputs x [n][5] over their
    first three features: G cells per axis spanning [lo_i, hi_i]; returns
    (occ [G][G][G] uint8, glo float32[3], ginv float32[3]) with
    ginv = G / (hi - lo) in float32."""
    lo3 = np.asarray(lo, np.float32)[:3]
    hi3 = np.asarray(hi, np.float32)[:3]
    span = np.where(hi3 > lo3, hi3 - lo3, np.float32(1.0)).astype(np.float32)
    ginv = (np.float32(G) / span).astype(np.float32)
    t = (np.asarray(x, np.float32)[:, :3] - lo3) * ginv
    k = np.clip(np.floor(t).astype(np.int64), 0, G - 1)
    occ = np.zeros((G, G, G), np.uint8)
    occ[k[:, 0], k[:, 1], k[:, 2]] = 1
    return occ, lo3, ginv


def seed_from_moments(M, select, n, dv):
    """Particles of each cell rebuilt from its moments (the surrogate's
    fallback to the particle method).  A selected cell with positive M0,
    M1, M2 (per unit volume) gets n SDs at the standard-normal quantiles
    z_i = sqrt(2) erfinv(2 (i + 1/2)/n - 1): volumes exp(sigma z_i) scaled
    to the mean volume M1/M0, where sigma solves
    R(sigma) = n sum exp(2 sigma z) / (sum exp(sigma z))^2 = M2 M0 / M1^2
    (R is 1 at sigma = 0 and grows towards n): 60 halvings of [0, hi], hi
    the first of 1, 2, 4, ..., 64 with R(hi) >= the target.  Multiplicities
    rint(M0 dv / n), at least 1.  Other cells: multiplicity 0 and volume 0.
    Returns xi [n_cell n] uint64 and v [n_cell n]."""
    from scipy.special import erfinv
    M = np.asarray(M, np.float64)
    nc = len(M)
    xi = np.zeros(nc * n, np.uint64)
    v = np.zeros(nc * n, np.float64)
    z = [math.sqrt(2.0) * float(erfinv(2.0 * ((i + 0.5) / n) - 1.0)) for i in range(n)]

    def ratio(sg):
        S1 = S2 = 0.0
        for zi in z:            # summed in slot order
            e = math.exp(sg * zi)
            S1 += e
            S2 += e * e
        return (n * S2) / (S1 * S1)

    for c in range(nc):
        M0, M1, M2 = (float(a) for a in M[c])
        if (select is not None and not select[c]) or not (M0 > 0 and M1 > 0 and M2 > 0):
            continue
        m1 = M1 / M0
        target = (M2 / M0) / (m1 * m1)
        sg = 0.0
        if target > 1.0 and n > 1:
            lo, hi = 0.0, 1.0
            while hi < 64.0 and ratio(hi) < target:
                hi *= 2.0
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if ratio(mid) < target:
                    lo = mid
                else:
                    hi = mid
            sg = 0.5 * (lo + hi)
        e = [math.exp(sg * zi) for zi in z]
        S = 0.0
        for ei in e:
            S += ei
        scale = (m1 * n) / S
        v[c * n:(c + 1) * n] = [ei * scale for ei in e]
        xi[c * n:(c + 1) * n] = np.uint64(max(1.0, float(np.rint(M0 * dv / n))))
    return xi, v


def moments_merge(M, M_src, select):
    """M[c] = M_src[c] for selected cells."""
    M = np.array(M, np.float64, copy=True)
    sel = np.asarray(select) != 0
    M[sel] = np.asarray(M_src, np.float64)[sel]
    return M
