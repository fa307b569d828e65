"""Brute-force enumeration of one SDM timestep for a single cell of n <= 4 SDs.

Test code, independent of the oracle: it enumerates every ordering of the
cell (each equally likely under a sort by i.i.d. random keys) and every
outcome of gamma = ceil(p - phi) per pair (floor(p) + 1 with probability
frac(p), floor(p) otherwise), then applies eqs. (4)-(6) of arXiv:2101.06318
with its own Python code.  The result is the exact distribution of the
post-step state.
"""
from __future__ import annotations

import itertools
import math
from collections import defaultdict
from fractions import Fraction


def pair_scale(n):
    """(n^2 - n)/2 divided by floor(n/2), from eq. (3), as an exact rational."""
    return Fraction(n * n - n, 2) / (n // 2)


def _apply(xi, A, j, k, gamma):
    """eqs. (4)-(6) on lists xi, A (A = list of attribute lists)."""
    if xi[j] < xi[k]:
        j, k = k, j
    if xi[k] == 0:
        return
    g = min(gamma, xi[j] // xi[k])
    if g == 0:
        return
    d = xi[j] - g * xi[k]
    if d > 0:
        xi[j] = d
        for row in A:
            row[k] = row[k] + float(g) * row[j]
    else:
        h = xi[k] // 2
        xi[j] = h
        xi[k] = xi[k] - h
        for row in A:
            row[j] = row[j] * float(g) + row[k]
            row[k] = row[j]


def distribution(xi, A, kernel, dt, dv):
    """Exact outcome distribution {(xi tuple, attr tuple): probability}.

    kernel(v1, v2) -> a.  p is evaluated in binary64 in the order
    ((a * max xi) * ((dt / dv) * F(n))) with F(n) an exact integer, and the
    probability of gamma = floor(p)+1 is frac(p) (a float, exact enough for a
    chi-square check)."""
    n = len(xi)
    F = pair_scale(n)
    assert F.denominator == 1
    Fi = int(F)
    out = defaultdict(float)
    perms = list(itertools.permutations(range(n)))
    for perm in perms:
        pairs = [(perm[2 * q], perm[2 * q + 1]) for q in range(n // 2)]
        probs = []
        for (j, k) in pairs:
            a = kernel(A[0][j], A[0][k])
            p = (a * float(max(xi[j], xi[k]))) * ((dt / dv) * float(Fi))
            fl = math.floor(p)
            fr = p - fl
            opts = [(fl, 1.0 - fr)] + ([(fl + 1, fr)] if fr > 0 else [])
            probs.append(opts)
        for choice in itertools.product(*probs):
            w = 1.0 / len(perms)
            x = list(xi)
            B = [list(r) for r in A]
            for (jk, (gam, pr)) in zip(pairs, choice):
                w *= pr
                _apply(x, B, jk[0], jk[1], int(gam))
            if w > 0:
                out[(tuple(x), tuple(tuple(r) for r in B))] += w
    return dict(out)


def expected_number_change(xi, A, kernel, dt, dv):
    """Closed form for E[sum xi after - sum xi before] when every p <= 1:
    -(dt/dv) * sum_{i<j} a_ij xi_i xi_j (each pair is picked with
    probability 1/F(n), E[gamma] = p and a collision removes min(xi))."""
    n = len(xi)
    s = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            s += kernel(A[0][i], A[0][j]) * xi[i] * xi[j]
    return -(dt / dv) * s
