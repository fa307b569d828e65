"""Pins of the O(n) per-cell permutations (Sec. 3.2: the CPU backend's serial
permutation, after Appendix A of Shima et al. 2009, and MergeShuffle,
Bacher et al. 2015), CPU only.

* The merge step of MergeShuffle, enumerated exactly (every coin and every
  insertion position with its probability, every arrangement of the two
  shuffled halves), yields every permutation with the same probability.
* The oracle's own output over many seeds: uniform over all n! orders for
  n <= 5, every element equally likely at every position and every pair of
  SDs equally likely to be paired for cells that go through merges,
  a permutation within each cell, cells in the order of a stable cell sort.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest


def _merge_distribution(a, b):
    """Exact output distribution of one merge of shuffled [0, a) and [a, a+b),
    averaged over the a! b! equally likely arrangements of the halves."""
    dist = {}

    def run(T, i, j, p, phase):
        e = len(T)
        if phase == 0:
            # coin 0: stop if i == j, else advance; coin 1: stop if j == e,
            # else swap and advance both
            if i == j:
                run(T, i, j, p / 2, 1)
            else:
                run(T, i + 1, j, p / 2, 0)
            if j == e:
                run(T, i, j, p / 2, 1)
            else:
                U = list(T)
                U[i], U[j] = U[j], U[i]
                run(U, i + 1, j + 1, p / 2, 0)
            return
        if i == e:
            key = tuple(T)
            dist[key] = dist.get(key, 0) + p
            return
        for k in range(0, i + 1):          # uniform position in [s, i], s = 0
            U = list(T)
            U[i], U[k] = U[k], U[i]
            run(U, i + 1, j, p / (i + 1), 1)

    halves = [(A, B) for A in itertools.permutations(range(a))
              for B in itertools.permutations(range(a, a + b))]
    for A, B in halves:
        run(list(A) + list(B), 0, a, Fraction(1, len(halves)), 0)
    return dist


@pytest.mark.parametrize("a,b", [(1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (2, 3), (3, 3)])
def test_merge_step_is_exactly_uniform(a, b):
    dist = _merge_distribution(a, b)
    n = a + b
    assert len(dist) == math.factorial(n)
    assert all(p == Fraction(1, math.factorial(n)) for p in dist.values()), dist


def _chi2_uniform(counts, n_cat):
    tot = sum(counts.values())
    exp = tot / n_cat
    return sum((c - exp) ** 2 / exp for c in counts.values()) + exp * (n_cat - len(counts))


@pytest.mark.parametrize("method", ["fisher_yates", "merge"])
@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_small_cells_uniform(oracle_mod, method, n):
    from scipy.stats import chi2
    counts = {}
    idx = np.arange(n, dtype=np.uint32)[::-1].copy()
    cid = np.zeros(n, np.int32)
    seeds = 6000 if n < 5 else 24000
    for s in range(seeds):
        out, _ = oracle_mod.shuffle_variant(method, idx, n, cid, 1, s, 0, 3)
        counts[tuple(out)] = counts.get(tuple(out), 0) + 1
    assert len(counts) == math.factorial(n)
    stat = _chi2_uniform(counts, math.factorial(n))
    assert chi2.sf(stat, math.factorial(n) - 1) > 1e-4, (counts, stat)


@pytest.mark.parametrize("method", ["fisher_yates", "merge"])
def test_positions_and_pairs_uniform_through_merges(oracle_mod, method):
    """n = 37 (merges at levels 1 and 2): element-at-position and pairing
    frequencies over 8000 seeds."""
    from scipy.stats import chi2
    n, seeds = 37, 8000
    idx = np.arange(n, dtype=np.uint32)
    cid = np.zeros(n, np.int32)
    pos = np.zeros((n, n))
    pair = np.zeros((n, n))
    for s in range(seeds):
        out, _ = oracle_mod.shuffle_variant(method, idx, n, cid, 1, s, 1, 0)
        pos[out, np.arange(n)] += 1
        a, b = out[0:n - 1:2], out[1:n:2]
        pair[np.minimum(a, b), np.maximum(a, b)] += 1
    e = seeds / n
    stat = ((pos - e) ** 2 / e).sum()
    assert chi2.sf(stat, (n - 1) ** 2) > 1e-4, stat
    # (n // 2) pairs per draw, spread over n (n - 1) / 2 unordered pairs
    iu = np.triu_indices(n, 1)
    obs = pair[iu]
    ep = seeds * (n // 2) / len(obs)
    stat = ((obs - ep) ** 2 / ep).sum()
    assert chi2.sf(stat, len(obs) - 1) > 1e-4, stat


@pytest.mark.parametrize("method", ["fisher_yates", "merge"])
def test_cells_keep_their_sds(oracle_mod, method):
    rng = np.random.default_rng(8)
    n, n_cell = 3000, 37
    cid = rng.integers(0, n_cell, n).astype(np.int32)
    idx = rng.permutation(n).astype(np.uint32)
    out, cs = oracle_mod.shuffle_variant(method, idx, n, cid, n_cell, 5, 2, 9)
    ref_idx, ref_cs = oracle_mod.cell_sort(idx, n, cid, n_cell)
    assert np.array_equal(cs, ref_cs)
    for c in range(n_cell):
        a, b = cs[c], cs[c + 1]
        assert sorted(out[a:b]) == sorted(ref_idx[a:b])
    # not the identity: the cells really are permuted
    assert not np.array_equal(out, ref_idx)
    # deterministic in (seed, run, step), different across steps
    out2, _ = oracle_mod.shuffle_variant(method, idx, n, cid, n_cell, 5, 2, 9)
    out3, _ = oracle_mod.shuffle_variant(method, idx, n, cid, n_cell, 5, 2, 10)
    assert np.array_equal(out, out2) and not np.array_equal(out, out3)
