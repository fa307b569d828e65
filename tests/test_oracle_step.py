"""Pins of the oracle's Steps 0-2 and of the whole timestep.

* F(n) against the exact rational ratio of eq. (3);
* flag predicate (GPU listing, Fig. 3) on hand-built cell layouts;
* shuffle/sort properties (Sec. 3.1-3.2);
* whole step vs brute-force enumeration of every ordering and gamma outcome
  for n <= 4 (chi-square on oracle outcomes over many seeds);
* the one-step expectation identity E[d sum xi] = -(dt/dV) sum a_ij xi_i xi_j;
* invariants over long runs.
"""
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

from tests import brute


def test_pair_scale_exact(oracle_mod):
    assert [oracle_mod.pair_scale(n) for n in (2, 3, 4, 5)] == [1, 3, 3, 5]
    for n in range(2, 3000):
        r = Fraction(n * n - n, 2) / (n // 2)
        assert r.denominator == 1 and oracle_mod.pair_scale(n) == int(r)
    assert oracle_mod.pair_scale(0) == 0 and oracle_mod.pair_scale(1) == 0


LAYOUT_COUNTS = [3, 0, 1, 4, 2]
LAYOUT_FLAGS = [1, 0, 0, 0, 1, 0, 1, 0, 1, 0]   # worked by hand from the predicate


def _layout():
    cell_id = np.repeat(np.arange(len(LAYOUT_COUNTS), dtype=np.int32), LAYOUT_COUNTS)
    n = len(cell_id)
    perm = np.random.default_rng(0).permutation(n)
    # SD ids are scrambled relative to positions; idx lists them cell-major.
    cid = np.empty(n, np.int32)
    cid[perm] = cell_id
    idx = perm.astype(np.uint32)
    cs = np.concatenate([[0], np.cumsum(LAYOUT_COUNTS)]).astype(np.uint32)
    return cid, idx, cs, n


def test_flag_pairs_hand_layout(oracle_mod):
    cid, idx, cs, n = _layout()
    assert list(oracle_mod.flag_pairs(cid, cs, idx, n)) == LAYOUT_FLAGS


def test_normalize_uses_cell_counts(oracle_mod):
    cid, idx, cs, n = _layout()
    flag = oracle_mod.flag_pairs(cid, cs, idx, n)
    dv = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    p = oracle_mod.normalize(np.ones(n // 2), 2.0, dv, cid, cs, flag, idx, n)
    # slots 0 (cell 0, n=3, F=3), 2 and 3 (cell 3, n=4, F=3), 4 (cell 4, n=2, F=1)
    assert p[0] == 2.0 / 1.0 * 3 and p[2] == 2.0 / 8.0 * 3 and p[3] == 2.0 / 8.0 * 3
    assert p[4] == 2.0 / 16.0 * 1
    assert p[1] == 1.0  # unused slot untouched by normalize


def test_shuffle_properties(oracle_mod):
    rng = np.random.default_rng(1)
    n_sd, n_cell = 5000, 37
    cid = rng.integers(0, n_cell, n_sd).astype(np.int32)
    idx0 = rng.permutation(n_sd).astype(np.uint32)
    u = oracle_mod.urand(n_sd, 11, 0, 0, 0)
    idx, cs = oracle_mod.shuffle_per_cell(idx0, n_sd, cid, n_cell, u)
    assert sorted(idx.tolist()) == list(range(n_sd))
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(np.bincount(cid, minlength=n_cell))]))
    c = cid[idx]
    assert np.all(np.diff(c) >= 0)
    key = (u[idx] * 2.0 ** 53).astype(np.uint64)
    same = c[1:] == c[:-1]
    assert np.all(key[1:][same] >= key[:-1][same])
    # independent of the incoming order (keys are indexed by SD id)
    idx_b, cs_b = oracle_mod.shuffle_per_cell(rng.permutation(n_sd).astype(np.uint32), n_sd,
                                              cid, n_cell, u)
    assert np.array_equal(idx, idx_b)
    # equal keys are ordered by SD id
    u_tie = np.zeros(n_sd)
    idx_t, _ = oracle_mod.shuffle_per_cell(idx0, n_sd, cid, n_cell, u_tie)
    for cc in range(n_cell):
        seg = idx_t[cs[cc]:cs[cc + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)


def test_cell_sort_stable(oracle_mod):
    rng = np.random.default_rng(2)
    n_sd, n_cell = 3000, 20
    cid = rng.integers(0, n_cell, n_sd).astype(np.int32)
    idx0 = rng.permutation(n_sd).astype(np.uint32)
    idx, cs = oracle_mod.cell_sort(idx0, n_sd, cid, n_cell)
    ref = idx0[np.argsort(cid[idx0], kind="stable")]
    assert np.array_equal(idx, ref)
    with pytest.raises(ValueError):
        bad = cid.copy()
        bad[3] = n_cell
        oracle_mod.cell_sort(idx0, n_sd, bad, n_cell)


def test_remove_if_equal_0_stable(oracle_mod):
    xi = np.array([3, 0, 5, 0, 0, 7, 1], np.uint64)
    idx = np.array([6, 1, 0, 3, 5, 2, 4], np.uint32)
    out, n = oracle_mod.remove_if_equal_0(idx, 7, xi)
    assert n == 4 and list(out[:4]) == [6, 0, 5, 2]


# ------------------------------------------------------ brute force -------
def _golovin(b):
    return lambda v1, v2: b * (v1 + v2)


BRUTE_CASES = [
    # (xi, volumes, b, dt, dv): moderate p < 1
    ([3, 5, 2, 7], [0.5, 1.25, 2.0, 0.75], 1.0, 1.0, 100.0),
    # odd cell: one SD left unpaired
    ([4, 4, 9], [1.0, 0.5, 1.5], 1.0, 1.0, 40.0),
    # large p: gamma >= 2, caps, case-2 splits, a tie and xi_k = 1
    ([9, 2, 4, 1], [1.0, 2.0, 0.5, 3.0], 1.0, 1.0, 6.0),
    ([2, 2], [1.0, 1.0], 1.0, 1.0, 9.0),
]


@pytest.mark.parametrize("case", range(len(BRUTE_CASES)))
def test_step_matches_bruteforce_distribution(oracle_mod, case):
    xi, vol, b, dt, dv = BRUTE_CASES[case]
    n = len(xi)
    dist = brute.distribution(xi, [vol], _golovin(b), dt, dv)
    assert abs(sum(dist.values()) - 1.0) < 1e-12
    M = 20000
    seen = Counter()
    for seed in range(M):
        out = oracle_mod.step(np.array(xi, np.uint64), np.array([vol]), np.zeros(n, np.int32), 1,
                              [dv], np.arange(n, dtype=np.uint32), n, dt=dt,
                              kernel_id=oracle_mod.KERNEL_GOLOVIN, kparams=[b], seed=seed,
                              run=0, step=0)
        key = (tuple(int(x) for x in out["xi"]), tuple(tuple(float(a) for a in r) for r in out["attr"]))
        assert key in dist, "oracle outcome outside the exact support"
        seen[key] += 1
    chi, dof, other_e, other_o = 0.0, 0, 0.0, 0
    for k, p in dist.items():
        e = p * M
        if e >= 5:
            chi += (seen[k] - e) ** 2 / e
            dof += 1
        else:
            other_e += e
            other_o += seen[k]
    if other_e >= 5:
        chi += (other_o - other_e) ** 2 / other_e
        dof += 1
    dof = max(dof - 1, 1)
    assert chi2_dist.sf(chi, dof) > 1e-4, (chi, dof)


def test_bruteforce_matches_expectation_identity():
    """The exact distribution reproduces the closed-form one-step identity
    (a check on the enumeration itself: selection probability 1/F(n) times
    the F(n) up-scaling of eq. 3, and E[ceil(p - phi)] = p)."""
    for xi, vol, b, dt, dv in BRUTE_CASES[:2]:
        dist = brute.distribution(xi, [vol], _golovin(b), dt, dv)
        e_change = sum(p * (sum(k[0]) - sum(xi)) for k, p in dist.items())
        ref = brute.expected_number_change(xi, [vol], _golovin(b), dt, dv)
        assert abs(e_change - ref) <= 1e-12 * abs(ref)


def test_expectation_identity_monte_carlo(oracle_mod):
    """E[d sum xi] = -(dt/dV) sum_{i<j} a_ij xi_i xi_j at n = 24, every p <= 1."""
    rng = np.random.default_rng(3)
    n = 24
    xi = rng.integers(1, 20, n).astype(np.uint64)
    vol = rng.uniform(0.2, 1.0, n)
    b, dt, dv = 1.0, 1.0, 2000.0
    pmax = (2 * vol.max()) * float(xi.max()) * (dt / dv) * (n - 1)
    assert pmax <= 1.0
    ref = brute.expected_number_change(xi.tolist(), [vol.tolist()], _golovin(b), dt, dv)
    M = 6000
    d = np.empty(M)
    for seed in range(M):
        out = oracle_mod.step(xi, vol[None, :], np.zeros(n, np.int32), 1, [dv],
                              np.arange(n, dtype=np.uint32), n, dt=dt,
                              kernel_id=oracle_mod.KERNEL_GOLOVIN, kparams=[b], seed=seed,
                              run=0, step=0)
        d[seed] = float(out["xi"].sum()) - float(xi.sum())
    se = d.std(ddof=1) / np.sqrt(M)
    assert abs(d.mean() - ref) < 5 * se, (d.mean(), ref, se)


def test_invariants_long_run(oracle_mod):
    from paper_2101_06318_amd import workloads
    w = workloads.box(1024, seed=21)
    # scale the kernel up so collisions, gamma >= 2 and caps all occur
    st = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(1024, dtype=np.uint32), n_live=1024)
    mass0 = float(np.sum(w["xi"].astype(np.float64) * w["attr"][0]))
    tot_prev = int(w["xi"].sum())
    cnt = np.zeros(8, np.uint64)
    for t in range(300):
        out = oracle_mod.step(st["xi"], st["attr"], w["cell_id"], 1, w["dv"], st["idx"],
                              st["n_live"], dt=1.0, kernel_id=0, kparams=[1500.0 * 50],
                              seed=5, run=0, step=t, counters=cnt)
        cnt = out["counters"]
        tot = int(out["xi"].sum())
        assert tot <= tot_prev
        assert np.all(out["xi"] <= st["xi"].max())
        tot_prev = tot
        st = out
    mass1 = float(np.sum(st["xi"].astype(np.float64) * st["attr"][0]))
    assert abs(mass1 - mass0) <= 1e-12 * mass0
    assert cnt[oracle_mod.CNT_COLLISIONS] > 0 and cnt[oracle_mod.CNT_GAMMA_GE2] > 0
    assert cnt[oracle_mod.CNT_CAPPED] > 0
    # SD count constant except removals of xi = 0 (zeroed SDs leave at the next Step 0)
    idx, n = oracle_mod.remove_if_equal_0(st["idx"], st["n_live"], st["xi"])
    assert n == int(np.count_nonzero(st["xi"])) and n <= st["n_live"]


def test_cell_id_out_of_range(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.step(np.ones(4, np.uint64), np.ones((1, 4)), np.array([0, 1, 2, 5], np.int32), 3,
                        [1.0, 1.0, 1.0], np.arange(4, dtype=np.uint32), 4, dt=1.0,
                        kernel_id=0, kparams=[1.0], seed=0, run=0, step=0)
