"""Pins of the oracle's collision update (eqs. 4-6 of arXiv:2101.06318).

Expected values are worked by hand from the equations (attributes are small
integers so every sum is exact) plus the paper's own worked example.
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _one_pair(oracle_mod, xi, A, gamma, order=(0, 1)):
    """Two SDs (ids 0, 1) in one cell, sorted positions given by `order`."""
    idx = np.array(order, np.uint32)
    flag = np.array([1, 0], np.uint8)
    attr = np.array(A, np.float64)
    if attr.ndim == 1:
        attr = attr[None, :]
    return oracle_mod.update_attributes(np.array(xi, np.uint64), attr,
                                        np.array([gamma], np.float64), flag, idx, 2)


def test_worked_example(oracle_mod):
    ex = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    A = [[1.0, 3.0], [10.0, 20.0]]           # two attributes, SD 0 = j, SD 1 = k
    xi, attr, cnt = _one_pair(oracle_mod, [ex["xi_j"], ex["xi_k"]], A, float(ex["gamma"]))
    assert int(xi[0]) == ex["xi_j_after"] and int(xi[1]) == ex["xi_k_after"]
    g = ex["gamma_tilde"]
    assert attr[0, 0] == 1.0 and attr[0, 1] == 3.0 + g * 1.0      # 7.0
    assert attr[1, 0] == 10.0 and attr[1, 1] == 20.0 + g * 10.0   # 60.0
    assert cnt[oracle_mod.CNT_COLLISIONS] == 1 and cnt[oracle_mod.CNT_CAPPED] == 1
    assert cnt[oracle_mod.CNT_GAMMA_GE2] == 1


def test_j_is_larger_multiplicity_regardless_of_position(oracle_mod):
    # SD 1 sorted first but has the smaller multiplicity: j must be SD 0.
    xi, attr, _ = _one_pair(oracle_mod, [9, 2], [1.0, 3.0], 5.0, order=(1, 0))
    assert list(xi) == [1, 2] and list(attr[0]) == [1.0, 7.0]


def test_case2_even_split(oracle_mod):
    # xi_j = 6, xi_k = 2, gamma = 3 -> g = 3, 6 - 3*2 = 0: eq. (6)
    xi, attr, cnt = _one_pair(oracle_mod, [6, 2], [1.0, 3.0], 3.0)
    assert list(xi) == [1, 1]
    assert list(attr[0]) == [6.0, 6.0]          # 3*1 + 3 on both
    assert cnt[oracle_mod.CNT_ZEROED] == 0


def test_case2_odd_split(oracle_mod):
    # xi_j = 9, xi_k = 3, gamma = 3 -> g = 3, split floor(3/2)=1 to j, 2 to k
    xi, attr, _ = _one_pair(oracle_mod, [9, 3], [2.0, 5.0], 3.0)
    assert list(xi) == [1, 2]
    assert list(attr[0]) == [11.0, 11.0]


def test_case2_xi_k_one_removes_j(oracle_mod):
    # xi_j = xi_k = 1, gamma = 1: split impossible, j left with xi = 0 (Sec. 2.2)
    xi, attr, cnt = _one_pair(oracle_mod, [1, 1], [2.0, 5.0], 1.0)
    assert list(xi) == [0, 1]
    assert cnt[oracle_mod.CNT_ZEROED] == 1
    idx, n = oracle_mod.remove_if_equal_0(np.array([0, 1], np.uint32), 2, xi)
    assert n == 1 and idx[0] == 1


def test_tie_j_is_earlier_position(oracle_mod):
    # equal multiplicities 5,5, gamma 1 -> case 2: j (earlier position) gets 2.
    xi, attr, _ = _one_pair(oracle_mod, [5, 5], [1.0, 3.0], 1.0, order=(1, 0))
    assert int(xi[1]) == 2 and int(xi[0]) == 3
    assert list(attr[0]) == [4.0, 4.0]


def test_no_collision_paths(oracle_mod):
    for gamma in (0.0, -0.0, np.nan, 0.999):
        xi, attr, cnt = _one_pair(oracle_mod, [9, 2], [1.0, 3.0], gamma)
        assert list(xi) == [9, 2] and list(attr[0]) == [1.0, 3.0]
        assert cnt[oracle_mod.CNT_COLLISIONS] == 0


def test_gamma_cap_and_saturation(oracle_mod):
    # gamma far above 2^64 saturates; cap floor(9/2) = 4 applies
    xi, attr, cnt = _one_pair(oracle_mod, [9, 2], [1.0, 3.0], 1e30)
    assert list(xi) == [1, 2] and attr[0, 1] == 7.0
    assert cnt[oracle_mod.CNT_CAPPED] == 1
    # gamma = 2 below the cap: case 1 with g = 2
    xi, attr, cnt = _one_pair(oracle_mod, [9, 2], [1.0, 3.0], 2.0)
    assert list(xi) == [5, 2] and attr[0, 1] == 5.0
    assert cnt[oracle_mod.CNT_CAPPED] == 0


def test_unflagged_positions_untouched(oracle_mod):
    xi = np.array([9, 2, 7], np.uint64)
    attr = np.array([[1.0, 3.0, 4.0]])
    flag = np.array([0, 1, 0], np.uint8)
    idx = np.array([2, 0, 1], np.uint32)  # pair at positions (1,2) = SDs 0,1; slot 0
    out_xi, out_attr, _ = oracle_mod.update_attributes(xi, attr, np.array([1.0]), flag, idx, 3)
    assert list(out_xi) == [7, 2, 7] and list(out_attr[0]) == [1.0, 4.0, 4.0]


def test_mass_conserved_and_no_wrap_random_pairs(oracle_mod):
    rng = np.random.default_rng(5)
    n = 4000
    xi = rng.integers(1, 50, n).astype(np.uint64)
    attr = rng.random((2, n))
    idx = rng.permutation(n).astype(np.uint32)
    flag = np.zeros(n, np.uint8)
    flag[0::2] = 1
    gamma = rng.integers(0, 6, n // 2).astype(np.float64)
    out_xi, out_attr, _ = oracle_mod.update_attributes(xi, attr, gamma, flag, idx, n)
    assert np.all(out_xi <= xi)          # never grows, never wraps
    for a in range(2):
        m0 = np.sum(xi.astype(np.float64) * attr[a])
        m1 = np.sum(out_xi.astype(np.float64) * out_attr[a])
        assert abs(m1 - m0) <= 1e-12 * abs(m0)
