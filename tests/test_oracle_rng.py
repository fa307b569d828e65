"""Pins of the oracle's uniform stream (Philox4x32-10 + 53-bit mapping).

The paper names only its GPU random source (CURandRTC, Sec. 3.2); the reading
taken is Philox4x32-10 with counter (e>>1, step, stream, run) and key
(lo32(seed), hi32(seed)).  Pinned against (i) the published known-answer
vectors and (ii) PyTorch's header-only Philox engine compiled into a small
harness -- an implementation independent of the oracle.
"""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(oracle_mod.philox(ctr, key)) == out


@pytest.fixture(scope="module")
def torch_harness(tmp_path_factory):
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("torch Philox header not present")
    exe = str(tmp_path_factory.mktemp("ph") / "philox_torch")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc,
                           os.path.join(HERE, "harness", "philox_torch.cpp"), "-o", exe])
    return exe


def test_philox_matches_torch_engine(oracle_mod, torch_harness):
    rng = np.random.default_rng(12345)
    cases = rng.integers(0, 2 ** 32, size=(500, 6), dtype=np.uint64)
    cases[:5] = 0
    cases[5] = 2 ** 32 - 1
    txt = "\n".join(" ".join(str(int(x)) for x in row) for row in cases) + "\n"
    out = subprocess.run([torch_harness], input=txt, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        got = oracle_mod.philox(row[:4].astype(np.uint32), row[4:6].astype(np.uint32))
        assert list(got) == ref


def test_word_layout(oracle_mod):
    """Element e uses block ctr=(e>>1, step, stream, run): even e takes words
    0-1, odd e words 2-3, high word first."""
    seed = 0x0123456789ABCDEF
    for e in (0, 1, 2, 3, 1000, 1001, 2 ** 31 + 7):
        blk = oracle_mod.philox([e >> 1, 17, 1, 5], [seed & 0xFFFFFFFF, seed >> 32])
        hi, lo = (blk[2], blk[3]) if e & 1 else (blk[0], blk[1])
        assert oracle_mod.word(seed, 5, 17, 1, e) == (int(hi) << 32) | int(lo)


def test_uniform_is_53bit_and_in_range(oracle_mod):
    u = oracle_mod.urand(20000, 7, 0, 3, 0)
    assert np.all(u >= 0.0) and np.all(u < 1.0)
    k = u * 2.0 ** 53
    assert np.all(k == np.floor(k))
    for e in (0, 1, 99):
        w = oracle_mod.word(7, 0, 3, 0, e)
        assert u[e] == (w >> 11) * 2.0 ** -53


def test_uniform_statistics(oracle_mod):
    n = 200000
    u = oracle_mod.urand(n, 99, 3, 1, 1)
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = ((h - n / 64) ** 2 / (n / 64)).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5
    # streams, steps and runs are distinct sequences
    v = oracle_mod.urand(1000, 99, 3, 1, 0)
    w = oracle_mod.urand(1000, 99, 3, 2, 1)
    assert not np.array_equal(u[:1000], v) and not np.array_equal(u[:1000], w)
