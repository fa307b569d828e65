"""Pins of the oracle's coalescence kernels, cube root and moments.

The Golovin, constant and multiplicative kernels are the analytically
solvable ones the paper lists (Sec. 2.1); the gravitational (geometric)
kernel is only named by the paper (Sec. 4), so its terminal-velocity
constants are a reading (textbook three-regime power law) and its values are
parity unpinned beyond the properties checked here.
"""
import numpy as np

from paper_2101_06318_amd import workloads


def test_cbrt_accuracy_and_exact_cubes(oracle_mod):
    for x, y in ((8.0, 2.0), (27.0, 3.0), (0.125, 0.5), (1e-18, 1e-6), (0.0, 0.0), (64.0, 4.0)):
        assert oracle_mod.cbrt(x) == y
    rng = np.random.default_rng(0)
    xs = 10.0 ** rng.uniform(-21, -6, 3000)
    for x in xs:
        got = oracle_mod.cbrt(float(x))
        ref = np.cbrt(x)
        assert abs(got - ref) <= 2 * np.spacing(ref), (x, got, ref)


def test_kernel_values(oracle_mod):
    # Golovin: b (v1 + v2), symmetric bit for bit
    assert oracle_mod.kernel_value(0, [1500.0], 1e-12, 3e-12) == 1500.0 * (1e-12 + 3e-12)
    assert oracle_mod.kernel_value(2, [7.5], 1.0, 2.0) == 7.5
    assert oracle_mod.kernel_value(3, [2.0], 3.0, 5.0) == 30.0
    rng = np.random.default_rng(4)
    for _ in range(200):
        v1, v2 = (4.0 / 3.0 * np.pi * (10.0 ** rng.uniform(-6.5, -3, 2)) ** 3)
        for kid in (0, 1):
            a = oracle_mod.kernel_value(kid, [1500.0 if kid == 0 else 1.0], v1, v2)
            b = oracle_mod.kernel_value(kid, [1500.0 if kid == 0 else 1.0], v2, v1)
            assert a == b and a >= 0


def test_geometric_kernel_properties(oracle_mod):
    v = 4.0 / 3.0 * np.pi * (20e-6) ** 3
    assert oracle_mod.kernel_value(1, [1.0], v, v) == 0.0      # equal fall speeds
    # larger drop falls faster: kernel grows with the size contrast
    a1 = oracle_mod.kernel_value(1, [1.0], v, 2 * v)
    a2 = oracle_mod.kernel_value(1, [1.0], v, 8 * v)
    assert a2 > a1 > 0
    # efficiency scales the kernel linearly
    assert oracle_mod.kernel_value(1, [0.5], v, 8 * v) == a2 * 0.5
    # pi (r1 + r2)^2 |w1 - w2| written out for one pair, r from the volume
    r1, r2 = 15e-6, 150e-6
    v1, v2 = 4.0 / 3.0 * np.pi * r1 ** 3, 4.0 / 3.0 * np.pi * r2 ** 3
    want = np.pi * (r1 + r2) ** 2 * abs(1.19e8 * r1 ** 2 - 8e3 * r2)
    assert abs(oracle_mod.kernel_value(1, [1.0], v1, v2) - want) <= 1e-12 * want


K1, K2, K3 = 1.19e8, 8.0e3, 201.0   # textbook power-law coefficients [1/(m s), 1/s, m^0.5/s]


def test_terminal_velocity_laws():
    """The three laws with their textbook coefficients, each inside its own
    range: Stokes k1 r^2, linear k2 r, square-root k3 sqrt(r)."""
    import oracle
    tv = oracle.terminal_velocity
    assert abs(tv(10e-6) - 1.19e-2) <= 1e-15                 # 10 um: 1.19 cm/s
    assert abs(tv(30e-6) - K1 * 30e-6 ** 2) <= 1e-15
    assert abs(tv(100e-6) - 0.8) <= 1e-15                    # 100 um: 0.8 m/s
    assert abs(tv(400e-6) - K2 * 400e-6) <= 1e-15
    assert abs(tv(1e-3) - K3 * np.sqrt(1e-3)) <= 1e-15       # 1 mm: 6.36 m/s
    assert abs(tv(2e-3) - K3 * np.sqrt(2e-3)) <= 1e-15


def test_terminal_velocity_continuous_at_the_regime_changes():
    """The law changes where the neighbouring laws meet (r = k2/k1 and
    r = (k3/k2)^2), so w(r) has no jump there and increases throughout."""
    import oracle
    tv = oracle.terminal_velocity
    for rb in (K2 / K1, (K3 / K2) ** 2):
        lo, hi = tv(np.nextafter(rb, 0.0)), tv(rb)
        assert abs(hi - lo) <= 1e-14 * hi, (rb, lo, hi)
        # within 0.1 % of the boundary w moves by at most 0.3 %
        assert abs(tv(rb * 0.999) - tv(rb * 1.001)) < 0.003 * tv(rb)
    assert abs(K2 / K1 - 67.2269e-6) < 1e-10 and abs((K3 / K2) ** 2 - 631.2656e-6) < 1e-10
    rs = np.geomspace(1e-6, 5e-3, 4000)
    w = np.array([tv(r) for r in rs])
    assert np.all(w > 0) and np.all(np.diff(w) > 0)


def test_moments_definition(oracle_mod):
    w = workloads.grid(seed=3, nx=4, ny=4)
    n = w["n_sd"]
    idx = np.arange(n, dtype=np.uint32)
    M = oracle_mod.moments(w["xi"], w["attr"][0], w["cell_id"], idx, n, w["n_cell"], w["dv"])
    for c in range(w["n_cell"]):
        sel = w["cell_id"] == c
        x = w["xi"][sel].astype(np.float64)
        v = w["attr"][0][sel]
        assert M[c, 0] == x.sum() / w["dv"][c]          # integers < 2^53: exact
        assert abs(M[c, 1] - np.sum(x * v) / w["dv"][c]) <= 1e-13 * M[c, 1]
        assert abs(M[c, 2] - np.sum(x * v * v) / w["dv"][c]) <= 1e-13 * M[c, 2]
    # SDs outside the Index do not count
    M2 = oracle_mod.moments(w["xi"], w["attr"][0], w["cell_id"], idx[1:], n - 1, w["n_cell"], w["dv"])
    c0 = w["cell_id"][0]
    sel = w["cell_id"] == c0
    assert M2[c0, 0] == (w["xi"][sel].astype(np.float64).sum() - float(w["xi"][0])) / w["dv"][c0]


def test_reassign_uniform_cells(oracle_mod):
    cid = oracle_mod.reassign(200000, 16384, 3, 7)
    assert cid.min() >= 0 and cid.max() < 16384
    counts = np.bincount(cid, minlength=16384)
    assert abs(counts.mean() - 200000 / 16384) < 1e-9
    assert abs(counts.var() / counts.mean() - 1) < 0.05   # Poisson occupancy
    u = oracle_mod.uniform(3, 0, 7, oracle_mod.STREAM_REASSIGN, 11)
    assert cid[11] == int(u * 16384)
