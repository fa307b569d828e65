"""GPU parity of each backend-API routine (workflow figure of arXiv:2101.06318)
against the oracle, bit for bit, through the C ABI."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, host, zeros

pytestmark = pytest.mark.gpu

N_MAX = 20000


@pytest.fixture(scope="module")
def sdm():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(sdm):
    c = sdm.Context(N_MAX, n_cell_max=20000, n_attr_max=2)
    yield c
    c.close()


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 2, 7, 1000, 4097])
@pytest.mark.parametrize("stream_id", [0, 1, 3])
def test_urand(sdm, ctx, n, stream_id):
    import torch
    u = zeros(n, torch.float64)
    ctx.urand(u, sdm.rng(0xDEADBEEF12345, 3, 17), stream_id)
    _sync()
    ref = oracle.urand(n, 0xDEADBEEF12345, 3, 17, stream_id)
    assert np.array_equal(host(u), ref)


def test_urand_step_from_device(sdm, ctx):
    import torch
    u = zeros(513, torch.float64)
    step = dev(np.array([41], np.uint32))
    ctx.urand(u, sdm.rng(5, 0, 0, step_dev=step), 1)
    _sync()
    assert np.array_equal(host(u), oracle.urand(513, 5, 0, 41, 1))


@pytest.mark.parametrize("n_sd,n_live", [(1, 1), (10, 7), (5000, 5000), (9001, 8000)])
def test_remove_if_equal_0(sdm, ctx, n_sd, n_live):
    rng = np.random.default_rng(n_sd)
    xi = rng.integers(1, 10, n_sd).astype(np.uint64)
    xi[rng.random(n_sd) < 0.3] = 0
    idx = rng.permutation(n_sd).astype(np.uint32)
    d_idx, d_n, d_xi = dev(idx), dev(np.array([n_live], np.int64)), dev(xi)
    ctx.remove_if_equal_0(d_idx, d_n, d_xi)
    _sync()
    ref_idx, ref_n = oracle.remove_if_equal_0(idx, n_live, xi)
    assert int(host(d_n)[0]) == ref_n
    assert np.array_equal(host(d_idx, np.uint32)[:ref_n], ref_idx[:ref_n])


def _cells(n_sd, n_cell, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_cell, n_sd).astype(np.int32), rng.permutation(n_sd).astype(np.uint32)


@pytest.mark.parametrize("n_sd,n_cell,n_live", [(5000, 37, 4900), (3, 1, 3), (10000, 1, 9999),
                                                (12000, 4096, 12000)])
def test_cell_sort(sdm, ctx, n_sd, n_cell, n_live):
    cid, idx = _cells(n_sd, n_cell, 5)
    d_idx, d_cs = dev(idx), zeros(n_cell + 1, __import__("torch").int32)
    ctx.cell_sort(d_cs, d_idx, dev(np.array([n_live], np.int64)), dev(cid), n_cell)
    _sync()
    ref_idx, ref_cs = oracle.cell_sort(idx, n_live, cid, n_cell)
    assert np.array_equal(host(d_idx, np.uint32)[:n_live], ref_idx[:n_live])
    assert np.array_equal(host(d_cs, np.uint32), ref_cs)


@pytest.mark.parametrize("n_sd,n_cell,n_live", [(5000, 37, 4900), (2, 1, 2), (20000, 1, 20000),
                                                (16000, 250, 15999)])
@pytest.mark.parametrize("keys", ["inline", "given"])
def test_shuffle_per_cell(sdm, ctx, n_sd, n_cell, n_live, keys):
    import torch
    cid, idx = _cells(n_sd, n_cell, 6)
    u = oracle.urand(n_sd, 99, 2, 7, oracle.STREAM_SHUFFLE)
    d_idx, d_cs = dev(idx), zeros(n_cell + 1, torch.int32)
    if keys == "inline":
        ctx.shuffle_per_cell(d_cs, d_idx, dev(np.array([n_live], np.int64)), None, dev(cid),
                             n_cell, None, sdm.rng(99, 2, 7))
    else:
        ctx.shuffle_per_cell(d_cs, d_idx, dev(np.array([n_live], np.int64)), None, dev(cid),
                             n_cell, dev(u), None)
    _sync()
    ref_idx, ref_cs = oracle.shuffle_per_cell(idx, n_live, cid, n_cell, u)
    assert np.array_equal(host(d_idx, np.uint32)[:n_live], ref_idx[:n_live])
    assert np.array_equal(host(d_cs, np.uint32), ref_cs)


def test_shuffle_ties_and_cell_idx_invariance(sdm, ctx):
    import torch
    n_sd, n_cell = 3000, 16
    cid, idx = _cells(n_sd, n_cell, 8)
    u = np.floor(np.random.default_rng(1).random(n_sd) * 4) / 4.0   # many equal keys
    ref_idx, ref_cs = oracle.shuffle_per_cell(idx, n_sd, cid, n_cell, u)
    for cell_idx in (None, dev(np.random.default_rng(2).permutation(n_cell).astype(np.int32))):
        d_idx, d_cs = dev(idx), zeros(n_cell + 1, torch.int32)
        ctx.shuffle_per_cell(d_cs, d_idx, dev(np.array([n_sd], np.int64)), cell_idx, dev(cid),
                             n_cell, dev(u), None)
        _sync()
        assert np.array_equal(host(d_idx, np.uint32), ref_idx)
        assert np.array_equal(host(d_cs, np.uint32), ref_cs)


def _sorted_layout(n_sd, n_cell, seed):
    cid, idx = _cells(n_sd, n_cell, seed)
    u = oracle.urand(n_sd, seed, 0, 0, 0)
    idx, cs = oracle.shuffle_per_cell(idx, n_sd, cid, n_cell, u)
    return cid, idx, cs


@pytest.mark.parametrize("n_sd,n_cell", [(1, 1), (2, 1), (5001, 1), (7000, 300)])
def test_flag_pairs(sdm, ctx, n_sd, n_cell):
    import torch
    cid, idx, cs = _sorted_layout(n_sd, n_cell, 3)
    d_flag = zeros(n_sd, torch.uint8)
    ctx.flag_pairs(d_flag, dev(cid), None, dev(cs), dev(idx), dev(np.array([n_sd], np.int64)))
    _sync()
    assert np.array_equal(host(d_flag), oracle.flag_pairs(cid, cs, idx, n_sd))


KERNELS = [(0, [1500.0]), (1, [1.0]), (2, [3.5e-7]), (3, [2.0e20])]


@pytest.mark.parametrize("kid,kp", KERNELS)
def test_pair_rate_routines(sdm, ctx, kid, kp):
    import torch
    n_sd, n_cell = 6001, 97
    cid, idx, cs = _sorted_layout(n_sd, n_cell, 4)
    rng = np.random.default_rng(kid)
    # radii spanning all three terminal-velocity regimes (1 um .. 3 mm)
    r = 10.0 ** rng.uniform(-6, np.log10(3e-3), n_sd)
    vol = 4.0 / 3.0 * np.pi * r ** 3
    xi = rng.integers(1, 2 ** 40, n_sd).astype(np.uint64)
    dv = rng.uniform(0.5, 2.0, n_cell) * 1e3
    flag = oracle.flag_pairs(cid, cs, idx, n_sd)
    n = np.array([n_sd], np.int64)
    ref = oracle.coalescence_kernel(flag, vol, idx, n_sd, kid, kp)
    ref_m = oracle.times_max(ref, xi, flag, idx, n_sd)
    ref_n = oracle.normalize(ref_m, 2.0, dv, cid, cs, flag, idx, n_sd)
    d = dict(flag=dev(flag), vol=dev(vol), idx=dev(idx), n=dev(n), xi=dev(xi), dv=dev(dv),
             cid=dev(cid), cs=dev(cs))
    p = torch.full((n_sd // 2,), 7.0, dtype=torch.float64, device="cuda")
    k = sdm.kernel(kid, kp)
    ctx.coalescence_kernel(p, d["flag"], d["vol"], d["idx"], d["n"], k)
    _sync()
    assert np.array_equal(host(p), ref)
    ctx.times_max(p, d["xi"], d["flag"], d["idx"], d["n"])
    _sync()
    assert np.array_equal(host(p), ref_m)
    ctx.normalize(p, 2.0, d["dv"], d["cid"], None, d["cs"], d["flag"], d["idx"], d["n"])
    _sync()
    assert np.array_equal(host(p), ref_n)
    q = torch.full((n_sd // 2,), -1.0, dtype=torch.float64, device="cuda")
    ctx.pair_rate(q, 2.0, d["dv"], d["flag"], d["vol"], d["xi"], d["cid"], d["cs"], d["idx"],
                  d["n"], k)
    _sync()
    assert np.array_equal(host(q), ref_n)


@pytest.mark.parametrize("given", [False, True])
def test_compute_gamma(sdm, ctx, given):
    import torch
    n_live = 9999
    rng = np.random.default_rng(12)
    p = rng.uniform(0, 4, n_live // 2)
    p[::7] = 0.0
    p[3::11] = np.floor(p[3::11])   # exact integers
    u = oracle.urand(n_live // 2, 77, 1, 9, oracle.STREAM_GAMMA)
    ref = oracle.compute_gamma(p, u)
    d_p = dev(p)
    if given:
        ctx.compute_gamma(d_p, dev(np.array([n_live], np.int64)), dev(u), None)
    else:
        ctx.compute_gamma(d_p, dev(np.array([n_live], np.int64)), None, sdm.rng(77, 1, 9))
    _sync()
    got = host(d_p)
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_update_attributes(sdm, ctx):
    import torch
    n_sd, n_cell = 8000, 50
    cid, idx, cs = _sorted_layout(n_sd, n_cell, 21)
    flag = oracle.flag_pairs(cid, cs, idx, n_sd)
    rng = np.random.default_rng(22)
    xi = rng.integers(1, 12, n_sd).astype(np.uint64)
    xi[::5] = xi[1::5][: len(xi[::5])]                      # ties
    attr = rng.random((2, n_sd))
    gam = rng.choice([0.0, 1.0, 2.0, 3.0, 7.0, 1e30, np.nan, -0.0, 0.5], n_sd // 2)
    ref_xi, ref_attr, ref_cnt = oracle.update_attributes(xi, attr, gam, flag, idx, n_sd)
    d_xi, d_attr, d_cnt = dev(xi), dev(attr), zeros(8, torch.uint64)
    ctx.update_attributes(d_xi, d_attr, dev(gam), dev(flag), dev(idx),
                          dev(np.array([n_sd], np.int64)), d_cnt)
    _sync()
    assert np.array_equal(host(d_xi), ref_xi)
    assert np.array_equal(host(d_attr), ref_attr)
    assert np.array_equal(host(d_cnt), ref_cnt)
    assert ref_cnt[oracle.CNT_CAPPED] > 0 and ref_cnt[oracle.CNT_ZEROED] > 0


def test_moments(sdm, ctx):
    import torch
    from paper_2101_06318_amd import workloads
    w = workloads.grid(seed=3, nx=16, ny=16)
    n = w["n_sd"]
    idx, cs = oracle.cell_sort(np.arange(n, dtype=np.uint32), n, w["cell_id"], w["n_cell"])
    M = zeros(3 * w["n_cell"], torch.float64)
    ctx.moments(M, dev(w["xi"]), dev(w["attr"][0]), dev(idx), dev(cs), w["n_cell"], dev(w["dv"]))
    _sync()
    ref = oracle.moments(w["xi"], w["attr"][0], w["cell_id"], idx, n, w["n_cell"], w["dv"])
    got = host(M).reshape(-1, 3)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref))


def test_reassign(sdm, ctx):
    import torch
    n_sd = 12345
    c = zeros(n_sd, torch.int32)
    ctx.reassign(c, n_sd, 16384, sdm.rng(3, 0, 12))
    _sync()
    assert np.array_equal(host(c), oracle.reassign(n_sd, 16384, 3, 12))


def test_invalid_calls_raise(sdm, ctx):
    import torch
    with pytest.raises(sdm.SdmError):
        ctx.reassign(zeros(10, torch.int32), 10, 3, sdm.rng(1))      # not a power of two
    with pytest.raises(sdm.SdmError):
        ctx.cell_sort(zeros(2, torch.int32), zeros(4, torch.int32),
                      dev(np.array([4], np.int64)), zeros(4, torch.int32), 10 ** 6)


@pytest.mark.parametrize("n_sd,n_cell", [(1 << 21, 1), (1049600, 16384)])
def test_list_routines_at_full_size(sdm, n_sd, n_cell):
    """sdm_cell_sort and sdm_shuffle_per_cell (inline keys) at the sizes of
    the box and the grid: every entry of the Index and of cell_start."""
    import torch
    big = sdm.Context(n_sd, n_cell, 1)
    cid, idx = _cells(n_sd, n_cell, 13)
    n_live = n_sd - 17
    for routine in ("cell_sort", "shuffle"):
        d_idx, d_cs = dev(idx), zeros(n_cell + 1, torch.int32)
        nl = dev(np.array([n_live], np.int64))
        if routine == "cell_sort":
            big.cell_sort(d_cs, d_idx, nl, dev(cid), n_cell)
            ref_idx, ref_cs = oracle.cell_sort(idx, n_live, cid, n_cell)
        else:
            big.shuffle_per_cell(d_cs, d_idx, nl, None, dev(cid), n_cell, None,
                                 sdm.rng(31, 0, 4))
            u = oracle.urand(n_sd, 31, 0, 4, oracle.STREAM_SHUFFLE)
            ref_idx, ref_cs = oracle.shuffle_per_cell(idx, n_live, cid, n_cell, u)
        _sync()
        assert np.array_equal(host(d_idx, np.uint32)[:n_live], ref_idx[:n_live]), routine
        assert np.array_equal(host(d_cs, np.uint32), ref_cs), routine
    big.close()


@pytest.mark.parametrize("caps", [(32, -1), (0, 64), (16, 40)])
def test_list_routines_overflow_and_global_sort_paths(sdm, caps):
    """Tiny buckets / group capacities force the list routines through the
    overflow and global-memory bitonic paths: results unchanged."""
    import torch
    for n_sd, n_cell in ((20000, 1), (12000, 300)):
        c = sdm.Context(n_sd, n_cell, 1)
        c.set_plan_limits(*caps)
        cid, idx = _cells(n_sd, n_cell, 21)
        u = oracle.urand(n_sd, 8, 1, 2, oracle.STREAM_SHUFFLE)
        ref_idx, ref_cs = oracle.shuffle_per_cell(idx, n_sd, cid, n_cell, u)
        d_idx, d_cs = dev(idx), zeros(n_cell + 1, torch.int32)
        c.shuffle_per_cell(d_cs, d_idx, dev(np.array([n_sd], np.int64)), None, dev(cid),
                           n_cell, None, sdm.rng(8, 1, 2))
        _sync()
        assert np.array_equal(host(d_idx, np.uint32), ref_idx), (caps, n_cell)
        assert np.array_equal(host(d_cs, np.uint32), ref_cs), (caps, n_cell)
        ref_idx, ref_cs = oracle.cell_sort(idx, n_sd, cid, n_cell)
        d_idx, d_cs = dev(idx), zeros(n_cell + 1, torch.int32)
        c.cell_sort(d_cs, d_idx, dev(np.array([n_sd], np.int64)), dev(cid), n_cell)
        _sync()
        assert np.array_equal(host(d_idx, np.uint32), ref_idx), (caps, n_cell)
        assert np.array_equal(host(d_cs, np.uint32), ref_cs), (caps, n_cell)
        c.close()
