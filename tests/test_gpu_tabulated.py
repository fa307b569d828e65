"""GPU parity of the tabulated kernel (the plug-in point for general kernels)
against the oracle: the pair-rate routines and whole fused timesteps of a
box and of a grid, bit for bit, with a random symmetric table."""
import numpy as np
import pytest

import oracle
from paper_2101_06318_amd import workloads
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdm():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as m
    m.lib()
    return m


def _table(n, seed, scale):
    rng = np.random.default_rng(seed)
    T = rng.uniform(0.0, scale, (n, n))
    return (T + T.T) / 2.0


# the box's volumes (about 1e-18 .. 1e-11 m^3) in four cells per octave
LO, N, M = 3850, 160, 2


def _steps(sdm, w, steps, kp, T, seed, n_cell=1, dv=None):
    import torch
    n_sd = w["n_sd"]
    cid = w["cell_id"] if n_cell > 1 else None
    st = sdm.State(w["xi"], w["attr"], cid, n_cell, want_gamma=True)
    ctx = sdm.Context(n_sd, n_cell, w["attr"].shape[0])
    T_dev = dev(T)
    k = sdm.kernel(oracle.KERNEL_TABULATED, kp, table=T_dev)
    dvs = np.broadcast_to(np.asarray(w["dv"], np.float64), (n_cell,)).copy()
    d_dv = dev(dvs)
    ref = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
    cnt = np.zeros(8, np.uint64)
    for t in range(steps):
        ctx.step(st, w["dt"], k, sdm.rng(seed, 0, t), dv_per_cell=d_dv)
        ref = oracle.step(ref["xi"], ref["attr"], cid, n_cell, dvs, ref["idx"], ref["n_live"],
                          dt=w["dt"], kernel_id=oracle.KERNEL_TABULATED, kparams=kp,
                          seed=seed, run=0, step=t, counters=cnt, want_gamma=True, table=T)
        cnt = ref["counters"]
        torch.cuda.synchronize()
        n = int(host(st.n_live)[0])
        assert n == ref["n_live"], t
        assert np.array_equal(host(st.xi), ref["xi"]), t
        assert np.array_equal(host(st.attr), ref["attr"]), t
        assert np.array_equal(host(st.idx, np.uint32)[:n], ref["idx"][:n]), t
        assert np.array_equal(host(st.gamma_out), ref["gamma"]), t
    assert np.array_equal(host(st.counters), cnt)
    assert cnt[oracle.CNT_COLLISIONS] > 0
    ctx.close()


@pytest.mark.parametrize("n_sd", [7, 5000, 40001])
def test_tabulated_box_steps(sdm, n_sd):
    w = workloads.box(n_sd, seed=n_sd)
    _steps(sdm, w, 3, [1.0, LO, N, M], _table(N, 1, 4e-8), seed=5)


def test_tabulated_grid_steps(sdm):
    w = workloads.grid(seed=3, nx=16, ny=16)
    # scaled so that pairs of the grid's small cells collide
    _steps(sdm, w, 3, [2.0, LO, N, M], _table(N, 2, 1e-9), seed=6, n_cell=w["n_cell"])


def test_tabulated_pair_rate_routine(sdm):
    import torch
    n_sd = 3001
    rng = np.random.default_rng(3)
    vol = 10.0 ** rng.uniform(-19, -10, n_sd)
    xi = rng.integers(1, 2 ** 30, n_sd).astype(np.uint64)
    idx = rng.permutation(n_sd).astype(np.uint32)
    cid = np.zeros(n_sd, np.int32)
    cs = np.array([0, n_sd], np.uint32)
    flag = oracle.flag_pairs(cid, cs, idx, n_sd)
    T = _table(N, 4, 1.0)
    kp = [0.25, LO, N, M]
    ref = oracle.coalescence_kernel(flag, vol, idx, n_sd, oracle.KERNEL_TABULATED, kp, table=T)
    ref = oracle.times_max(ref, xi, flag, idx, n_sd)
    ref = oracle.normalize(ref, 1.5, np.array([7.0]), cid, cs, flag, idx, n_sd)
    ctx = sdm.Context(n_sd, 1, 1)
    T_dev = dev(T)
    q = torch.full((n_sd // 2,), -1.0, dtype=torch.float64, device="cuda")
    ctx.pair_rate(q, 1.5, dev(np.array([7.0])), dev(flag), dev(vol), dev(xi), dev(cid),
                  dev(cs), dev(idx), dev(np.array([n_sd], np.int64)),
                  sdm.kernel(oracle.KERNEL_TABULATED, kp, table=T_dev))
    torch.cuda.synchronize()
    assert np.array_equal(host(q), ref)
    ctx.close()


def test_tabulated_kernel_needs_a_valid_table(sdm):
    import ctypes
    lib = sdm.lib()
    ctx = sdm.Context(16, 1, 1)
    st = sdm.State(np.ones(16, np.uint64), np.ones((1, 16)), None, 1)
    for kp, table in (([1.0, LO, N, M], None), ([1.0, LO, 0, M], dev(np.ones(4))),
                      ([1.0, LO, N, 13], dev(np.ones(4))), ([1.0, -1, N, M], dev(np.ones(4)))):
        k = sdm.kernel(oracle.KERNEL_TABULATED, kp, table=table)
        with pytest.raises(sdm.SdmError):
            ctx.step(st, 1.0, k, sdm.rng(1, 0, 0), dv=1.0)
    ctx.close()
