"""GPU parity with many attributes per SD: the update of eqs. (4)-(6)
applies to every extensive attribute (Sec. 2.2; attributes stored as a 2-D
row-major array, Sec. 3.1; chemistry named as an extension, Sec. 5).
Bit-exact multiplicities, every attribute row, permutation and gammas against
the oracle over whole fused timesteps."""
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


def _steps(sdm, w, steps, kp, seed, reassign=False):
    import torch
    n_sd, n_cell, n_attr = w["n_sd"], w["n_cell"], w["attr"].shape[0]
    cid = w["cell_id"] if n_cell > 1 else None
    st = sdm.State(w["xi"], w["attr"], cid, n_cell, want_gamma=True)
    ctx = sdm.Context(n_sd, n_cell, n_attr)
    k = sdm.kernel(w["kernel_id"], kp)
    dvs = np.broadcast_to(np.asarray(w["dv"], np.float64), (n_cell,)).copy()
    d_dv = dev(dvs)
    ref = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
    cnt = np.zeros(8, np.uint64)
    for t in range(steps):
        if reassign:
            cid = oracle.reassign(n_sd, n_cell, seed, t)
            ctx.reassign(st.cell_id, n_sd, n_cell, sdm.rng(seed, 0, t))
        ctx.step(st, w["dt"], k, sdm.rng(seed, 0, t), dv_per_cell=d_dv)
        ref = oracle.step(ref["xi"], ref["attr"], cid, n_cell, dvs, ref["idx"], ref["n_live"],
                          dt=w["dt"], kernel_id=w["kernel_id"], kparams=kp, seed=seed, run=0,
                          step=t, counters=cnt, want_gamma=True)
        cnt = ref["counters"]
        torch.cuda.synchronize()
        n = int(host(st.n_live)[0])
        assert n == ref["n_live"], t
        assert np.array_equal(host(st.xi), ref["xi"]), t
        got = host(st.attr)
        for r in range(n_attr):
            assert np.array_equal(got[r], ref["attr"][r]), (t, r)
        assert np.array_equal(host(st.idx, np.uint32)[:n], ref["idx"][:n]), t
        assert np.array_equal(host(st.gamma_out), ref["gamma"]), t
    assert np.array_equal(host(st.counters), cnt)
    assert cnt[oracle.CNT_COLLISIONS] > 100
    ctx.close()
    return cnt


@pytest.mark.parametrize("n_attr", [2, 8, 16])
def test_box_many_attributes(sdm, n_attr):
    w = workloads.with_extra_attributes(workloads.box(30001, seed=n_attr), n_attr)
    _steps(sdm, w, 4, [1500.0 * 200], seed=7)


def test_grid_eight_attributes_with_reassignment(sdm):
    w = workloads.with_extra_attributes(workloads.grid(seed=5, nx=16, ny=16), 8)
    _steps(sdm, w, 3, [50.0], seed=8, reassign=True)


def test_attribute_rows_conserve_their_totals(sdm):
    """Every extensive attribute's total sum(xi A) is conserved by eqs.
    (5)-(6) up to rounding: checked on the GPU state after 10 steps."""
    import torch
    n_attr = 12
    w = workloads.with_extra_attributes(workloads.box(20000, seed=3), n_attr)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    ctx = sdm.Context(w["n_sd"], 1, n_attr)
    k = sdm.kernel(w["kernel_id"], [1500.0 * 300])
    tot0 = (w["xi"].astype(np.float64)[None, :] * w["attr"]).sum(1)
    for t in range(10):
        ctx.step(st, w["dt"], k, sdm.rng(4, 0, t), dv=w["dv"][0])
    torch.cuda.synchronize()
    xi, A = host(st.xi).astype(np.float64), host(st.attr)
    tot = (xi[None, :] * A).sum(1)
    assert np.all(np.abs(tot / tot0 - 1) < 1e-12), tot / tot0 - 1
    assert int(host(st.counters)[oracle.CNT_COLLISIONS]) > 1000
    ctx.close()
