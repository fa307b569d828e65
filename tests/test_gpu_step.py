"""GPU parity of the fused timestep (sdm_step) against the oracle's
routine-by-routine timestep (workflow figure of arXiv:2101.06318): bit-exact
multiplicities, attributes, permutation, live count, cell starts, slot
gammas and counters."""
import time

import numpy as np
import pytest

import oracle
from paper_2101_06318_amd import workloads
from tests.gpu_util import dev, host
from tests.parity import compare_step, slot_probabilities

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdm():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as m
    m.lib()
    return m


def _sync():
    import torch
    torch.cuda.synchronize()


def _gpu_result(st):
    n = int(host(st.n_live)[0])
    out = dict(n_live=n, xi=host(st.xi).copy(), attr=host(st.attr).copy(),
               idx=host(st.idx, np.uint32).copy(), cell_start=host(st.cell_start, np.uint32))
    if st.gamma_out is not None:
        out["gamma"] = host(st.gamma_out).copy()
    return out


def _check(st, ref, n_sd, what="", pre=None):
    """Element-by-element comparison of one step; gamma mismatches are
    classified (threshold flips are counted, anything else fails).  Returns
    the number of flips."""
    got = _gpu_result(st)
    flips = compare_step(got, ref, pre, what)
    assert np.array_equal(got["cell_start"], ref["cell_start"]), what
    return flips


def _run_pair(sdm, ctx, w, steps, seed, kparams=None, gamma=True, reassign=False, cell_id=None,
              dead=None, run=0, dv_scalar=False):
    n_sd = w["n_sd"]
    kp = kparams if kparams is not None else w["kparams"]
    xi = w["xi"].copy()
    if dead is not None:
        xi[dead] = 0
    cid = w["cell_id"] if cell_id is None else cell_id
    n_cell = w["n_cell"]
    st = sdm.State(xi, w["attr"], cid if n_cell > 1 else None, n_cell, want_gamma=gamma)
    dv = dev(np.asarray(w["dv"], np.float64))
    k = sdm.kernel(w["kernel_id"], kp)
    ref = dict(xi=xi, attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
    ref["n_live"] = n_sd
    cnt = np.zeros(8, np.uint64)
    cur_cid = cid
    total_flips = 0
    for t in range(steps):
        if reassign:
            cur_cid = oracle.reassign(n_sd, n_cell, seed, t)
            ctx.reassign(st.cell_id, n_sd, n_cell, sdm.rng(seed, 0, t))
        ctx.step(st, w["dt"], k, sdm.rng(seed, run, t), dv_per_cell=dv)
        prev = ref
        step_cid = cur_cid if n_cell > 1 else None
        ref = oracle.step(prev["xi"], prev["attr"], step_cid, n_cell, w["dv"],
                          prev["idx"], prev["n_live"], dt=w["dt"], kernel_id=w["kernel_id"],
                          kparams=kp, seed=seed, run=run, step=t, counters=cnt,
                          want_gamma=gamma)
        cnt = ref["counters"]
        _sync()

        def pre(prev=prev, step_cid=step_cid, t=t):
            return slot_probabilities(prev["xi"], prev["attr"], step_cid, n_cell, w["dv"],
                                      prev["idx"], prev["n_live"], dt=w["dt"],
                                      kernel_id=w["kernel_id"], kparams=kp, seed=seed,
                                      run=run, step=t)
        flips = _check(st, ref, n_sd, "step %d" % t, pre=pre)
        if flips:
            # a flipped pair: the trajectories continue from the GPU's state
            got = _gpu_result(st)
            ref = dict(ref, xi=got["xi"], attr=got["attr"])
            total_flips += flips
    if total_flips:
        print("gamma threshold flips: %d" % total_flips)
    else:
        assert np.array_equal(host(st.counters), cnt)
    return st, ref


@pytest.mark.parametrize("n_sd", [1, 2, 3, 64, 4095, 8192, 8192 + 131, 40000])
def test_step_single_cell(sdm, n_sd):
    w = workloads.box(n_sd, seed=n_sd)
    ctx = sdm.Context(n_sd, 1, 1)
    # kernel scaled up so collisions, gamma >= 2 and caps occur within a few steps
    _run_pair(sdm, ctx, w, 4, seed=3, kparams=[1500.0 * 300])
    ctx.close()


def test_step_with_dead_sds_and_removals(sdm):
    n_sd = 6000
    w = workloads.box(n_sd, seed=1)
    w["xi"] = np.random.default_rng(0).integers(1, 4, n_sd).astype(np.uint64)  # xi_k = 1 splits
    ctx = sdm.Context(n_sd, 1, 1)
    dead = np.random.default_rng(1).random(n_sd) < 0.2
    st, ref = _run_pair(sdm, ctx, w, 6, seed=9, kparams=[5.0e14], dead=dead)
    assert ref["counters"][oracle.CNT_ZEROED] > 0
    ctx.close()


@pytest.mark.parametrize("nx", [4, 32])
def test_step_grid_geometric_with_reassignment(sdm, nx):
    w = workloads.grid(seed=3, nx=nx, ny=nx)
    ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
    _run_pair(sdm, ctx, w, 3, seed=3, kparams=[50.0], reassign=True)
    ctx.close()


def test_full_size_grid_128x128_with_reassignment(sdm):
    """The 128 x 128 grid at full size (about 1.05e6 SDs, 16384 cells),
    reassigned before every step as in the benchmark, element by element."""
    w = workloads.grid(seed=3)
    ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
    _run_pair(sdm, ctx, w, 2, seed=3, reassign=True)
    ctx.close()


def test_step_grid_static_cells(sdm):
    w = workloads.grid(seed=5, nx=64, ny=64, mean_per_cell=20)
    ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
    _run_pair(sdm, ctx, w, 3, seed=5, kparams=[100.0])
    ctx.close()


@pytest.mark.parametrize("mean", [1500.0, 3000.0])
def test_step_grid_of_multi_bucket_cells(sdm, mean):
    """Cells of two or four buckets each, so that a group of about 3000 SDs
    holds whole cells (two cells of two buckets, or one of four) and sums
    its cells' bucket starts from the tiles' own offsets: two steps against
    the oracle, element by element (cell starts included)."""
    w = workloads.grid(seed=11, nx=8, ny=8, mean_per_cell=mean, n_max=4 * int(mean))
    ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
    _run_pair(sdm, ctx, w, 2, seed=11)
    ctx.close()


@pytest.mark.parametrize("caps", [(32, -1), (0, 64), (16, 40)])
def test_step_overflow_and_global_sort_paths(sdm, caps):
    """Tiny bucket regions / group capacities force the overflow list and the
    global-memory bitonic sort; the result must not change."""
    w = workloads.box(20000, seed=2)
    ctx = sdm.Context(20000, 1, 1)
    ctx.set_plan_limits(*caps)
    _run_pair(sdm, ctx, w, 3, seed=4, kparams=[1500.0 * 300])
    g = workloads.grid(seed=7, nx=8, ny=8)
    ctx2 = sdm.Context(g["n_sd"], g["n_cell"], 2)
    ctx2.set_plan_limits(*caps)
    _run_pair(sdm, ctx2, g, 2, seed=7, kparams=[50.0], reassign=True)
    ctx.close()
    ctx2.close()


def test_golovin_box_trajectory_bit_exact(sdm):
    """The paper's validation box at 2^13 SDs for 3600 steps (dt = 1 s)."""
    n_sd = 8192
    w = workloads.box(n_sd, seed=1)
    ctx = sdm.Context(n_sd, 1, 1)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    k = sdm.kernel(0, w["kparams"])
    for t in range(3600):
        ctx.step(st, 1.0, k, sdm.rng(1, 0, t), dv=w["dv"][0])
    _sync()
    ref = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
    for t in range(3600):
        ref = oracle.step(ref["xi"], ref["attr"], None, 1, w["dv"], ref["idx"], ref["n_live"],
                          dt=1.0, kernel_id=0, kparams=w["kparams"], seed=1, run=0, step=t)
    _check(st, ref, n_sd, "t=3600")
    ctx.close()


def test_full_size_box_2_22(sdm):
    """The throughput configuration (2^22 SDs) in the launch configuration
    the benchmark times: two whole steps against the oracle."""
    n_sd = 1 << 22
    w = workloads.box(n_sd, seed=2)
    ctx = sdm.Context(n_sd, 1, 1)
    t0 = time.time()
    _run_pair(sdm, ctx, w, 2, seed=2, gamma=True)
    print("2^22 parity: %.1f s" % (time.time() - t0))
    ctx.close()


def test_box_tiles_of_a_whole_number_of_rounds(sdm):
    """2^22 + 4098 SDs need 257 tiles of 16384 slots; the plan takes 512
    tiles of 8200 instead (two full rounds on the CUs, no one-tile tail):
    one step against the oracle, element by element."""
    n_sd = (1 << 22) + 4098
    w = workloads.box(n_sd, seed=8)
    ctx = sdm.Context(n_sd, 1, 1)
    _run_pair(sdm, ctx, w, 1, seed=8, gamma=True)
    ctx.close()


def test_graph_replay_matches_eager(sdm):
    import torch
    n_sd = 30000
    w = workloads.box(n_sd, seed=4)
    k = sdm.kernel(0, [1500.0 * 100])
    ctx = sdm.Context(n_sd, 1, 1)
    a = sdm.State(w["xi"], w["attr"], None, 1)
    b = sdm.State(w["xi"], w["attr"], None, 1)
    step_dev = dev(np.array([0], np.uint32))
    s = torch.cuda.Stream()
    ctx.prepare_step(b, 1.0, k, sdm.rng(4, 0, 0, step_dev=step_dev), dv=w["dv"][0])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.step(b, 1.0, k, sdm.rng(4, 0, 0, step_dev=step_dev), dv=w["dv"][0],
                     step_advance=step_dev, stream=s)
    _sync()
    for t in range(5):
        ctx.step(a, 1.0, k, sdm.rng(4, 0, t), dv=w["dv"][0])
        _sync()
        g.replay()
        _sync()
        for name in ("xi", "attr", "idx", "n_live", "cell_start"):
            assert np.array_equal(host(getattr(a, name)), host(getattr(b, name))), (t, name)
        assert int(host(step_dev)[0]) == t + 1
    ctx.close()


def test_small_launch_graph_replay_and_attributes(sdm):
    """Single-cell launches of at most 8192 slots run as one workgroup: its
    step under graph replay (device step counter advanced by the graph)
    equals the eager steps, and with four attribute rows, a per-cell volume
    array and gamma it matches the oracle element by element."""
    import torch
    n_sd = 8000
    w = workloads.box(n_sd, seed=14)
    k = sdm.kernel(0, [1500.0 * 100])
    ctx = sdm.Context(n_sd, 1, 1)
    a = sdm.State(w["xi"], w["attr"], None, 1)
    b = sdm.State(w["xi"], w["attr"], None, 1)
    step_dev = dev(np.array([0], np.uint32))
    s = torch.cuda.Stream()
    ctx.prepare_step(b, 1.0, k, sdm.rng(14, 0, 0, step_dev=step_dev), dv=w["dv"][0])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.step(b, 1.0, k, sdm.rng(14, 0, 0, step_dev=step_dev), dv=w["dv"][0],
                     step_advance=step_dev, stream=s)
    _sync()
    for t in range(5):
        ctx.step(a, 1.0, k, sdm.rng(14, 0, t), dv=w["dv"][0])
        _sync()
        g.replay()
        _sync()
        for name in ("xi", "attr", "idx", "n_live", "cell_start", "counters"):
            assert np.array_equal(host(getattr(a, name)), host(getattr(b, name))), (t, name)
        assert int(host(step_dev)[0]) == t + 1
    assert int(host(a.counters)[sdm.CNT_COLLISIONS]) > 0
    ctx.close()
    w4 = workloads.with_extra_attributes(workloads.box(5000, seed=15), 4)
    ctx4 = sdm.Context(5000, 1, 4)
    _run_pair(sdm, ctx4, w4, 3, seed=15, kparams=[1500.0 * 100], gamma=True)
    ctx4.close()


def test_run_twice_deterministic(sdm):
    import torch
    w = workloads.grid(seed=11, nx=16, ny=16)
    outs = []
    for _ in range(2):
        ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
        st = sdm.State(w["xi"], w["attr"], w["cell_id"], w["n_cell"])
        for t in range(5):
            ctx.step(st, 1.0, sdm.kernel(1, [50.0]), sdm.rng(11, 0, t), dv_per_cell=dev(w["dv"]))
        _sync()
        outs.append((host(st.xi).copy(), host(st.attr).copy(), host(st.idx).copy()))
        ctx.close()
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_bad_cell_id_is_reported(sdm):
    w = workloads.grid(seed=1, nx=4, ny=4)
    cid = w["cell_id"].copy()
    cid[5] = w["n_cell"] + 3
    ctx = sdm.Context(w["n_sd"], w["n_cell"], 2)
    st = sdm.State(w["xi"], w["attr"], cid, w["n_cell"])
    ctx.step(st, 1.0, sdm.kernel(1, [1.0]), sdm.rng(1, 0, 0), dv_per_cell=dev(w["dv"]))
    assert ctx.read_errors() & 1
    assert int(host(st.n_live)[0]) == w["n_sd"] - 1
    ctx.close()


def test_checkpoint_resume_equals_uninterrupted(sdm):
    """The step's state is (xi, attributes, cell ids) plus the step index:
    copying it to the host after step 3 and resuming in a fresh context
    gives the uninterrupted trajectory bit for bit."""
    w = workloads.grid(seed=13, nx=16, ny=16)
    n_sd, n_cell = w["n_sd"], w["n_cell"]
    dv = dev(np.asarray(w["dv"], np.float64))
    k = sdm.kernel(w["kernel_id"], [80.0])

    def run(st, ctx, t0, t1):
        for t in range(t0, t1):
            ctx.reassign(st.cell_id, n_sd, n_cell, sdm.rng(21, 0, t))
            ctx.step(st, w["dt"], k, sdm.rng(21, 0, t), dv_per_cell=dv)

    ctx = sdm.Context(n_sd, n_cell, 2)
    a = sdm.State(w["xi"], w["attr"], w["cell_id"], n_cell)
    run(a, ctx, 0, 6)
    b = sdm.State(w["xi"], w["attr"], w["cell_id"], n_cell)
    run(b, ctx, 0, 3)
    _sync()
    saved = (host(b.xi).copy(), host(b.attr).copy(), host(b.cell_id).copy())
    ctx.close()
    ctx2 = sdm.Context(n_sd, n_cell, 2)
    c = sdm.State(*saved, n_cell)
    run(c, ctx2, 3, 6)
    _sync()
    for name in ("xi", "attr", "idx", "cell_start", "n_live"):
        assert np.array_equal(host(getattr(a, name)), host(getattr(c, name))), name
    ctx2.close()


def test_empty_and_all_dead_states(sdm):
    """No SDs at all, and SDs that are all dead (xi = 0): the step succeeds
    with no live SDs, empty cells and no pairs, as the oracle says."""
    import torch
    ctx = sdm.Context(128, 4, 1)
    st = sdm.State(np.zeros(0, np.uint64), np.zeros((1, 0)), None, 1)
    ctx.step(st, 1.0, sdm.kernel(0, [1500.0]), sdm.rng(1, 0, 0), dv=1e6)
    _sync()
    assert int(host(st.n_live)[0]) == 0
    assert np.array_equal(host(st.cell_start), [0, 0])
    w = workloads.grid(seed=2, nx=2, ny=2)
    xi = np.zeros(w["n_sd"], np.uint64)
    ctx2 = sdm.Context(w["n_sd"], w["n_cell"], 2)
    _run_pair(sdm, ctx2, dict(w, xi=xi), 2, seed=5)
    ctx.close()
    ctx2.close()


def test_largest_single_plan_and_the_limit(sdm):
    """2^25 SDs in one cell (the most one plan takes: 2048 tiles of 16384
    slots), one step element by element against the oracle; one slot pair
    more is refused with a clean error, not a fault."""
    n_sd = 1 << 25
    w = workloads.box(n_sd, seed=6)
    ctx = sdm.Context(n_sd + 2, 1, 1)
    _run_pair(sdm, ctx, w, 1, seed=6, gamma=False)
    big = workloads.box(n_sd + 2, seed=6)
    st = sdm.State(big["xi"], big["attr"], None, 1)
    with pytest.raises(sdm.SdmError):
        ctx.step(st, 1.0, sdm.kernel(0, [1500.0]), sdm.rng(6, 0, 0), dv=1e6)
    ctx.close()


def test_cell_beyond_2_16_records_in_a_multi_cell_plan(sdm):
    """A 256-cell plan sized for about 300 SDs per cell, with 70 000 of the
    SDs in one cell: that cell's single bucket holds more than 2^16 records,
    so its group is sorted in global memory and its opener positions need
    all 32 bits.  Two steps against the oracle, element by element."""
    n_sd, n_cell, big = 78000, 256, 70000
    w = workloads.box(n_sd, seed=12)
    cid = np.random.default_rng(12).integers(0, n_cell, n_sd).astype(np.int32)
    cid[np.random.default_rng(13).permutation(n_sd)[:big]] = 37
    w = dict(w, n_cell=n_cell, cell_id=cid, dv=np.full(n_cell, w["dv"][0] / n_cell))
    ctx = sdm.Context(n_sd, n_cell, 1)
    _run_pair(sdm, ctx, w, 2, seed=12, kparams=[1500.0 * 50])
    ctx.close()
