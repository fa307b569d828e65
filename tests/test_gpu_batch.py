"""Batched ensemble (sdm_batch_*): every member advanced in one launch
sequence must equal (bit for bit) the same member run alone, which must equal
the oracle's single-run timestep with that run id; the result must not depend
on the block/segment schedule; graph replay equals eager execution."""
import os

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


def _sync():
    import torch
    torch.cuda.synchronize()


SMALL_SIZES = [1, 2, 3, 7, 64, 255, 256, 1000, 2049, 4097, 9000, 0, 300, 17, 5000, 12000, 2]


def _small_ensemble(scale=300.0):
    ens = workloads.ensemble(seed=5, n_runs=len(SMALL_SIZES), n_sd_override=SMALL_SIZES)
    for m in ens["runs"]:  # scaled kernels: collisions, gamma >= 2 and caps occur
        m["kparams"] = [m["kparams"][0] * scale, 0.0, 0.0, 0.0]
    return ens


def _batch_state(sdm, ens, want_gamma=True):
    xi, attr, segs = workloads.ensemble_layout(ens)
    st = sdm.State(xi, attr, None, len(segs), want_gamma=want_gamma)
    return st, segs


def _oracle_members(ens, states, seed, t):
    out = []
    for m, s in zip(ens["runs"], states):
        n = m["n_sd"]
        out.append(oracle.step(s["xi"], s["attr"], None, 1, [m["dv"]], s["idx"], s["n_live"],
                               dt=ens["dt"], kernel_id=m["kernel_id"], kparams=m["kparams"],
                               seed=seed, run=m["run"], step=t, want_gamma=True))
    return out


def _check_members(st, segs, refs, what):
    xi, attr = host(st.xi), host(st.attr)
    idx, cs = host(st.idx, np.uint32), host(st.cell_start, np.uint32)
    gam = host(st.gamma_out) if st.gamma_out is not None else None
    total = 0
    for r, ((off, n, *_), ref) in enumerate(zip(segs, refs)):
        assert np.array_equal(xi[off:off + n], ref["xi"]), (what, r)
        assert np.array_equal(attr[:, off:off + n], ref["attr"]), (what, r)
        nl = ref["n_live"]
        assert int(cs[r]) == total, (what, r)
        assert np.array_equal(idx[cs[r]:cs[r] + nl] - off, ref["idx"][:nl]), (what, r)
        if gam is not None:
            assert np.array_equal(gam[off // 2: off // 2 + n // 2], ref["gamma"]), (what, r)
        total += nl
    assert int(host(st.n_live)[0]) == total
    assert int(cs[len(segs)]) == total


def test_batch_matches_oracle_per_member(sdm):
    ens = _small_ensemble()
    st, segs = _batch_state(sdm, ens)
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                   n_live=m["n_sd"]) for m in ens["runs"]]
    cnt = np.zeros(8, np.uint64)
    for t in range(4):
        b.step(st, 1.0, sdm.rng(8, 0, t))
        states = _oracle_members(ens, states, 8, t)
        for s in states:
            cnt += s["counters"]
        _sync()
        _check_members(st, segs, states, "step %d" % t)
    assert np.array_equal(host(st.counters), cnt)
    assert cnt[oracle.CNT_COLLISIONS] > 0 and cnt[oracle.CNT_GAMMA_GE2] > 0
    b.close()
    ctx.close()


def test_batch_equals_members_run_alone(sdm):
    ens = _small_ensemble()
    st, segs = _batch_state(sdm, ens)
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    for t in range(3):
        b.step(st, 1.0, sdm.rng(9, 0, t))
    _sync()
    xi, attr = host(st.xi), host(st.attr)
    for m, (off, n, dv, kid, kp, run) in zip(ens["runs"], segs):
        c1 = sdm.Context(max(n, 1), 1, 1)
        s1 = sdm.State(m["xi"], m["attr"], None, 1)
        for t in range(3):
            c1.step(s1, 1.0, sdm.kernel(kid, kp), sdm.rng(9, run, t), dv=dv)
        _sync()
        assert np.array_equal(host(s1.xi), xi[off:off + n]), run
        assert np.array_equal(host(s1.attr), attr[:, off:off + n]), run
        c1.close()
    b.close()
    ctx.close()


def test_every_schedule_gives_the_same_result(sdm):
    ens = _small_ensemble()
    outs = []
    ctx = None
    n_sched = 1
    sched = 0
    while sched < n_sched:
        st, segs = _batch_state(sdm, ens)
        if ctx is None:
            ctx = sdm.Context(st.n_sd, len(segs), 1)
        b = sdm.Batch(ctx, segs)
        n_sched = b.n_schedules()
        b.set_schedule(sched)
        sched += 1
        for t in range(3):
            b.step(st, 1.0, sdm.rng(10, 0, t))
        _sync()
        outs.append((host(st.xi).copy(), host(st.attr).copy(), host(st.idx).copy(),
                     host(st.gamma_out).copy()))
        b.close()
    assert len(outs) >= 12
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)
    ctx.close()


def test_autotune_and_cache(sdm, tmp_path):
    ens = _small_ensemble()
    st, segs = _batch_state(sdm, ens)
    scratch, _ = _batch_state(sdm, ens, want_gamma=False)
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    cache = str(tmp_path / "sched.txt")
    chosen = b.autotune(scratch, 1.0, sdm.rng(11, 0, 0), steps=2, cache_path=cache)
    assert 0 <= chosen < b.n_schedules()
    assert os.path.exists(cache) and open(cache).read().strip()
    b2 = sdm.Batch(ctx, segs)
    assert b2.autotune(scratch, 1.0, sdm.rng(11, 0, 0), steps=2, cache_path=cache) == chosen
    # the tuned batch still matches the oracle
    states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                   n_live=m["n_sd"]) for m in ens["runs"]]
    b.step(st, 1.0, sdm.rng(12, 0, 0))
    states = _oracle_members(ens, states, 12, 0)
    _sync()
    _check_members(st, segs, states, "tuned")
    b.close()
    b2.close()
    ctx.close()


def test_batch_graph_replay_matches_eager(sdm):
    import torch
    ens = _small_ensemble()
    a, segs = _batch_state(sdm, ens, want_gamma=False)
    g_st, _ = _batch_state(sdm, ens, want_gamma=False)
    ctx = sdm.Context(a.n_sd, len(segs), 1)
    ba = sdm.Batch(ctx, segs)
    bg = sdm.Batch(ctx, segs)
    step_dev = dev(np.array([0], np.uint32))
    s = torch.cuda.Stream()
    bg.step(g_st, 1.0, sdm.rng(13, 0, 0, step_dev=step_dev), step_advance=step_dev)
    ba.step(a, 1.0, sdm.rng(13, 0, 0))
    _sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            bg.step(g_st, 1.0, sdm.rng(13, 0, 0, step_dev=step_dev), step_advance=step_dev,
                    stream=s)
    _sync()
    for t in range(1, 5):
        ba.step(a, 1.0, sdm.rng(13, 0, t))
        _sync()
        graph.replay()
        _sync()
        for name in ("xi", "attr", "idx", "n_live", "cell_start"):
            assert np.array_equal(host(getattr(a, name)), host(getattr(g_st, name))), (t, name)
    ba.close()
    bg.close()
    ctx.close()


def test_full_size_ensemble_one_step(sdm):
    """1024 members, sizes log-uniform in 2^8..2^16 (about 1.2e7 SDs), mixed
    Golovin / geometric kernels: one batched step against the oracle."""
    ens = workloads.ensemble(seed=4, n_runs=1024)
    st, segs = _batch_state(sdm, ens)
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    b.step(st, 1.0, sdm.rng(4, 0, 0))
    states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                   n_live=m["n_sd"]) for m in ens["runs"]]
    states = _oracle_members(ens, states, 4, 0)
    _sync()
    _check_members(st, segs, states, "full")
    b.close()
    ctx.close()
