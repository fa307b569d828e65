"""Throughput of the SDM coagulation step (and of its moment surrogate) on one
MI355X.  One JSON line per run.

Workloads (--workload, default box):

  box        the paper's Golovin box (arXiv:2101.06318, Sec. 4: dV = 1e6 m^3,
             N0 = 2^23 m^-3, exponential volumes with mean
             (4 pi/3)(30.531 um)^3, b = 1500 1/s, dt = 1 s), scaled to
             2^22 super-droplets (--log2-n-sd), synthetic, seed 2.  A step is
             one whole timestep (Steps 0-3 of the workflow figure) through the
             C ABI (sdm_step).
  grid       128 x 128 cells, Poisson(64) SDs per cell clipped to [2, 512],
             wet and dry volume attributes, gravitational kernel, random cell
             reassignment before every step (sdm_reassign + sdm_step).
  ensemble   1024 independent boxes of 2^8..2^16 SDs (log-uniform), Golovin
             and gravitational kernels alternating, advanced together
             (sdm_batch_step) with the autotuned schedule.
             --n-attr K adds K - 1 passive extensive attribute rows (chemistry
             as an extension, Sec. 5; 16 in the sub-results).
  golovin    the paper's validation run itself: the box with 2^13 SDs for
             3600 steps from its initial state, 16 seeds, each timed as graph
             replays of 1200 steps; mean moments at 1200, 2400 and 3600 s
             against the Golovin closed form (eq. 7 moments).
  surrogate  the moment surrogate's step for the 16384 cells of the grid
             (features, hull test, bf16 MFMA forward, moment update), beside
             one SDM step of the same grid (cell-steps/s of both).
  train      the surrogate's training step: a minibatch of 4096 samples
             through forward, MSE gradient, backward and Adam (samples/s).

With the box workload (the default) the line also carries `sub_results`:
every other workload measured in the same run, without oracle baselines.

W warm-up steps run first.  Then K steps are captured in one HIP graph,
replayed once untimed and five times timed, each bracketed by
synchronisation: the median replay gives value and ms_per_step (--eager:
the eager pass below instead).
A separate eager pass of K steps on one stream, where the library records
HIP events between its kernels, gives the per-kernel durations for the
roofline of the dominant kernel (eager_ms_per_step is that pass's wall
time).  The oracle (plain C, one host thread pinned to one core) is timed
on a bounded sample of the same workload (cpu_baseline); the ensemble also
reports one oracle process per host core (cpu_baseline_whole_host).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_SAMPLE = 67584.0      # 2 (5*128 + 128*128*2 + 128*3)


STEP_SOURCES = ("sdm_engine.hip", "sdm_device.h", "sdm_internal.h")


def source_hash():
    """Hash of the sources of the step's kernels (the fused step, its
    device helpers and plan layout); other files of the library do not
    change what the step's counters measure."""
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2101_06318_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(workload):
    """Counter-measured HBM bytes of one whole step (every kernel of the
    step: FETCH_SIZE and WRITE_SIZE, each scaled by what the counters read for
    a plain copy of known size), if profiles/ holds a record taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_step_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_step")


class HipEvent:
    """A HIP event created through the runtime the library uses; the
    library records it on the launch stream between its kernels."""

    def __init__(self, lib):
        import ctypes
        self._lib = lib
        h = ctypes.c_void_p()
        fn = lib.hipEventCreate
        fn.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        fn.restype = ctypes.c_int
        if fn(ctypes.byref(h)) != 0:
            raise RuntimeError("hipEventCreate failed")
        self.cuda_event = h.value

    def record(self, stream):
        import ctypes
        fn = self._lib.hipEventRecord
        fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        fn.restype = ctypes.c_int
        if fn(ctypes.c_void_p(self.cuda_event), ctypes.c_void_p(stream.cuda_stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self, other):
        import ctypes
        f = ctypes.c_float(0.0)
        fn = self._lib.hipEventElapsedTime
        fn.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        fn.restype = ctypes.c_int
        rc = fn(ctypes.byref(f), ctypes.c_void_p(self.cuda_event),
                ctypes.c_void_p(other.cuda_event))
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed (%d)" % rc)
        return float(f.value)

    def destroy(self):
        import ctypes
        fn = self._lib.hipEventDestroy
        fn.argtypes = [ctypes.c_void_p]
        fn(ctypes.c_void_p(self.cuda_event))


# Step kernels between the library's four event marks.
INTERVALS = ("k_tile+k_scan", "k_group", "k_finish")
# how the headline is timed (--eager: the event-marked eager pass instead)
GRAPH_REPLAYS = 5
TIMING = ("K steps captured in one HIP graph, median of 5 timed replays (value, ms_per_step); "
          "per-kernel durations from a separate eager pass of K steps with HIP events")
TIMING_EAGER = "K eager steps on one stream, HIP events between the kernels"


def algorithmic_bytes(pairs, f_coll, per_pair, per_pair_coll):
    """Algorithmic HBM bytes of one step: per pair, the state of two SDs
    read, their Index entries written and read back, and the write-back of
    a colliding pair times the collision fraction."""
    return pairs * (per_pair + per_pair_coll * f_coll)


def event_overhead_ms(torch, lib, stream, n=50):
    """Mean HIP-event interval around an empty kernel (torch's zero-cycle
    spin) on the stream: the dispatch and event cost that every marked
    interval carries besides its kernel's own duration."""
    ev = [(HipEvent(lib), HipEvent(lib)) for _ in range(n)]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for a, b in ev:
            a.record(stream)
            torch.cuda._sleep(0)
            b.record(stream)
    torch.cuda.synchronize()
    vals = sorted(a.elapsed_ms(b) for a, b in ev)
    for a, b in ev:
        a.destroy()
        b.destroy()
    return vals[len(vals) // 2]


def timed_steps(sdm, torch, run_step, K, lib):
    """K steps on one stream with the library's event marks; returns the total
    wall time (ms) and the mean duration of each marked interval, less the
    event interval around an empty kernel (the per-interval overhead)."""
    ev = [[HipEvent(lib) for _ in range(4)] for _ in range(K)]
    stream = torch.cuda.Stream()
    over = event_overhead_ms(torch, lib, stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        start.record(stream)
        for t in range(K):
            run_step(t, stream, ev[t])
        end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    per = {k: [] for k in INTERVALS}
    for t in range(K):
        for i, k in enumerate(INTERVALS):
            per[k].append(ev[t][i].elapsed_ms(ev[t][i + 1]))
    for row in ev:
        for e in row:
            e.destroy()
    kms = {k: max(sum(v) / len(v) - over, 0.0) for k, v in per.items()}
    kms["event_overhead_subtracted"] = over
    return total_ms, kms, stream


def graph_ms(torch, run_step, K, stream):
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(g, stream=stream):
                for t in range(K):
                    run_step(t, stream, None)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        times = []
        for _ in range(GRAPH_REPLAYS):
            gs = torch.cuda.Event(enable_timing=True)
            ge = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                gs.record(stream)
                g.replay()
                ge.record(stream)
            torch.cuda.synchronize()
            times.append(gs.elapsed_time(ge) / K)
        del g
        return sorted(times)[len(times) // 2]
    except Exception as e:  # reported, not fatal
        print("bench: graph replay not measured (%s)" % e, file=sys.stderr, flush=True)
        return None


def roofline(b_alg, kernel_ms, workload):
    """The dominant (longest) kernel against the step's algorithmic bytes,
    which one launch of it covers (it processes every pair of the step):
    achieved = B_alg / its mean duration.  traffic: counter bytes of the
    whole step, when measured on the current sources."""
    dom = max((k for k in kernel_ms if k in INTERVALS), key=kernel_ms.get)
    achieved = b_alg / (kernel_ms[dom] / 1e3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record(workload), "algorithmic_bytes": b_alg}


def step_roofline(b_alg, step_ms):
    gbs = b_alg / (step_ms / 1e3) / 1e9
    return {"bound": "hbm", "bytes_per_step": b_alg, "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def host_oracle(fn, seconds):
    """Runs fn(deadline) (the oracle on a bounded sample) pinned to one host
    core; returns (its result, the core, host description)."""
    from oracle.hostbench import host_info
    cpus = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {cpus[0]})
    try:
        res = fn(time.perf_counter() + seconds)
    finally:
        os.sched_setaffinity(0, set(cpus))
    return res, cpus[0], host_info()


def base_line(metric, value, unit, K, W, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# ---------------------------------------------------------------- workloads
def oracle_box_sample(np, w, seed, deadline, cell_id_fn=None, n_cell=1):
    """Whole oracle steps from the initial state until the deadline."""
    import oracle
    n = w["xi"].shape[0]
    s = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n, dtype=np.uint32), n_live=n)
    t0 = time.perf_counter()
    npairs = steps = 0
    while steps == 0 or time.perf_counter() < deadline:
        cid = cell_id_fn(steps) if cell_id_fn else None
        s = oracle.step(s["xi"], s["attr"], cid, n_cell, w["dv"], s["idx"], s["n_live"],
                        dt=w["dt"], kernel_id=w["kernel_id"], kparams=w["kparams"],
                        seed=seed, run=0, step=steps)
        npairs += int(s["counters"][oracle.CNT_PAIRS])
        steps += 1
    return npairs, steps, time.perf_counter() - t0


def first_step_parity(sdm, torch, np, ctx, w, k, steps=2):
    """Part of the oracle leg: the workload's first steps from its initial
    state on the GPU (fresh state, slot gammas kept) against the oracle,
    element by element; a gamma mismatch within 1e-12 of a threshold is a
    counted flip, any other difference fails the run."""
    import oracle
    from tests.parity import compare_step, slot_probabilities
    n = w["xi"].shape[0]
    st = sdm.State(w["xi"], w["attr"], None, 1, want_gamma=True)
    ref = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n, dtype=np.uint32), n_live=n)
    flips = 0
    for t in range(steps):
        prev = ref
        ctx.step(st, w["dt"], k, sdm.rng(2, 0, t), dv=w["dv"][0])
        ref = oracle.step(prev["xi"], prev["attr"], None, 1, w["dv"], prev["idx"],
                          prev["n_live"], dt=w["dt"], kernel_id=w["kernel_id"],
                          kparams=w["kparams"], seed=2, run=0, step=t, want_gamma=True)
        torch.cuda.synchronize()
        nl = int(st.n_live.item())
        got = dict(n_live=nl, xi=st.xi.cpu().numpy(), attr=st.attr.cpu().numpy(),
                   idx=st.idx.cpu().numpy().view(np.uint32), gamma=st.gamma_out.cpu().numpy())

        def pre(prev=prev, t=t):
            return slot_probabilities(prev["xi"], prev["attr"], None, 1, w["dv"], prev["idx"],
                                      prev["n_live"], dt=w["dt"], kernel_id=w["kernel_id"],
                                      kparams=w["kparams"], seed=2, run=0, step=t)
        f = compare_step(got, ref, pre, "step %d" % t)
        flips += f
        if f:
            ref = dict(ref, xi=got["xi"], attr=got["attr"])
    return {"steps": steps, "pairs_per_step": n // 2, "gamma_threshold_flips": flips,
            "result": "bit-exact" if flips == 0 else "bit-exact except flipped pairs",
            "against": "oracle (plain C, one thread)"}


def cpu_line(value, unit, seconds, core, host, sample):
    return {"value": value, "unit": unit, "cores": 1, "kind": "oracle",
            "seconds": round(seconds, 3), "pinned_core": core, "host": host, "sample": sample}


def bench_box(args, sdm, torch, np, workloads):
    n_sd = 1 << args.log2_n_sd
    w = workloads.box(n_sd, seed=2)
    n_attr = getattr(args, "n_attr", 1)
    if n_attr > 1:
        w = workloads.with_extra_attributes(w, n_attr)
    ctx = sdm.Context(n_sd, 1, n_attr)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(2, 0, 0, step_dev=step_dev)
    kw = dict(dv=w["dv"][0], step_advance=step_dev)
    for _ in range(args.warmup):
        ctx.step(st, w["dt"], k, r, **kw)
    torch.cuda.synchronize()
    c0 = st.counters.cpu().numpy().copy()

    def run_step(t, stream, ev):
        ctx.step(st, w["dt"], k, r, stream=stream, events=ev, **kw)

    K = args.steps
    total_ms, kms, stream = timed_steps(sdm, torch, run_step, K, sdm.lib())
    c1 = st.counters.cpu().numpy()
    gms = None if args.eager else graph_ms(torch, run_step, K, stream)
    pairs = int(c1[sdm.CNT_PAIRS] - c0[sdm.CNT_PAIRS]) // K
    f_coll = int(c1[sdm.CNT_COLLISIONS] - c0[sdm.CNT_COLLISIONS]) / max(pairs * K, 1)
    assert ctx.read_errors() == 0
    # per pair: xi and v of two SDs (32 B) read, their Index entries written
    # and read back (16 B); on a collision the other attribute rows of both
    # read (16 (n_attr - 1) B) and xi and every row of both written back
    # (16 + 16 n_attr B): 48 + 32 n_attr f_coll
    b_alg = algorithmic_bytes(pairs, f_coll, 48.0, 32.0 * n_attr)
    workload = "golovin_box_2_%d" % args.log2_n_sd
    if n_attr > 1:
        workload += "_%d_attributes" % n_attr
    step_ms = gms if gms else total_ms / K
    out = base_line("SDM pair-steps/s at n_sd=2^%d" % args.log2_n_sd +
                    (", %d attributes" % n_attr if n_attr > 1 else ""),
                    (n_sd // 2) / (step_ms / 1e3), "pair-steps/s", K, args.warmup,
                    step_ms, "f64",
                    {"workload": workload, "n_sd": n_sd, "n_attr": n_attr, "cells": 1,
                     "kernel": "golovin",
                     "b_per_s": w["b"], "dt_s": w["dt"], "dv_m3": float(w["dv"][0]), "seed": 2,
                     "timing": TIMING if gms else TIMING_EAGER,
                     "n_live": int(st.n_live.item()), "collision_fraction": f_coll})
    out["roofline"] = roofline(b_alg, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    out["step_roofline"] = step_roofline(b_alg, step_ms)
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["parity_check"] = first_step_parity(sdm, torch, np, ctx, w, k)
    ctx.close()
    if not args.no_cpu_baseline:
        (npairs, steps, dt), core, host = host_oracle(
            lambda dl: oracle_box_sample(np, w, 2, dl), args.cpu_seconds)
        out["cpu_baseline"] = cpu_line(
            npairs / dt, "pair-steps/s", dt, core, host,
            "the first %d steps of the 2^%d-SD Golovin box (seed 2) from its initial state, "
            "oracle (plain C, one thread pinned to one core, qsort-based shuffle)"
            % (steps, args.log2_n_sd))
    return out


def bench_grid(args, sdm, torch, np, workloads):
    w = workloads.grid(seed=3)
    n_sd, n_cell = w["n_sd"], w["n_cell"]
    ctx = sdm.Context(n_sd, n_cell, 2)
    st = sdm.State(w["xi"], w["attr"], w["cell_id"], n_cell)
    dv = torch.as_tensor(np.asarray(w["dv"], np.float64)).cuda()
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(3, 0, 0, step_dev=step_dev)

    def run_step(t, stream, ev):
        ctx.reassign(st.cell_id, n_sd, n_cell, r, stream=stream)
        ctx.step(st, w["dt"], k, r, stream=stream, events=ev, dv_per_cell=dv,
                 step_advance=step_dev)

    for t in range(args.warmup):
        run_step(t, None, None)
    torch.cuda.synchronize()
    c0 = st.counters.cpu().numpy().copy()
    K = args.steps
    total_ms, kms, stream = timed_steps(sdm, torch, run_step, K, sdm.lib())
    c1 = st.counters.cpu().numpy()
    gms = None if args.eager else graph_ms(torch, run_step, K, stream)
    pairs = int(c1[sdm.CNT_PAIRS] - c0[sdm.CNT_PAIRS]) / K
    f_coll = int(c1[sdm.CNT_COLLISIONS] - c0[sdm.CNT_COLLISIONS]) / max(pairs * K, 1)
    assert ctx.read_errors() == 0
    # per pair: xi, two attributes and the cell id of two SDs (56 B) read,
    # their Index entries written and read back (16 B); xi and both
    # attributes of two SDs written back on a collision (48 B): 72 + 48 f_coll
    b_alg = algorithmic_bytes(pairs, f_coll, 72.0, 48.0)
    workload = "grid_128x128"
    step_ms = gms if gms else total_ms / K
    out = base_line("SDM pair-steps/s on the 128x128 grid", pairs / (step_ms / 1e3),
                    "pair-steps/s", K, args.warmup, step_ms, "f64",
                    {"workload": workload, "n_sd": n_sd, "cells": n_cell, "kernel": "geometric",
                     "dt_s": w["dt"], "dv_m3": float(w["dv"][0]), "seed": 3,
                     "reassignment": "every step, inside the timed region",
                     "pairs_per_step": pairs, "collision_fraction": f_coll,
                     "timing": TIMING if gms else TIMING_EAGER})
    out["cell_steps_per_s"] = n_cell / (step_ms / 1e3)
    out["roofline"] = roofline(b_alg, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    out["step_roofline"] = step_roofline(b_alg, step_ms)
    out["cpu_baseline"] = None
    ctx.close()
    if not args.no_cpu_baseline:
        import oracle
        (npairs, steps, dt), core, host = host_oracle(
            lambda dl: oracle_box_sample(np, w, 3, dl,
                                         lambda t: oracle.reassign(n_sd, n_cell, 3, t),
                                         n_cell), args.cpu_seconds)
        out["cpu_baseline"] = cpu_line(npairs / dt, "pair-steps/s", dt, core, host,
                                       "%d reassignment + step passes of the full grid, "
                                       "oracle (plain C, one thread pinned to one core)" % steps)
    return out


def whole_host_ensemble(seconds):
    """One oracle process per usable host core (at most 16), each on its
    share of the 1024 runs; their pairs summed over the common wall time."""
    import subprocess
    P = min(16, len(os.sched_getaffinity(0)))
    procs = [subprocess.Popen([sys.executable, "-m", "oracle.hostbench", "--core", str(c),
                               "--of", str(P), "--seconds", str(seconds)],
                              cwd=ROOT, stdout=subprocess.PIPE, text=True) for c in range(P)]
    res = []
    for p in procs:
        o, _ = p.communicate(timeout=seconds + 300)
        if p.returncode != 0:
            raise RuntimeError("oracle host process failed")
        res.append(json.loads(o.strip().splitlines()[-1]))
    wall = max(r["seconds"] for r in res)
    return sum(r["pairs"] for r in res) / wall, P, wall


def bench_ensemble(args, sdm, torch, np, workloads):
    ens = workloads.ensemble(seed=4, n_runs=1024)
    xi, attr, segs = workloads.ensemble_layout(ens)
    st = sdm.State(xi, attr, None, len(segs))
    scratch = sdm.State(xi, attr, None, len(segs))
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    chosen = b.autotune(scratch, ens["dt"], sdm.rng(4, 0, 0), steps=5)
    del scratch
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(4, 0, 0, step_dev=step_dev)

    def run_step(t, stream, ev):
        b.step(st, ens["dt"], r, stream=stream, events=ev, step_advance=step_dev)

    def measure():
        for t in range(args.warmup):
            run_step(t, None, None)
        torch.cuda.synchronize()
        c0 = st.counters.cpu().numpy().copy()
        total_ms, kms, stream = timed_steps(sdm, torch, run_step, args.steps, sdm.lib())
        c1 = st.counters.cpu().numpy()
        gms = None if args.eager else graph_ms(torch, run_step, args.steps, stream)
        return total_ms, kms, gms, c0, c1

    # the schedule the library uses without tuning (0) and the autotuner's
    # choice, each timed here the same way; the line reports the faster
    # (the autotuner times eager steps on a scratch copy, and candidates are
    # often within a few per cent of each other) and both
    K = args.steps
    meas = {}
    for sch in ([0] if chosen == 0 else [0, chosen]):
        b.set_schedule(sch)
        total_ms, kms, gms, c0, c1 = measure()
        pairs = int(c1[sdm.CNT_PAIRS] - c0[sdm.CNT_PAIRS]) / K
        f_coll = int(c1[sdm.CNT_COLLISIONS] - c0[sdm.CNT_COLLISIONS]) / max(pairs * K, 1)
        step_ms = gms if gms else total_ms / K
        meas[sch] = dict(total_ms=total_ms, kms=kms, gms=gms, pairs=pairs, f_coll=f_coll,
                         step_ms=step_ms)
    assert ctx.read_errors() == 0
    best = min(meas, key=lambda k: meas[k]["step_ms"])
    m = meas[best]
    total_ms, kms, gms, pairs, f_coll, step_ms = (m["total_ms"], m["kms"], m["gms"], m["pairs"],
                                                  m["f_coll"], m["step_ms"])
    b_alg = algorithmic_bytes(pairs, f_coll, 48.0, 32.0)
    workload = "ensemble_1024"
    out = base_line("SDM pair-steps/s, 1024-run batched ensemble", pairs / (step_ms / 1e3),
                    "pair-steps/s", K, args.warmup, step_ms, "f64",
                    {"workload": workload, "runs": len(segs), "n_sd": int(sum(s[1] for s in segs)),
                     "kernels": "golovin (even runs), geometric (odd runs)", "dt_s": ens["dt"],
                     "seed": 4, "schedule": best, "autotuned_schedule": chosen,
                     "pairs_per_step": pairs, "collision_fraction": f_coll,
                     "timing": TIMING if gms else TIMING_EAGER})
    for key, sch in (("default_schedule", 0), ("autotuned_schedule", chosen)):
        out[key] = {"schedule": sch, "ms_per_step": meas[sch]["step_ms"],
                    "value": meas[sch]["pairs"] / (meas[sch]["step_ms"] / 1e3),
                    "kernel_ms": meas[sch]["kms"]}
    out["roofline"] = roofline(b_alg, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    out["step_roofline"] = step_roofline(b_alg, step_ms)
    out["cpu_baseline"] = None
    b.close()
    ctx.close()
    if not args.no_cpu_baseline:
        import oracle
        runs = ens["runs"]

        def sample(deadline):
            states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                           n_live=m["n_sd"]) for m in runs]
            t0 = time.perf_counter()
            npairs = done = 0
            while done == 0 or time.perf_counter() < deadline:
                r_ = done % len(runs)
                m, s = runs[r_], states[r_]
                s = oracle.step(s["xi"], s["attr"], None, 1, [m["dv"]], s["idx"], s["n_live"],
                                dt=ens["dt"], kernel_id=m["kernel_id"], kparams=m["kparams"],
                                seed=4, run=m["run"], step=done // len(runs))
                states[r_] = s
                npairs += int(s["counters"][oracle.CNT_PAIRS])
                done += 1
            return npairs, done, time.perf_counter() - t0

        (npairs, done, dt), core, host = host_oracle(sample, args.cpu_seconds)
        out["cpu_baseline"] = cpu_line(npairs / dt, "pair-steps/s", dt, core, host,
                                       "%d run-steps (the 1024 runs in turn, each from its "
                                       "initial state), oracle (plain C, one thread pinned to "
                                       "one core)" % done)
        v, P, wall = whole_host_ensemble(args.cpu_seconds)
        out["cpu_baseline_whole_host"] = {
            "value": v, "unit": "pair-steps/s", "cores": P, "kind": "oracle",
            "seconds": round(wall, 3),
            "sample": "%d oracle processes, one per host core, each on every %d-th run of the "
                      "1024 in turn from the initial states" % (P, P)}
    return out


def bench_shuffles(args, sdm, torch, np, workloads):
    """The per-cell permutation routines on the 128x128 grid (1.05e6 SDs in
    16384 cells): sort by random keys (sdm_shuffle_per_cell, the GPU strategy
    of Sec. 3.2), Fisher-Yates (one thread per cell) and MergeShuffle (one
    launch per level), each from a scrambled Index; SDs permuted per second."""
    w = workloads.grid(seed=3)
    n, n_cell = w["n_sd"], w["n_cell"]
    ctx = sdm.Context(n, n_cell, 1)
    idx0 = torch.as_tensor(np.random.default_rng(1).permutation(n).astype(np.int32)).cuda()
    idx = idx0.clone()
    cs = torch.zeros(n_cell + 1, dtype=torch.int32, device="cuda")
    nl = torch.tensor([n], dtype=torch.int64, device="cuda")
    cid = torch.as_tensor(w["cell_id"]).cuda()
    res = {}
    for name, method in (("sort_by_random_key", 0), ("fisher_yates", 1), ("merge_shuffle", 2)):
        def call(t):
            r = sdm.rng(3, 0, t)
            if method == 0:
                ctx.shuffle_per_cell(cs, idx, nl, None, cid, n_cell, r=r)
            else:
                ctx.shuffle_variant(method, cs, idx, nl, cid, n_cell, r)
        for t in range(3):
            call(t)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        K = min(args.steps, 20)
        e0.record()
        for t in range(K):
            call(t)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        res[name] = {"ms_per_call": ms, "sds_per_s": n / (ms / 1e3)}
    ctx.close()
    out = base_line("per-cell permutations on the 128x128 grid (SDs/s)",
                    res["fisher_yates"]["sds_per_s"], "SDs/s", min(args.steps, 20), 3,
                    res["fisher_yates"]["ms_per_call"], "u32",
                    {"workload": "shuffle_grid_128x128", "n_sd": n, "cells": n_cell,
                     "timing": "eager, CUDA events around K calls (cell sort included)"})
    out["methods"] = res
    out["roofline"] = None
    out["cpu_baseline"] = None
    return out


def golovin_moments(t, N0, b, vbar):
    """Moments of the additive-kernel solution from an exponential start
    (eq. 7): M0 = N0 (1 - tau), M1 = N0 vbar, M2 = 2 N0 vbar^2 / (1 - tau)^2,
    tau = 1 - exp(-N0 b vbar t)."""
    import math
    tau = 1.0 - math.exp(-N0 * b * vbar * t)
    return N0 * (1.0 - tau), N0 * vbar, 2.0 * N0 * vbar ** 2 / (1.0 - tau) ** 2


def golovin_run(sdm, torch, np, workloads, seed):
    """One 2^13-SD box (initial state and Philox seed `seed`) over 3600 s as
    three graph replays of 1200 steps; moments at 1200, 2400, 3600 s and the
    replay time."""
    n_sd = 1 << 13
    w = workloads.box(n_sd, seed=seed)
    ctx = sdm.Context(n_sd, 1, 1)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(seed, 0, 0, step_dev=step_dev)
    kw = dict(dv=w["dv"][0], step_advance=step_dev)
    ctx.prepare_step(st, w["dt"], k, r, **kw)
    stream = torch.cuda.Stream()
    seg = 1200
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            for _ in range(seg):
                ctx.step(st, w["dt"], k, r, stream=stream, **kw)
    torch.cuda.synchronize()
    # capture does not run the steps: reset the state and the step index
    st2 = sdm.State(w["xi"], w["attr"], None, 1)
    st.xi.copy_(st2.xi)
    st.attr.copy_(st2.attr)
    st.counters.zero_()
    step_dev.zero_()
    M = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    moms = []
    total_ms = 0.0
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            e0.record(stream)
            g.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        ctx.moments(M, st.xi, st.attr[0], st.idx, st.cell_start, 1, dv=w["dv"][0])
        torch.cuda.synchronize()
        moms.append(M.cpu().numpy()[0].copy())
    del g
    assert int(step_dev.item()) == 3 * seg and ctx.read_errors() == 0
    ctx.close()
    return w, np.array(moms), total_ms


def bench_golovin(args, sdm, torch, np, workloads):
    """The paper's validation run (Sec. 4): the Golovin box with 2^13 SDs over
    3600 s, 16 seeds; mean moments against the closed form of eq. (7).
    Timing is seed 1's three graph replays."""
    seeds = list(range(1, 17))
    runs = [golovin_run(sdm, torch, np, workloads, s) for s in seeds]
    w, _, total_ms = runs[0]
    n_sd = 1 << 13
    K = 3600
    M = np.stack([m for _, m, _ in runs])  # [seed][time][k]
    out_m = []
    ok = True
    for it, t_end in enumerate((1200, 2400, 3600)):
        ref = golovin_moments(float(t_end), w["N0"], w["b"], w["vbar"])
        row = {"t_s": t_end}
        for kk, name in ((0, "M0"), (1, "M1"), (2, "M2")):
            vals = M[:, it, kk] / ref[kk]
            mean = float(vals.mean())
            se = float(vals.std(ddof=1) / np.sqrt(len(seeds)))
            row[name + "_mean_rel_err"] = mean - 1.0
            row[name + "_std_err"] = se
            if kk != 1:
                ok = ok and abs(mean - 1.0) <= 3.0 * se + 0.01
        out_m.append(row)
    out = base_line("SDM pair-steps/s, 2^13-SD Golovin box over 3600 s",
                    (n_sd // 2) * K / (total_ms / 1e3), "pair-steps/s", K, 0, total_ms / K,
                    "f64", {"workload": "golovin_box_2_13_3600s", "n_sd": n_sd, "cells": 1,
                            "kernel": "golovin", "b_per_s": w["b"], "dt_s": w["dt"],
                            "seeds": "1-16 (timing: seed 1)",
                            "timing": "three graph replays of 1200 steps"})
    out["wall_s_3600_steps"] = total_ms / 1e3
    out["golovin_moments_16_seeds"] = out_m
    out["golovin_within_tolerance"] = ok
    out["golovin_tolerance"] = "|mean/closed form - 1| <= 3 standard errors + 1 % for M0 and M2"
    out["roofline"] = None
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        def sample(deadline):
            import oracle
            s_ = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32),
                      n_live=n_sd)
            t0 = time.perf_counter()
            npairs = steps = 0
            while (steps == 0 or time.perf_counter() < deadline) and steps < 3600:
                s_ = oracle.step(s_["xi"], s_["attr"], None, 1, w["dv"], s_["idx"],
                                 s_["n_live"], dt=w["dt"], kernel_id=w["kernel_id"],
                                 kparams=w["kparams"], seed=1, run=0, step=steps)
                npairs += int(s_["counters"][oracle.CNT_PAIRS])
                steps += 1
            return npairs, steps, time.perf_counter() - t0

        (npairs, steps, dt), core, host = host_oracle(sample, args.cpu_seconds)
        out["cpu_baseline"] = cpu_line(npairs / dt, "pair-steps/s", dt, core, host,
                                       "the first %d of the 3600 steps of seed 1, oracle "
                                       "(plain C, one thread pinned to one core)" % steps)
    return out


def bench_surrogate(args, sdm, torch, np, workloads):
    """The moment surrogate for steps of 10 s: trained (replica means of the
    particle method, the library's training kernels), judged against a
    4096-member particle-method mean of 64 held-out grid cells at 600 s
    (surrogate_gate), then its step (features, joint out-of-distribution
    test, bf16 MFMA forward, update) timed on the 16384 cells of the grid
    beside the particle method's step of the same grid (static cells)."""
    from paper_2101_06318_amd import surrogate
    m = 10
    t0 = time.perf_counter()
    ev, sur, sctx = surrogate.pipeline(torch, log=None, epochs=20, m=m)
    pipe_s = time.perf_counter() - t0
    w = workloads.grid(seed=3)
    n_sd, n_cell = w["n_sd"], w["n_cell"]
    ctx = sdm.Context(n_sd, n_cell, 2)
    st = sdm.State(w["xi"], w["attr"], w["cell_id"], n_cell)
    dv = torch.as_tensor(np.asarray(w["dv"], np.float64)).cuda()
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    ctx.cell_sort(st.cell_start, st.idx, st.n_live, st.cell_id, n_cell)
    M0 = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")
    ctx.moments(M0, st.xi, st.attr[0], st.idx, st.cell_start, n_cell, dv_per_cell=dv)
    M = M0.clone()
    bufs = sur.buffers(torch, n_cell)
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    lib = sdm.lib()
    e_fwd = [HipEvent(lib) for _ in range(2 * args.steps)]

    def sur_step(t, stream, ev_):
        # the steps below are sur.step's calls, with events around the forward pass
        c = sur.ctx
        c.mlp_features(bufs["x"], M, m * w["dt"], w["kernel_id"], sur.x_mean, sur.x_std,
                       stream=stream)
        c.ood_check(bufs["fb"], bufs["x"], sur.lo, sur.hi, sur.occ, sur.glo, sur.ginv,
                    counters=counters, stream=stream)
        if ev_ is not None:
            ev_[0].record(stream)
        c.mlp_forward(bufs["y"], bufs["x"], sur.net, stream=stream)
        if ev_ is not None:
            ev_[1].record(stream)
        c.mlp_apply(M, bufs["y"], m * w["dt"], sur.t_mean, sur.t_std, fallback=bufs["fb"],
                    stream=stream)

    for t in range(args.warmup):
        sur_step(t, None, None)
    K = args.steps
    stream = torch.cuda.Stream()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    M.copy_(M0)
    counters.zero_()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s0.record(stream)
        for t in range(K):
            sur_step(t, stream, e_fwd[2 * t:2 * t + 2])
        s1.record(stream)
    torch.cuda.synchronize()
    sur_ms = s0.elapsed_time(s1)
    ood_rows = int(counters[5].item())
    over = event_overhead_ms(torch, lib, stream)
    fwd_ms = max(sum(e_fwd[2 * t].elapsed_ms(e_fwd[2 * t + 1]) for t in range(K)) / K - over,
                 1e-6)
    for e in e_fwd:
        e.destroy()
    gms = None if args.eager else graph_ms(torch, sur_step, K, stream)

    # the particle method on the same cells (no reassignment)
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(3, 0, 1, step_dev=step_dev)

    def sdm_step(t, stream, ev_):
        ctx.step(st, w["dt"], k, r, stream=stream, events=ev_, dv_per_cell=dv,
                 step_advance=step_dev)

    for t in range(args.warmup):
        sdm_step(t, None, None)
    sdm_ms, _, sdm_stream = timed_steps(sdm, torch, sdm_step, K, lib)
    sdm_gms = None if args.eager else graph_ms(torch, sdm_step, K, sdm_stream)
    flop = MLP_FLOP_PER_SAMPLE * n_cell
    achieved = flop / (fwd_ms / 1e3) / 1e12
    step_ms = gms if gms else sur_ms / K
    sdm_step_ms = sdm_gms if (gms and sdm_gms) else sdm_ms / K
    out = base_line("surrogate cell-steps/s on the 128x128 grid", n_cell / (step_ms / 1e3),
                    "cell-steps/s", K, args.warmup, step_ms, "bf16",
                    {"workload": "surrogate_grid_128x128", "cells": n_cell,
                     "network": "5-128-128-128-3 GELU", "surrogate_step_s": m * w["dt"],
                     "sdm_dt_s": w["dt"], "seed": 3,
                     "step": "features + joint OOD test + forward + moment update",
                     "timing": TIMING if gms else TIMING_EAGER})
    out["sdm_cell_steps_per_s"] = n_cell / (sdm_step_ms / 1e3)
    out["speedup_vs_sdm"] = out["value"] / out["sdm_cell_steps_per_s"]
    # per simulated second: one surrogate step stands for m particle steps
    out["speedup_per_simulated_second"] = m * out["speedup_vs_sdm"]
    eq = ev.get("equivalent_members_m2")
    out["surrogate_gate"] = {
        "metric": "mean over 64 held-out cells of |M2_surrogate - M2_ref| / M2_ref at 600 s",
        "m2_err": ev["err_surrogate"][2], "limit": 0.05, "met": bool(ev["gate_m2_5pct"]),
        "m2_err_along_s": ev["err_m2_along"], "m0_err": ev["err_surrogate"][0],
        "reference": "%d-member particle-method mean" % ev["members"],
        "reference_m2_rel_se": ev["ref_rel_se"][2],
        "single_sdm_run_m2_err": ev["err_single_sdm"][2],
        "constant_tendency_m2_err": ev["err_constant_tendency"][2],
        "domain_m2_err": ev["domain_err_surrogate"][2],
        "equivalent_sdm_members_m2": eq,
        "speedup_vs_equivalent_sdm_ensemble": (None if eq is None else
                                               eq * out["speedup_per_simulated_second"]),
        "fallback_fraction": ev["fallback_fraction"], "train_samples": ev["train_samples"],
        "train_and_evaluate_s": round(pipe_s, 2)}
    out["ood_fallback_rows_in_timing"] = ood_rows
    out["roofline"] = {"bound": "mfma", "kernel": "k_mlp_forward_split", "achieved": achieved,
                       "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None}
    out["kernel_ms"] = {"k_mlp_forward_split": fwd_ms, "event_overhead_subtracted": over}
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = sur_ms / K
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        from oracle import mlp
        xh = bufs["x"].cpu().numpy()
        th = sur.net.params.cpu().numpy()

        def sample(deadline):
            net_o = mlp.Net("bf16")
            reps = 0
            t0_ = time.perf_counter()
            while reps == 0 or time.perf_counter() < deadline:
                net_o.forward(th, xh)
                reps += 1
            return reps, time.perf_counter() - t0_

        (reps, dt_), core, host = host_oracle(sample, args.cpu_seconds)
        out["cpu_baseline"] = cpu_line(n_cell * reps / dt_, "cell-steps/s", dt_, core, host,
                                       "%d bf16-emulated forward passes over the 16384 cells "
                                       "(numpy, one core)" % reps)
    ctx.close()
    sctx.close()
    return out


MLP_TRAIN_BATCH = 4096
MLP_BWD_FLOP_PER_SAMPLE = 133888.0  # dW of all four layers + dH of layers 4, 3, 2


def bench_train(args, sdm, torch, np, workloads):
    """Surrogate training: one step is one minibatch of 4096 samples through
    the forward pass (writing the training cache), the MSE gradient, the
    backward pass and Adam.  Synthetic standardised data: 2^20 samples (the
    size of one training set of cell-steps) with standard-normal inputs and
    targets, walked in order, a new batch every step.  Timed eagerly (Adam's
    step count is a host argument, so the steps are not graph-captured)."""
    n = 1 << 20
    B = MLP_TRAIN_BATCH
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    X = torch.randn((n, 5), generator=g, device="cuda")
    T = torch.randn((n, 3), generator=g, device="cuda")
    ctx = sdm.Context(1 << 12, 1 << 12, 2)
    net = sdm.Mlp(ctx, workloads.mlp_init(7))
    y = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
    dy = torch.zeros_like(y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cache = sdm.Mlp.cache_for(B)
    grad = torch.zeros(net.params.numel(), dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    nb = n // B
    lib = sdm.lib()

    def train_step(t, stream, ev):
        i = t % nb
        xb, tb = X[i * B:(i + 1) * B], T[i * B:(i + 1) * B]
        if ev is not None:
            ev[0].record(stream)
        ctx.mlp_forward(y, xb, net, cache=cache, stream=stream)
        ctx.mlp_mse(dy, loss, y, tb, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.mlp_backward(grad, dy, xb, cache, net, stream=stream)
        if ev is not None:
            ev[2].record(stream)
        ctx.mlp_adam(net, m, v, grad, t + 1, stream=stream)

    for t in range(args.warmup):
        train_step(t, None, None)
    K = args.steps
    ev = [[HipEvent(lib) for _ in range(3)] for _ in range(K)]
    stream = torch.cuda.Stream()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s0.record(stream)
        for t in range(K):
            train_step(args.warmup + t, stream, ev[t])
        s1.record(stream)
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / K
    fwd_ms = sum(e[0].elapsed_ms(e[1]) for e in ev) / K
    bwd_ms = sum(e[1].elapsed_ms(e[2]) for e in ev) / K
    for row in ev:
        for e in row:
            e.destroy()
    achieved = MLP_BWD_FLOP_PER_SAMPLE * B / (bwd_ms / 1e3) / 1e12
    out = base_line("surrogate training samples/s", B / (ms / 1e3), "samples/s", K,
                    args.warmup, ms, "bf16",
                    {"workload": "surrogate_train_batch_4096", "batch": B, "samples": n,
                     "network": "5-128-128-128-3 GELU", "optimizer": "Adam",
                     "step": "forward (with the training cache) + MSE gradient + backward + Adam",
                     "timing": TIMING_EAGER})
    out["roofline"] = {"bound": "mfma", "kernel": "k_mlp_backward+k_mlp_reduce", "achieved": achieved,
                       "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None}
    out["kernel_ms"] = {"k_mlp_forward+k_mlp_mse": fwd_ms, "k_mlp_backward+k_mlp_reduce": bwd_ms}
    out["flop_per_sample"] = MLP_FLOP_PER_SAMPLE + MLP_BWD_FLOP_PER_SAMPLE
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        from oracle import mlp
        xh, th_t = X[:B].cpu().numpy(), T[:B].cpu().numpy()
        th = workloads.mlp_init(7).astype(np.float64)
        mo = np.zeros_like(th)
        vo = np.zeros_like(th)
        net_o = mlp.Net("bf16")
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            yo, c = net_o.forward(th, xh)
            _, d = net_o.mse(yo, th_t)
            go = net_o.backward(th, c, d)
            th, mo, vo = mlp.adam(th, mo, vo, go, reps + 1)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": B * reps / dt, "unit": "samples/s", "cores": 1,
                               "kind": "oracle", "seconds": round(dt, 3),
                               "sample": "%d bf16-emulated training steps of 4096 samples "
                                         "(numpy forward, MSE, backward, Adam)" % reps}
    ctx.close()
    return out

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="box",
                    choices=["box", "grid", "ensemble", "golovin", "surrogate", "train",
                             "shuffles"])
    ap.add_argument("--log2-n-sd", type=int, default=22)
    ap.add_argument("--n-attr", type=int, default=1,
                    help="box: attribute rows per SD (row 0 the volume, the others passive "
                         "extensive attributes)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="host time given to the oracle baseline (whole steps, at least one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="skip the graph-replay measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-sub", action="store_true",
                    help="box workload: skip the other workloads' sub-results")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the SDM step runs and is measured on one MI355X only (no sharded "
              "path); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_06318_amd as sdm
    from paper_2101_06318_amd import workloads

    sdm.lib()  # raises if the HIP library is not built
    torch.cuda.set_device(0)
    print("bench: workload=%s warmup=%d steps=%d" % (args.workload, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    if args.calib_copy:
        # A copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale
        # the counters of the SDM kernels to bytes.
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fn = {"box": bench_box, "grid": bench_grid, "ensemble": bench_ensemble,
          "golovin": bench_golovin, "surrogate": bench_surrogate,
          "train": bench_train, "shuffles": bench_shuffles}[args.workload]
    out = fn(args, sdm, torch, np, workloads)
    if args.workload == "box" and not args.no_sub:
        out["sub_results"] = sub_results(args, sdm, torch, np, workloads)
    print(json.dumps(out), flush=True)


SUB_KEYS = ("metric", "value", "unit", "ms_per_step", "dtype", "config", "kernel_ms",
            "roofline", "step_roofline", "cell_steps_per_s", "sdm_cell_steps_per_s",
            "speedup_vs_sdm", "default_schedule", "autotuned_schedule", "golovin_moments_16_seeds",
            "golovin_within_tolerance", "golovin_tolerance", "wall_s_3600_steps",
            "surrogate_gate", "methods")


def sub_results(args, sdm, torch, np, workloads):
    """The other workloads, measured in the same run (no oracle baselines:
    `--workload X` gives each its own line with one)."""
    import copy
    res = {}
    def box16(a, *rest):
        a.n_attr = 16
        return bench_box(a, *rest)

    for name, fn in (("box_16_attributes", box16), ("grid", bench_grid),
                     ("ensemble", bench_ensemble),
                     ("golovin", bench_golovin), ("surrogate", bench_surrogate),
                     ("train", bench_train), ("shuffles", bench_shuffles)):
        a = copy.copy(args)
        a.no_cpu_baseline = True
        a.steps = min(args.steps, 100)
        t0 = time.perf_counter()
        try:
            o = fn(a, sdm, torch, np, workloads)
            res[name] = {k: o[k] for k in SUB_KEYS if k in o}
        except Exception as e:  # reported in the line, the headline stands
            res[name] = {"error": "%s: %s" % (type(e).__name__, e)}
        res[name]["wall_s"] = round(time.perf_counter() - t0, 2)
        print("bench: sub-result %s done (%.1f s)" % (name, res[name]["wall_s"]),
              file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
