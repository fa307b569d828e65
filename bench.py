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
  golovin    the paper's validation run itself: the box with 2^13 SDs (seed 1)
             for 3600 steps from its initial state, timed as graph replays of
             1200 steps; moments at 1200, 2400 and 3600 s against the Golovin
             closed form (eq. 7 moments).
  surrogate  the moment surrogate's step for the 16384 cells of the grid
             (features, hull test, bf16 MFMA forward, moment update), beside
             one SDM step of the same grid (cell-steps/s of both).
  train      the surrogate's training step: a minibatch of 4096 samples
             through forward, MSE gradient, backward and Adam (samples/s).

W warm-up steps run first.  Then K steps are captured in one HIP graph,
replayed once untimed and five times timed, each bracketed by
synchronisation: the median replay gives value and ms_per_step (--eager:
the eager pass below instead).
A separate eager pass of K steps on one stream, where the library records
HIP events between its kernels, gives the per-kernel durations for the
roofline of the dominant kernel (eager_ms_per_step is that pass's wall
time).  The oracle (plain C, one host thread) is timed on a bounded sample
of the same workload (cpu_baseline).
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


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2101_06318_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_record(kernel, workload):
    """Counter-measured bytes per launch, if profiles/ holds a record taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


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


def algorithmic_bytes(pairs, f_coll, per_pair_read, per_pair_write_idx, per_pair_coll):
    """Algorithmic HBM bytes of one step, split per kernel: per pair, the
    state of two SDs read and the Index read (charged to the tile kernel),
    the Index written and the write-back of a colliding pair (charged to
    the group kernel, times the collision fraction)."""
    return {"step": pairs * (per_pair_read + per_pair_write_idx + per_pair_coll * f_coll),
            "k_tile+k_scan": pairs * per_pair_read,
            "k_group": pairs * (per_pair_write_idx + per_pair_coll * f_coll),
            "k_finish": 0.0}


def timed_steps(sdm, torch, run_step, K, lib):
    """K steps on one stream with the library's event marks; returns the total
    wall time (ms) and the mean duration of each marked interval."""
    ev = [[HipEvent(lib) for _ in range(4)] for _ in range(K)]
    stream = torch.cuda.Stream()
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
    return total_ms, {k: sum(v) / len(v) for k, v in per.items()}, stream


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


def roofline(ab, kernel_ms, workload):
    dom = max(kernel_ms, key=kernel_ms.get)
    achieved = ab[dom] / (kernel_ms[dom] / 1e3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record(dom, workload)}


def base_line(metric, value, unit, K, W, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# ---------------------------------------------------------------- workloads
def bench_box(args, sdm, torch, np, workloads):
    n_sd = 1 << args.log2_n_sd
    w = workloads.box(n_sd, seed=2)
    ctx = sdm.Context(n_sd, 1, 1)
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
    # per pair: xi and v of two SDs (32 B) and their Index entries (8 B)
    # read, Index written (8 B), xi and v of both written back on a
    # collision (32 B): 48 + 32 f_coll
    ab = algorithmic_bytes(pairs, f_coll, 40.0, 8.0, 32.0)
    workload = "golovin_box_2_%d" % args.log2_n_sd
    step_ms = gms if gms else total_ms / K
    out = base_line("SDM pair-steps/s at n_sd=2^%d" % args.log2_n_sd,
                    (n_sd // 2) / (step_ms / 1e3), "pair-steps/s", K, args.warmup,
                    step_ms, "f64",
                    {"workload": workload, "n_sd": n_sd, "cells": 1, "kernel": "golovin",
                     "b_per_s": w["b"], "dt_s": w["dt"], "dv_m3": float(w["dv"][0]), "seed": 2,
                     "timing": TIMING if gms else TIMING_EAGER,
                     "n_live": int(st.n_live.item()), "collision_fraction": f_coll})
    out["roofline"] = roofline(ab, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    step_gbs = ab["step"] / (step_ms / 1e3) / 1e9
    out["step_roofline"] = {"bound": "hbm", "bytes_per_step": ab["step"], "achieved": step_gbs,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": step_gbs / HBM_PEAK_GBS}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        n = n_sd
        s = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n, dtype=np.uint32), n_live=n)
        t0 = time.perf_counter()
        npairs = steps = 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            s = oracle.step(s["xi"], s["attr"], None, 1, w["dv"], s["idx"], s["n_live"],
                            dt=w["dt"], kernel_id=w["kernel_id"], kparams=w["kparams"],
                            seed=2, run=0, step=steps)
            npairs += int(s["counters"][oracle.CNT_PAIRS])
            steps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": npairs / dt, "unit": "pair-steps/s", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": "the first %d steps of the 2^%d-SD Golovin box (seed 2) from its initial "
                      "state, oracle (plain C, one thread, qsort-based shuffle)"
                      % (steps, args.log2_n_sd)}
    ctx.close()
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
    reass_ms = []

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
    # per pair: xi, two attributes and the cell id of two SDs (56 B) and
    # their Index entries (8 B) read, Index written (8 B), xi and both
    # attributes of two SDs written back on a collision (48 B): 72 + 48 f_coll
    ab = algorithmic_bytes(pairs, f_coll, 64.0, 8.0, 48.0)
    workload = "grid_128x128"
    step_ms = gms if gms else total_ms / K
    out = base_line("SDM pair-steps/s on the 128x128 grid", pairs / (step_ms / 1e3),
                    "pair-steps/s", K, args.warmup, step_ms, "f64",
                    {"workload": workload, "n_sd": n_sd, "cells": n_cell, "kernel": "geometric",
                     "dt_s": w["dt"], "dv_m3": float(w["dv"][0]), "seed": 3,
                     "reassignment": "every step, inside the timed region",
                     "pairs_per_step": pairs, "collision_fraction": f_coll, "timing": TIMING if gms else TIMING_EAGER})
    out["cell_steps_per_s"] = n_cell / (step_ms / 1e3)
    out["roofline"] = roofline(ab, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        s = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
        t0 = time.perf_counter()
        npairs = steps = 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            cid = oracle.reassign(n_sd, n_cell, 3, steps)
            s = oracle.step(s["xi"], s["attr"], cid, n_cell, w["dv"], s["idx"], s["n_live"],
                            dt=w["dt"], kernel_id=w["kernel_id"], kparams=w["kparams"], seed=3,
                            run=0, step=steps)
            npairs += int(s["counters"][oracle.CNT_PAIRS])
            steps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": npairs / dt, "unit": "pair-steps/s", "cores": 1,
                               "kind": "oracle", "seconds": round(dt, 3),
                               "sample": "%d reassignment + step passes of the full grid, "
                                         "oracle (plain C, one thread)" % steps}
    ctx.close()
    return out


def bench_ensemble(args, sdm, torch, np, workloads):
    ens = workloads.ensemble(seed=4, n_runs=1024)
    xi, attr, segs = workloads.ensemble_layout(ens)
    st = sdm.State(xi, attr, None, len(segs))
    scratch = sdm.State(xi, attr, None, len(segs))
    ctx = sdm.Context(st.n_sd, len(segs), 1)
    b = sdm.Batch(ctx, segs)
    chosen = b.autotune(scratch, ens["dt"], sdm.rng(4, 0, 0), steps=3)
    del scratch
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(4, 0, 0, step_dev=step_dev)

    def run_step(t, stream, ev):
        b.step(st, ens["dt"], r, stream=stream, events=ev, step_advance=step_dev)

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
    ab = algorithmic_bytes(pairs, f_coll, 40.0, 8.0, 32.0)
    workload = "ensemble_1024"
    step_ms = gms if gms else total_ms / K
    out = base_line("SDM pair-steps/s, 1024-run batched ensemble", pairs / (step_ms / 1e3),
                    "pair-steps/s", K, args.warmup, step_ms, "f64",
                    {"workload": workload, "runs": len(segs), "n_sd": int(sum(s[1] for s in segs)),
                     "kernels": "golovin (even runs), geometric (odd runs)", "dt_s": ens["dt"],
                     "seed": 4, "schedule": chosen, "pairs_per_step": pairs,
                     "collision_fraction": f_coll, "timing": TIMING if gms else TIMING_EAGER})
    out["roofline"] = roofline(ab, kms, workload)
    out["kernel_ms"] = kms
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = total_ms / K
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        runs = ens["runs"]
        states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                       n_live=m["n_sd"]) for m in runs]
        t0 = time.perf_counter()
        npairs = done = 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            r_ = done % len(runs)
            m, s = runs[r_], states[r_]
            s = oracle.step(s["xi"], s["attr"], None, 1, [m["dv"]], s["idx"], s["n_live"],
                            dt=ens["dt"], kernel_id=m["kernel_id"], kparams=m["kparams"],
                            seed=4, run=m["run"], step=done // len(runs))
            states[r_] = s
            npairs += int(s["counters"][oracle.CNT_PAIRS])
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": npairs / dt, "unit": "pair-steps/s", "cores": 1,
                               "kind": "oracle", "seconds": round(dt, 3),
                               "sample": "%d run-steps (the 1024 runs in turn, each from its "
                                         "initial state), oracle (plain C, one thread)" % done}
    b.close()
    ctx.close()
    return out


def golovin_moments(t, N0, b, vbar):
    """Moments of the additive-kernel solution from an exponential start
    (eq. 7): M0 = N0 (1 - tau), M1 = N0 vbar, M2 = 2 N0 vbar^2 / (1 - tau)^2,
    tau = 1 - exp(-N0 b vbar t)."""
    import math
    tau = 1.0 - math.exp(-N0 * b * vbar * t)
    return N0 * (1.0 - tau), N0 * vbar, 2.0 * N0 * vbar ** 2 / (1.0 - tau) ** 2


def bench_golovin(args, sdm, torch, np, workloads):
    n_sd = 1 << 13
    w = workloads.box(n_sd, seed=1)
    ctx = sdm.Context(n_sd, 1, 1)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(1, 0, 0, step_dev=step_dev)
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
    out_m = []
    total_ms = 0.0
    for t_end in (1200, 2400, 3600):
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
        m = M.cpu().numpy()[0]
        ref = golovin_moments(float(t_end), w["N0"], w["b"], w["vbar"])
        out_m.append({"t_s": t_end, "M0_rel_err": float(m[0] / ref[0] - 1.0),
                      "M1_rel_err": float(m[1] / ref[1] - 1.0),
                      "M2_rel_err": float(m[2] / ref[2] - 1.0)})
    del g
    K = 3 * seg
    assert int(step_dev.item()) == K and ctx.read_errors() == 0
    out = base_line("SDM pair-steps/s, 2^13-SD Golovin box over 3600 s",
                    (n_sd // 2) * K / (total_ms / 1e3), "pair-steps/s", K, 0, total_ms / K,
                    "f64", {"workload": "golovin_box_2_13_3600s", "n_sd": n_sd, "cells": 1,
                            "kernel": "golovin", "b_per_s": w["b"], "dt_s": w["dt"], "seed": 1,
                            "timing": "three graph replays of 1200 steps"})
    out["wall_s_3600_steps"] = total_ms / 1e3
    out["golovin_moments"] = out_m
    out["roofline"] = None
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        s_ = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
        t0 = time.perf_counter()
        npairs = steps = 0
        while time.perf_counter() - t0 < args.cpu_seconds and steps < 3600:
            s_ = oracle.step(s_["xi"], s_["attr"], None, 1, w["dv"], s_["idx"], s_["n_live"],
                             dt=w["dt"], kernel_id=w["kernel_id"], kparams=w["kparams"],
                             seed=1, run=0, step=steps)
            npairs += int(s_["counters"][oracle.CNT_PAIRS])
            steps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": npairs / dt, "unit": "pair-steps/s",
                               "cores": 1, "kind": "oracle", "seconds": round(dt, 3),
                               "sample": "the first %d of the 3600 steps, oracle (plain C, one "
                                         "thread)" % steps}
    ctx.close()
    return out


def bench_surrogate(args, sdm, torch, np, workloads):
    """Surrogate step for every cell of the grid vs one SDM step of the grid
    (static cells), both on the GPU; random-init weights (the arithmetic per
    step does not depend on the weights)."""
    w = workloads.grid(seed=3)
    n_sd, n_cell = w["n_sd"], w["n_cell"]
    ctx = sdm.Context(n_sd, n_cell, 2)
    st = sdm.State(w["xi"], w["attr"], w["cell_id"], n_cell)
    dv = torch.as_tensor(np.asarray(w["dv"], np.float64)).cuda()
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    ctx.step(st, w["dt"], k, sdm.rng(3, 0, 0), dv_per_cell=dv)
    M = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")
    ctx.moments(M, st.xi, st.attr[0], st.idx, st.cell_start, n_cell, dv_per_cell=dv)
    torch.cuda.synchronize()
    lm = torch.log(M).cpu().numpy()
    mean = np.concatenate([lm.mean(0), [1.0, 1.0]]).astype(np.float32)
    std = np.concatenate([lm.std(0) + 1e-6, [1.0, 1.0]]).astype(np.float32)
    net = sdm.Mlp(ctx, workloads.mlp_init(7))
    x = torch.zeros((n_cell, 5), dtype=torch.float32, device="cuda")
    y = torch.zeros((n_cell, 3), dtype=torch.float32, device="cuda")
    fb = torch.zeros(n_cell, dtype=torch.uint8, device="cuda")
    lo, hi = [-8.0] * 5, [8.0] * 5
    tm, ts = [0.0, 0.0, 0.0], [1e-6, 1e-9, 1e-6]
    lib = sdm.lib()
    e_fwd = [HipEvent(lib) for _ in range(2 * args.steps)]

    def sur_step(t, stream, ev):
        ctx.mlp_features(x, M, w["dt"], w["kernel_id"], mean, std, stream=stream)
        ctx.hull_check(fb, x, lo, hi, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        ctx.mlp_forward(y, x, net, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.mlp_apply(M, y, w["dt"], tm, ts, fallback=fb, stream=stream)

    for t in range(args.warmup):
        sur_step(t, None, None)
    K = args.steps
    stream = torch.cuda.Stream()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s0.record(stream)
        for t in range(K):
            sur_step(t, stream, e_fwd[2 * t:2 * t + 2])
        s1.record(stream)
    torch.cuda.synchronize()
    sur_ms = s0.elapsed_time(s1)
    fwd_ms = sum(e_fwd[2 * t].elapsed_ms(e_fwd[2 * t + 1]) for t in range(K)) / K
    for e in e_fwd:
        e.destroy()
    gms = None if args.eager else graph_ms(torch, sur_step, K, stream)

    # the particle method on the same cells (no reassignment)
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(3, 0, 1, step_dev=step_dev)

    def sdm_step(t, stream, ev):
        ctx.step(st, w["dt"], k, r, stream=stream, events=ev, dv_per_cell=dv,
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
                     "network": "5-128-128-128-3 GELU", "dt_s": w["dt"], "seed": 3,
                     "step": "features + hull test + forward + moment update",
                     "timing": TIMING if gms else TIMING_EAGER})
    out["sdm_cell_steps_per_s"] = n_cell / (sdm_step_ms / 1e3)
    out["speedup_vs_sdm"] = out["value"] / out["sdm_cell_steps_per_s"]
    out["roofline"] = {"bound": "mfma", "kernel": "k_mlp_forward_split", "achieved": achieved,
                       "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None}
    out["kernel_ms"] = {"k_mlp_forward_split": fwd_ms}
    out["graph_ms_per_step"] = gms
    out["eager_ms_per_step"] = sur_ms / K
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        from oracle import mlp
        xh = x.cpu().numpy()
        th = workloads.mlp_init(7)
        net_o = mlp.Net("bf16")
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            net_o.forward(th, xh)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_cell * reps / dt, "unit": "cell-steps/s",
                               "cores": 1, "kind": "oracle", "seconds": round(dt, 3),
                               "sample": "%d bf16-emulated forward passes over the 16384 cells "
                                         "(numpy)" % reps}
    ctx.close()
    return out


MLP_TRAIN_BATCH = 4096
MLP_BWD_FLOP_PER_SAMPLE = 133888.0  # dW of all four layers + dH of layers 4, 3, 2


def bench_train(args, sdm, torch, np, workloads):
    """Surrogate training: one step is one minibatch of 4096 samples through
    the forward pass (keeping pre-activations), the MSE gradient, the
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
                     "step": "forward (with pre-activations) + MSE gradient + backward + Adam",
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
                    choices=["box", "grid", "ensemble", "golovin", "surrogate", "train"])
    ap.add_argument("--log2-n-sd", type=int, default=22)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="host time given to the oracle baseline (whole steps, at least one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="skip the graph-replay measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (counter calibration)")
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
          "train": bench_train}[args.workload]
    out = fn(args, sdm, torch, np, workloads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
