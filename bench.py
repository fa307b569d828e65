"""Throughput of the fused SDM coagulation step on one MI355X.

Workload: the paper's Golovin box (arXiv:2101.06318, Sec. 4: dV = 1e6 m^3,
N0 = 2^23 m^-3, exponential volumes with mean (4 pi/3)(30.531 um)^3,
b = 1500 1/s, dt = 1 s), scaled to 2^22 super-droplets, synthetic, seed 2.
A step is one whole timestep (Steps 0-3: removal, shuffle, pairing, pair
probability, gamma, collision update) through the C ABI (sdm_step, three
kernels).  W warm-up steps run first; then exactly K steps are timed on
one stream, bracketed by synchronisation, with HIP events recorded by the
library before and after each of its kernels on that stream (per-kernel
durations for the roofline).  The same K steps are then also captured in a
HIP graph and replayed once; that time is reported as graph_ms_per_step.

Prints one JSON line (metric, value, ..., roofline, cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SDM pair-steps/s at n_sd=2^22"


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2101_06318_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_sd, f_coll):
    """Algorithmic HBM bytes of one step, split per kernel.

    Per pair-step (two SDs): xi (8 B) and volume (8 B) read for each SD,
    the Index written (4 B) and read (4 B) for each SD, and the two SDs'
    xi and volume written back when the pair collides (32 B * f_coll):
    48 + 32 f_coll bytes.  The scatter kernel is charged the reads (40 B per
    pair), the group kernel the Index write and the write-back
    (8 + 32 f_coll B per pair)."""
    pairs = n_sd // 2
    return dict(step=pairs * (48.0 + 32.0 * f_coll),
                k_scatter=pairs * 40.0,
                k_group=pairs * (8.0 + 32.0 * f_coll),
                k_seams=0.0)


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


def cpu_baseline(w, n_steps):
    import numpy as np

    import oracle
    n = w["n_sd"]
    st = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n, dtype=np.uint32), n_live=n)
    t0 = time.perf_counter()
    for t in range(n_steps):
        st = oracle.step(st["xi"], st["attr"], None, 1, w["dv"], st["idx"], st["n_live"],
                         dt=w["dt"], kernel_id=w["kernel_id"], kparams=w["kparams"], seed=2,
                         run=0, step=t)
    dt = time.perf_counter() - t0
    return dict(value=(n // 2) * n_steps / dt, unit="pair-steps/s", cores=1, kind="oracle",
                sample="%d steps of the 2^%d-SD Golovin box (seed 2) from its initial state, "
                       "oracle (plain C, one thread, qsort-based shuffle)"
                       % (n_steps, n.bit_length() - 1),
                seconds=round(dt, 3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--log2-n-sd", type=int, default=22)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="skip the graph-replay measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the SDM step of one run on one "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_06318_amd as sdm
    from paper_2101_06318_amd import workloads

    if not os.path.exists(sdm.LIB_PATH):
        from paper_2101_06318_amd import build
        build.build()
    torch.cuda.set_device(0)
    n_sd = 1 << args.log2_n_sd
    w = workloads.box(n_sd, seed=2)
    ctx = sdm.Context(n_sd, 1, 1)
    st = sdm.State(w["xi"], w["attr"], None, 1)
    k = sdm.kernel(w["kernel_id"], w["kparams"])
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = sdm.rng(2, 0, 0, step_dev=step_dev)
    kw = dict(dv=w["dv"][0], step_advance=step_dev)
    print("bench: n_sd=2^%d warmup=%d steps=%d" % (args.log2_n_sd, args.warmup, args.steps),
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
    for _ in range(args.warmup):
        ctx.step(st, w["dt"], k, r, **kw)
    torch.cuda.synchronize()
    coll0 = int(st.counters.cpu().numpy()[sdm.CNT_COLLISIONS])
    pairs0 = int(st.counters.cpu().numpy()[sdm.CNT_PAIRS])

    K = args.steps
    L = sdm.lib()
    ev = [[HipEvent(L) for _ in range(4)] for _ in range(K)]
    stream = torch.cuda.Stream()

    # Timed region: exactly K steps on one stream; the library records HIP
    # events before/after each of its three kernels on that stream.
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        start.record(stream)
        for t in range(K):
            ctx.step(st, w["dt"], k, r, stream=stream, events=ev[t], **kw)
        end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    per = {"k_scatter": [], "k_group": [], "k_seams": []}
    for t in range(K):
        per["k_scatter"].append(ev[t][0].elapsed_ms(ev[t][1]))
        per["k_group"].append(ev[t][1].elapsed_ms(ev[t][2]))
        per["k_seams"].append(ev[t][2].elapsed_ms(ev[t][3]))
    avg_ms = {kname: float(np.mean(v)) for kname, v in per.items()}

    cnt = st.counters.cpu().numpy()
    graph_ms = None
    if not args.eager:
        # Same K steps captured once in a HIP graph and replayed (reported
        # beside the timed region; the step index advances on the device).
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(stream):
                with torch.cuda.graph(g, stream=stream):
                    for t in range(K):
                        ctx.step(st, w["dt"], k, r, stream=stream, **kw)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            gs = torch.cuda.Event(enable_timing=True)
            ge = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                gs.record(stream)
                g.replay()
                ge.record(stream)
            torch.cuda.synchronize()
            graph_ms = gs.elapsed_time(ge) / K
            del g
        except Exception as e:
            print("bench: graph replay not measured (%s)" % e, file=sys.stderr, flush=True)
    pairs = int(cnt[sdm.CNT_PAIRS]) - pairs0
    f_coll = (int(cnt[sdm.CNT_COLLISIONS]) - coll0) / max(pairs, 1)
    n_live = int(st.n_live.item())
    assert ctx.read_errors() == 0
    pair_steps = (n_sd // 2) * K
    value = pair_steps / (total_ms / 1e3)
    ab = algorithmic_bytes(n_sd, f_coll)
    dom = max(avg_ms, key=avg_ms.get)
    achieved = ab[dom] / (avg_ms[dom] / 1e3) / 1e9
    workload = "golovin_box_2_%d" % args.log2_n_sd
    traffic = traffic_record(dom, workload)
    step_gbs = ab["step"] / (total_ms / K / 1e3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n_sd": n_sd, "cells": 1, "kernel": "golovin",
                   "b_per_s": w["b"], "dt_s": w["dt"], "dv_m3": float(w["dv"][0]),
                   "seed": 2, "timing": "eager, one stream, HIP events per kernel",
                   "n_live": n_live,
                   "collision_fraction": f_coll},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernel_ms": avg_ms,
        "graph_ms_per_step": graph_ms,
        "step_roofline": {"bound": "hbm", "bytes_per_step": ab["step"], "achieved": step_gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_gbs / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host (%d steps)" % args.cpu_steps,
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    for row in ev:
        for e in row:
            e.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
