"""Oracle throughput on the host, one process per core (TEST INFRASTRUCTURE:
the benchmark's CPU-baseline leg starts these as child processes).

    python -m oracle.hostbench --core C --of P --seconds S

runs the single-threaded oracle step (arXiv:2101.06318, Sec. 3.2) on the
1024-run ensemble: this process takes runs r with r mod P == C, each from its
own initial state, in turn, for S seconds, pinned to host core C (of those
the process may use), and prints one JSON line with the pairs visited and
the elapsed time.  P processes together give the whole-host throughput.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def host_info():
    """CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus_usable": len(os.sched_getaffinity(0)),
            "logical_cpus_total": os.cpu_count()}


def pin(core_index):
    """Pins this process to the core_index-th CPU it may use; returns its id."""
    cpus = sorted(os.sched_getaffinity(0))
    c = cpus[core_index % len(cpus)]
    os.sched_setaffinity(0, {c})
    return c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--core", type=int, required=True)
    ap.add_argument("--of", type=int, required=True)
    ap.add_argument("--seconds", type=float, default=10.0)
    a = ap.parse_args()
    cpu = pin(a.core)
    import numpy as np

    import oracle
    from paper_2101_06318_amd import workloads
    ens = workloads.ensemble(seed=4, n_runs=1024)
    mine = [m for m in ens["runs"] if m["run"] % a.of == a.core]
    states = [dict(xi=m["xi"], attr=m["attr"], idx=np.arange(m["n_sd"], dtype=np.uint32),
                   n_live=m["n_sd"]) for m in mine]
    oracle.lib()
    t0 = time.perf_counter()
    npairs = done = 0
    while time.perf_counter() - t0 < a.seconds:
        i = done % len(mine)
        m, s = mine[i], states[i]
        s = oracle.step(s["xi"], s["attr"], None, 1, [m["dv"]], s["idx"], s["n_live"],
                        dt=ens["dt"], kernel_id=m["kernel_id"], kparams=m["kparams"],
                        seed=4, run=m["run"], step=done // len(mine))
        states[i] = s
        npairs += int(s["counters"][oracle.CNT_PAIRS])
        done += 1
    print(json.dumps({"pairs": npairs, "seconds": time.perf_counter() - t0, "run_steps": done,
                      "cpu": cpu}), flush=True)


if __name__ == "__main__":
    main()
