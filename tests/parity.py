"""Parity helpers shared by the GPU tests and the benchmark's check leg.

gamma = ceil(p - phi) (Sec. 2.2, Step 3) is an integer decided by floating
point.  The GPU and the oracle evaluate p with the same IEEE operations in
the same order, so their gammas agree bit for bit.  Where they disagree,
the disagreement is a *threshold flip* when p - phi lies within
1e-12 max(1, p) of an integer (any rounding difference could move it across
the step of ceil), and an error otherwise.  Flips are counted and reported;
the pair's two SDs may then differ, every other SD must still agree.
"""
from __future__ import annotations

import numpy as np

import oracle

FLIP_TOL = 1e-12


def slot_probabilities(xi, attr, cell_id, n_cell, dv, idx, n_live, *, dt, kernel_id, kparams,
                       seed, run, step):
    """Steps 0-2 of one timestep through the oracle's routines: the pair
    probability p and the uniform phi of every pair slot, and the positions
    and sorted Index that give each slot its two SDs."""
    xi = np.ascontiguousarray(xi, np.uint64)
    n_sd = int(xi.shape[0])
    cid = np.zeros(n_sd, np.int32) if cell_id is None else np.ascontiguousarray(cell_id, np.int32)
    dvc = np.ascontiguousarray(np.broadcast_to(np.asarray(dv, np.float64), (n_cell,)))
    idx0, n = oracle.remove_if_equal_0(idx, n_live, xi)
    u = oracle.urand(n_sd, seed, run, step, oracle.STREAM_SHUFFLE)
    idx1, cs = oracle.shuffle_per_cell(idx0, n, cid, n_cell, u)
    flag = oracle.flag_pairs(cid, cs, idx1, n)
    v = np.ascontiguousarray(np.asarray(attr, np.float64).reshape(-1, n_sd)[0])
    p = oracle.coalescence_kernel(flag, v, idx1, n, kernel_id, kparams)
    p = oracle.times_max(p, xi, flag, idx1, n)
    p = oracle.normalize(p, dt, dvc, cid, cs, flag, idx1, n)
    phi = oracle.urand(n // 2, seed, run, step, oracle.STREAM_GAMMA)
    return dict(p=p, phi=phi, flag=flag, idx=idx1[:n], n_live=n)


def classify_gamma(g_gpu, g_ref, p, phi, tol=FLIP_TOL):
    """Splits the slots where the two gammas differ into threshold flips and
    errors.  Returns (flips, errors) as index arrays."""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    n = min(g_gpu.shape[0], g_ref.shape[0])
    differ = np.nonzero(~((g_gpu[:n] == g_ref[:n]) |
                          (np.isnan(g_gpu[:n]) & np.isnan(g_ref[:n]))))[0]
    flips, errors = [], []
    for q in differ:
        if q >= p.shape[0]:
            errors.append(q)
            continue
        x = float(p[q]) - float(phi[q])
        near = abs(x - round(x)) < tol * max(1.0, abs(float(p[q])))
        if near and abs(g_gpu[q] - g_ref[q]) == 1.0:
            flips.append(q)
        else:
            errors.append(q)
    return np.asarray(flips, np.int64), np.asarray(errors, np.int64)


def sds_of_slots(slots, flag, idx):
    """The SD ids of the pairs that own the given slots."""
    pos = np.nonzero(flag)[0]
    owner = {int(i) // 2: (int(idx[i]), int(idx[i + 1])) for i in pos}
    out = []
    for q in slots:
        out.extend(owner.get(int(q), ()))
    return np.asarray(out, np.int64)


def compare_step(gpu, ref, pre, what=""):
    """Compares one step's GPU result with the oracle's.

    gpu, ref: dicts with xi, attr, idx, n_live and gamma (ref from
    oracle.step); pre: slot_probabilities of the state before the step, or
    a function returning them (called only when the gammas differ).
    Returns the number of threshold flips; raises AssertionError on any
    other difference."""
    n = ref["n_live"]
    assert gpu["n_live"] == n, what
    assert np.array_equal(gpu["idx"][:n], ref["idx"][:n]), what
    flips = np.zeros(0, np.int64)
    if "gamma" in gpu and "gamma" in ref and not np.array_equal(gpu["gamma"], ref["gamma"]):
        if callable(pre):
            pre = pre()
        flips, errors = classify_gamma(gpu["gamma"], ref["gamma"], pre["p"], pre["phi"])
        assert errors.size == 0, (what, errors[:5], gpu["gamma"][errors[:5]],
                                  ref["gamma"][errors[:5]])
    excused = sds_of_slots(flips, pre["flag"], pre["idx"]) if flips.size else np.zeros(0, np.int64)
    keep = np.ones(ref["xi"].shape[0], bool)
    keep[excused] = False
    assert np.array_equal(gpu["xi"][keep], ref["xi"][keep]), what
    ga, ra = gpu["attr"][:, keep], ref["attr"][:, keep]
    if not np.array_equal(ga, ra):
        rel = np.abs(ga - ra) / np.maximum(np.abs(ra), 1e-300)
        assert rel.max() <= 1e-12, (what, rel.max())
        raise AssertionError("attributes within 1e-12 but not bit-identical: %s" % what)
    return int(flips.size)
