"""Oracle: plain single-threaded C99 reference of the Super-Droplet Method step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package; the product library
under ``paper_2101_06318_amd`` never does, and shares no code with it.

This module compiles ``sdm_oracle.c`` with gcc (``-O2 -ffp-contract=off``,
no fast-math) on first use and exposes numpy wrappers over its C entry
points.  Each wrapper follows the routine of the paper's backend API
(Bartman & Arabas, arXiv:2101.06318, Sec. 3.2, workflow figure) named in
its docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdm_oracle.c")
_HDR = os.path.join(_HERE, "sdm_oracle.h")
_LIB = os.path.join(_HERE, "libsdmo.so")
_lock = threading.Lock()
_lib = None

STREAM_SHUFFLE, STREAM_GAMMA, STREAM_INIT, STREAM_REASSIGN, STREAM_MLP, STREAM_FY = range(6)
STREAM_MERGE = 8
KERNEL_GOLOVIN, KERNEL_GEOMETRIC, KERNEL_CONSTANT, KERNEL_MULTIPLICATIVE, KERNEL_TABULATED = range(5)
CNT_PAIRS, CNT_COLLISIONS, CNT_CAPPED, CNT_ZEROED, CNT_GAMMA_GE2 = range(5)
N_COUNTERS = 8

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle shared library (gcc) if it is missing or stale."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            _declare(L)
            _lib = L
    return _lib


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("kernel_id", C.c_int32),
                ("kparams", C.c_double * 4), ("seed", C.c_uint64),
                ("run", C.c_uint32), ("step", C.c_uint32), ("table", C.c_void_p)]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_U32 = C.c_uint32
_U64 = C.c_uint64
_D = C.c_double


def _declare(L):
    sig = {
        "sdmo_philox4x32_10": (None, [_P, _P, _P]),
        "sdmo_word": (_U64, [_U64, _U32, _U32, _U32, _U64]),
        "sdmo_uniform": (_D, [_U64, _U32, _U32, _U32, _U64]),
        "sdmo_urand": (None, [_P, _I64, _U64, _U32, _U32, _U32]),
        "sdmo_remove_if_equal_0": (_I64, [_P, _I64, _P]),
        "sdmo_cell_sort": (C.c_int, [_P, _P, _I64, _P, _I32]),
        "sdmo_shuffle_per_cell": (C.c_int, [_P, _P, _I64, _P, _I32, _P]),
        "sdmo_flag_pairs": (None, [_P, _P, _P, _P, _I64]),
        "sdmo_shuffle_fisher_yates": (C.c_int, [_P, _P, _I64, _P, _I32, _U64, _U32, _U32]),
        "sdmo_shuffle_merge": (C.c_int, [_P, _P, _I64, _P, _I32, _U64, _U32, _U32]),
        "sdmo_kernel_value": (_D, [_I32, _P, _P, _D, _D]),
        "sdmo_coalescence_kernel": (None, [_P, _P, _P, _P, _I64, _I32, _P, _P]),
        "sdmo_times_max": (None, [_P, _P, _P, _P, _I64]),
        "sdmo_pair_scale": (_U64, [_U64]),
        "sdmo_normalize": (None, [_P, _D, _P, _P, _P, _P, _P, _I64]),
        "sdmo_compute_gamma": (None, [_P, _P, _I64]),
        "sdmo_update_attributes": (None, [_P, _P, _I32, _I64, _P, _P, _P, _I64, _P]),
        "sdmo_step": (C.c_int, [_P, _P, _I32, _I64, _I64, _P, _I32, _P, _P, _P, _P,
                                C.POINTER(Params), _P, _P, _P]),
        "sdmo_moments": (C.c_int, [_P, _P, _P, _P, _P, _I64, _I64, _I32, _P]),
        "sdmo_cbrt": (_D, [_D]),
        "sdmo_terminal_velocity": (_D, [_D]),
        "sdmo_reassign": (None, [_P, _I64, _I32, _U64, _U32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


# ---------------------------------------------------------------- RNG ----
def philox(ctr, key):
    """Raw Philox4x32-10 block for counter ctr[4] and key key[2]."""
    c = _arr(ctr, np.uint32)
    k = _arr(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().sdmo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def word(seed, run, step, stream, e):
    return int(lib().sdmo_word(seed, run, step, stream, e))


def uniform(seed, run, step, stream, e):
    return float(lib().sdmo_uniform(seed, run, step, stream, e))


def urand(n, seed, run, step, stream):
    """urand (workflow Steps 1 and 3): u01[e] = U(seed, run, step, stream, e)."""
    out = np.empty(int(n), np.float64)
    lib().sdmo_urand(_ptr(out), int(n), seed, run, step, stream)
    return out


# ------------------------------------------------------------ routines ----
def remove_if_equal_0(idx, n_live, xi):
    """Step 0: stable removal of zero-multiplicity SDs.  Returns (idx, n)."""
    idx = _arr(idx, np.uint32).copy()
    xi = _arr(xi, np.uint64)
    n = lib().sdmo_remove_if_equal_0(_ptr(idx), int(n_live), _ptr(xi))
    return idx, int(n)


def cell_sort(idx, n_live, cell_id, n_cell):
    """Stable counting sort of the Index by cell id.  Returns (idx, cell_start)."""
    idx = _arr(idx, np.uint32).copy()
    cell_id = _arr(cell_id, np.int32)
    cs = np.zeros(n_cell + 1, np.uint32)
    rc = lib().sdmo_cell_sort(_ptr(cs), _ptr(idx), int(n_live), _ptr(cell_id), int(n_cell))
    if rc:
        raise ValueError("cell id out of range")
    return idx, cs


def shuffle_per_cell(idx, n_live, cell_id, n_cell, u01_by_sd):
    """shuffle_per_cell (Step 1).  Returns (idx, cell_start)."""
    idx = _arr(idx, np.uint32).copy()
    cell_id = _arr(cell_id, np.int32)
    u = _arr(u01_by_sd, np.float64)
    cs = np.zeros(n_cell + 1, np.uint32)
    rc = lib().sdmo_shuffle_per_cell(_ptr(cs), _ptr(idx), int(n_live), _ptr(cell_id),
                                     int(n_cell), _ptr(u))
    if rc:
        raise ValueError("cell id out of range")
    return idx, cs


def flag_pairs(cell_id, cell_start, idx, n_live):
    flag = np.zeros(max(int(n_live), 1), np.uint8)
    lib().sdmo_flag_pairs(_ptr(flag), _ptr(_arr(cell_id, np.int32)),
                          _ptr(_arr(cell_start, np.uint32)), _ptr(_arr(idx, np.uint32)),
                          int(n_live))
    return flag[:int(n_live)]


def _table(table):
    return None if table is None else _arr(table, np.float64)


def shuffle_variant(method, idx, n_live, cell_id, n_cell, seed, run, step):
    """The O(n) per-cell permutations (Sec. 3.2): method "fisher_yates" or
    "merge"; returns (idx, cell_start)."""
    n = int(n_live)
    out = _arr(idx, np.uint32).copy()
    cs = np.zeros(n_cell + 1, np.uint32)
    cid = np.zeros(max(len(out), 1), np.int32) if cell_id is None else _arr(cell_id, np.int32)
    fn = {"fisher_yates": lib().sdmo_shuffle_fisher_yates,
          "merge": lib().sdmo_shuffle_merge}[method]
    if fn(_ptr(cs), _ptr(out), n, _ptr(cid), int(n_cell), int(seed), int(run), int(step)):
        raise ValueError("cell id out of range")
    return out[:n], cs


def kernel_value(kernel_id, kparams, v1, v2, table=None):
    kp = _arr(list(kparams) + [0.0] * (4 - len(kparams)), np.float64)
    tb = _table(table)
    return float(lib().sdmo_kernel_value(kernel_id, _ptr(kp), _ptr(tb), v1, v2))


def coalescence_kernel(flag, volume, idx, n_live, kernel_id, kparams, table=None):
    n = int(n_live)
    prob = np.zeros(max(n // 2, 1), np.float64)
    kp = _arr(list(kparams) + [0.0] * (4 - len(kparams)), np.float64)
    tb = _table(table)
    lib().sdmo_coalescence_kernel(_ptr(prob), _ptr(_arr(flag, np.uint8)),
                                  _ptr(_arr(volume, np.float64)), _ptr(_arr(idx, np.uint32)),
                                  n, kernel_id, _ptr(kp), _ptr(tb))
    return prob[:n // 2]


def times_max(pair_prob, xi, flag, idx, n_live):
    p = _arr(pair_prob, np.float64).copy()
    lib().sdmo_times_max(_ptr(p), _ptr(_arr(xi, np.uint64)), _ptr(_arr(flag, np.uint8)),
                         _ptr(_arr(idx, np.uint32)), int(n_live))
    return p


def pair_scale(n):
    return int(lib().sdmo_pair_scale(int(n)))


def normalize(pair_prob, dt, dv_per_cell, cell_id, cell_start, flag, idx, n_live):
    p = _arr(pair_prob, np.float64).copy()
    lib().sdmo_normalize(_ptr(p), float(dt), _ptr(_arr(dv_per_cell, np.float64)),
                         _ptr(_arr(cell_id, np.int32)), _ptr(_arr(cell_start, np.uint32)),
                         _ptr(_arr(flag, np.uint8)), _ptr(_arr(idx, np.uint32)), int(n_live))
    return p


def compute_gamma(pair_prob, u01_by_slot):
    p = _arr(pair_prob, np.float64).copy()
    u = _arr(u01_by_slot, np.float64)
    lib().sdmo_compute_gamma(_ptr(p), _ptr(u), int(p.shape[0]))
    return p


def update_attributes(xi, attr, gamma, flag, idx, n_live, counters=None):
    """update_attributes (Step 3).  attr is [n_attr, stride]; returns (xi, attr, counters)."""
    xi = _arr(xi, np.uint64).copy()
    attr = np.array(attr, dtype=np.float64, order="C", copy=True, ndmin=2)
    cnt = np.zeros(N_COUNTERS, np.uint64) if counters is None else _arr(counters, np.uint64).copy()
    lib().sdmo_update_attributes(_ptr(xi), _ptr(attr), int(attr.shape[0]), int(attr.shape[1]),
                                 _ptr(_arr(gamma, np.float64)), _ptr(_arr(flag, np.uint8)),
                                 _ptr(_arr(idx, np.uint32)), int(n_live), _ptr(cnt))
    return xi, attr, cnt


def step(xi, attr, cell_id, n_cell, dv_per_cell, idx, n_live, *, dt, kernel_id, kparams,
         seed, run, step, counters=None, want_gamma=False, want_flag=False, table=None):
    """One whole timestep (workflow figure, Steps 0-3) for one run.

    Returns a dict with the updated xi, attr, idx, n_live, cell_start,
    counters and, on request, the slot gammas and pair flags.
    """
    xi = _arr(xi, np.uint64).copy()
    attr = np.array(attr, dtype=np.float64, order="C", copy=True, ndmin=2)
    n_sd = int(xi.shape[0])
    idx = _arr(idx, np.uint32).copy()
    cid = None if cell_id is None else _arr(cell_id, np.int32)
    dv = _arr(np.broadcast_to(np.asarray(dv_per_cell, np.float64), (n_cell,)), np.float64)
    nl = C.c_int64(int(n_live))
    cs = np.zeros(n_cell + 1, np.uint32)
    cnt = np.zeros(N_COUNTERS, np.uint64) if counters is None else _arr(counters, np.uint64).copy()
    P = Params()
    P.dt = dt
    P.kernel_id = kernel_id
    kp = list(kparams) + [0.0] * (4 - len(kparams))
    for i in range(4):
        P.kparams[i] = kp[i]
    P.seed, P.run, P.step = seed, run, step
    tb = _table(table)
    P.table = _ptr(tb)
    gam = np.zeros(max(n_sd // 2, 1), np.float64) if want_gamma else None
    flg = np.zeros(max(n_sd, 1), np.uint8) if want_flag else None
    rc = lib().sdmo_step(_ptr(xi), _ptr(attr), int(attr.shape[0]), int(attr.shape[1]), n_sd,
                         _ptr(cid), int(n_cell), _ptr(dv), _ptr(idx), C.byref(nl), _ptr(cs),
                         C.byref(P), _ptr(cnt), _ptr(gam), _ptr(flg))
    if rc:
        raise ValueError("cell id out of range")
    out = dict(xi=xi, attr=attr, idx=idx, n_live=int(nl.value), cell_start=cs, counters=cnt)
    if want_gamma:
        out["gamma"] = gam[:n_sd // 2]
    if want_flag:
        out["flag"] = flg[:n_sd]
    return out


def moments(xi, volume, cell_id, idx, n_live, n_cell, dv_per_cell):
    """Per-cell moments M0, M1, M2 (each divided by the cell volume)."""
    xi = _arr(xi, np.uint64)
    M = np.zeros((n_cell, 3), np.float64)
    dv = _arr(np.broadcast_to(np.asarray(dv_per_cell, np.float64), (n_cell,)), np.float64)
    cid = None if cell_id is None else _arr(cell_id, np.int32)
    rc = lib().sdmo_moments(_ptr(M), _ptr(xi), _ptr(_arr(volume, np.float64)), _ptr(cid),
                            _ptr(_arr(idx, np.uint32)), int(n_live), int(xi.shape[0]),
                            int(n_cell), _ptr(dv))
    if rc:
        raise ValueError("cell id out of range")
    return M


def cbrt(x):
    return float(lib().sdmo_cbrt(float(x)))


def terminal_velocity(r):
    return float(lib().sdmo_terminal_velocity(float(r)))


def reassign(n_sd, n_cell, seed, step):
    """Grid workload driver: uniform random cell per SD for timestep `step`."""
    out = np.zeros(int(n_sd), np.int32)
    lib().sdmo_reassign(_ptr(out), int(n_sd), int(n_cell), seed, step)
    return out
