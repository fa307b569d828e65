"""MI355X (gfx950) Super-Droplet Method coagulation library -- Python binding.

A thin ctypes layer over the C ABI declared in include/sdm.h (libsdm.so,
built from csrc/*.hip).  Every routine here only marshals arguments: the
work runs in the library's HIP kernels.  Device arrays are torch tensors on
a ROCm device (torch serves as the allocator and stream provider); their
data_ptr() is passed through.  There is no CPU fallback: importing a
routine without the built library raises.

The routine names follow the backend API of arXiv:2101.06318 (Sec. 3.2).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdm.so")

SDM_OK = 0
STREAM_SHUFFLE, STREAM_GAMMA, STREAM_INIT, STREAM_REASSIGN, STREAM_MLP = range(5)
KERNEL_GOLOVIN, KERNEL_GEOMETRIC, KERNEL_CONSTANT, KERNEL_MULTIPLICATIVE, KERNEL_TABULATED = range(5)
SHUFFLE_FISHER_YATES, SHUFFLE_MERGE = 1, 2
CNT_PAIRS, CNT_COLLISIONS, CNT_CAPPED, CNT_ZEROED, CNT_GAMMA_GE2, CNT_FALLBACK = range(6)
N_COUNTERS = 8


class SdmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sdm error %d: %s" % (code, msg))
        self.code = code


class Kernel(C.Structure):
    _fields_ = [("id", C.c_int32), ("reserved", C.c_int32), ("p", C.c_double * 4),
                ("table", C.c_void_p)]


class Rng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("run", C.c_uint32), ("step", C.c_uint32),
                ("step_dev", C.c_void_p)]


class StateC(C.Structure):
    _fields_ = [("n_sd", C.c_int64), ("n_cell", C.c_int32), ("n_attr", C.c_int32),
                ("attr_stride", C.c_int64), ("xi", C.c_void_p), ("attr", C.c_void_p),
                ("cell_id", C.c_void_p), ("idx", C.c_void_p), ("n_live_dev", C.c_void_p),
                ("cell_start", C.c_void_p), ("counters_dev", C.c_void_p),
                ("gamma_out", C.c_void_p)]


class StepParamsC(C.Structure):
    _fields_ = [("dt", C.c_double), ("dv_per_cell", C.c_void_p), ("dv", C.c_double),
                ("kernel", Kernel), ("rng", Rng), ("step_advance", C.c_void_p),
                ("expected_per_cell", C.c_double), ("events", C.c_void_p * 4)]


class MlpC(C.Structure):
    _fields_ = [("params", C.c_void_p), ("packed", C.c_void_p)]


class MlpOptC(C.Structure):
    _fields_ = [("m", C.c_void_p), ("v", C.c_void_p)]


class AdamHpC(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("t", C.c_int32), ("reserved", C.c_int32)]


class Segment(C.Structure):
    _fields_ = [("offset", C.c_int64), ("n_sd", C.c_int64), ("dv", C.c_double),
                ("kernel", Kernel), ("run", C.c_uint32), ("reserved", C.c_uint32)]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_U32 = C.c_uint32
_D = C.c_double
_INT = C.c_int

SIGNATURES = {
    "sdm_abi_version": (_INT, []),
    "sdm_last_error": (C.c_char_p, []),
    "sdm_create": (_INT, [C.POINTER(_P), _I64, _I32, _I32]),
    "sdm_destroy": (_INT, [_P]),
    "sdm_read_errors": (_INT, [_P, C.POINTER(_U32)]),
    "sdm_set_plan_limits": (_INT, [_P, _I32, _I32]),
    "sdm_urand": (_INT, [_P, _P, _I64, C.POINTER(Rng), _U32, _P]),
    "sdm_remove_if_equal_0": (_INT, [_P, _P, _P, _P, _P]),
    "sdm_remove_if_equal_0_noalloc": (_INT, [_P, _P, _P, _I64, _P]),
    "sdm_cell_sort": (_INT, [_P, _P, _P, _P, _P, _I32, _P]),
    "sdm_shuffle_per_cell": (_INT, [_P, _P, _P, _P, _P, _P, _I32, _P, C.POINTER(Rng), _P]),
    "sdm_flag_pairs": (_INT, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "sdm_shuffle_variant": (_INT, [_P, _I32, _P, _P, _P, _P, _I32, C.POINTER(Rng), _P]),
    "sdm_coalescence_kernel": (_INT, [_P, _P, _P, _P, _P, _P, C.POINTER(Kernel), _P]),
    "sdm_times_max": (_INT, [_P, _P, _P, _P, _P, _P, _P]),
    "sdm_normalize": (_INT, [_P, _P, _D, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sdm_pair_rate": (_INT, [_P, _P, _D, _P, _P, _P, _P, _P, _P, _P, _P,
                             C.POINTER(Kernel), _P]),
    "sdm_compute_gamma": (_INT, [_P, _P, _P, C.POINTER(Rng), _P, _P]),
    "sdm_update_attributes": (_INT, [_P, _P, _P, _I32, _I64, _P, _P, _P, _P, _P, _P]),
    "sdm_prepare_step": (_INT, [_P, C.POINTER(StateC), C.POINTER(StepParamsC)]),
    "sdm_step": (_INT, [_P, C.POINTER(StateC), C.POINTER(StepParamsC), _P]),
    "sdm_batch_create": (_INT, [_P, C.POINTER(_P), C.POINTER(Segment), _I32]),
    "sdm_batch_destroy": (_INT, [_P, _P]),
    "sdm_batch_step": (_INT, [_P, _P, C.POINTER(StateC), C.POINTER(StepParamsC), _P]),
    "sdm_batch_set_schedule": (_INT, [_P, _P, _I32, C.POINTER(_I32)]),
    "sdm_autotune": (_INT, [_P, _P, C.POINTER(StateC), C.POINTER(StepParamsC), _I32,
                            C.c_char_p, C.POINTER(_I32)]),
    "sdm_moments": (_INT, [_P, _P, _P, _P, _P, _P, _I32, _P, _D, _P]),
    "sdm_reassign": (_INT, [_P, _P, _I64, _I32, C.POINTER(Rng), _P]),
    "sdm_mlp_pack": (_INT, [_P, C.POINTER(MlpC), _P]),
    "sdm_mlp_forward": (_INT, [_P, _P, _P, _P, _I64, C.POINTER(MlpC), _P]),
    "sdm_mlp_backward": (_INT, [_P, _P, _P, _P, _P, _I64, C.POINTER(MlpC), _P]),
    "sdm_mlp_mse": (_INT, [_P, _P, _P, _P, _P, _I64, _P]),
    "sdm_mlp_adam": (_INT, [_P, C.POINTER(MlpC), C.POINTER(MlpOptC), _P, C.POINTER(AdamHpC),
                            _P]),
    "sdm_hull_check": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "sdm_mlp_features": (_INT, [_P, _P, _P, _I64, _D, _I32, _P, _P, _P]),
    "sdm_mlp_apply": (_INT, [_P, _P, _P, _P, _I64, _D, _P, _P, _P]),
    "sdm_ood_check": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P]),
    "sdm_seed_from_moments": (_INT, [_P, _P, _P, _P, _P, _I32, _I32, _D, _P]),
    "sdm_moments_merge": (_INT, [_P, _P, _P, _P, _I64, _P]),
}

MLP_N_PARAMS = 34179
MLP_PACKED_BYTES = 151552
MLP_CACHE_FLOATS_PER_ROW = 576

_lib = None


def lib():
    """Load libsdm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsdm.so is not built; run __graft_entry__.build() "
                              "or python -m paper_2101_06318_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SDM_OK:
        raise SdmError(rc, lib().sdm_last_error().decode(errors="replace"))


def _ptr(t):
    """Device (or None) pointer of a tensor."""
    if t is None:
        return None
    return t.data_ptr()


def _row_stride(a):
    """Element stride between attribute rows (a single row: its length; the
    stride of a size-1 dimension is arbitrary)."""
    return int(a.shape[1]) if a.shape[0] == 1 else int(a.stride(0))


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def kernel(kernel_id, params=(0.0,), table=None):
    """An sdm_kernel; table: device tensor of float64 (tabulated kernels),
    which the caller keeps alive while the kernel is in use."""
    k = Kernel()
    k.id = int(kernel_id)
    p = list(params) + [0.0] * (4 - len(params))
    for i in range(4):
        k.p[i] = float(p[i])
    k.table = _ptr(table)
    return k


def rng(seed, run=0, step=0, step_dev=None):
    r = Rng()
    r.seed, r.run, r.step = int(seed), int(run), int(step)
    r.step_dev = _ptr(step_dev)
    return r


NOALLOC_MAX_IDS = 1 << 22


def remove_if_equal_0_noalloc(idx, n_live, xi, n_sd_max=None, stream=None):
    """Step 0 without a context or any allocation (the library's fixed
    scratch); n_sd_max defaults to idx's length."""
    cap = int(idx.numel()) if n_sd_max is None else int(n_sd_max)
    _check(lib().sdm_remove_if_equal_0_noalloc(_ptr(idx), _ptr(n_live), _ptr(xi), cap,
                                               _stream(stream)))


class Context:
    """Owns an sdm_ctx (device workspace) for up to n_sd_max SDs."""

    def __init__(self, n_sd_max, n_cell_max=1, n_attr_max=2):
        self._h = C.c_void_p()
        _check(lib().sdm_create(C.byref(self._h), int(n_sd_max), int(n_cell_max),
                                int(n_attr_max)))
        self.n_sd_max, self.n_cell_max, self.n_attr_max = n_sd_max, n_cell_max, n_attr_max

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().sdm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def read_errors(self):
        f = C.c_uint32(0)
        _check(lib().sdm_read_errors(self._h, C.byref(f)))
        return int(f.value)

    def set_plan_limits(self, bucket_cap=0, group_cap=-1):
        _check(lib().sdm_set_plan_limits(self._h, int(bucket_cap), int(group_cap)))

    # ------------------------------------------------ workflow routines
    def urand(self, u01, r, stream_id, n=None, stream=None):
        n = u01.numel() if n is None else n
        _check(lib().sdm_urand(self._h, _ptr(u01), int(n), C.byref(r), int(stream_id),
                               _stream(stream)))

    def remove_if_equal_0(self, idx, n_live, xi, stream=None):
        _check(lib().sdm_remove_if_equal_0(self._h, _ptr(idx), _ptr(n_live), _ptr(xi),
                                           _stream(stream)))

    def shuffle_variant(self, method, cell_start, idx, n_live, cell_id, n_cell, r,
                        stream=None):
        _check(lib().sdm_shuffle_variant(self._h, int(method), _ptr(cell_start), _ptr(idx),
                                         _ptr(n_live), _ptr(cell_id), int(n_cell), C.byref(r),
                                         _stream(stream)))

    def cell_sort(self, cell_start, idx, n_live, cell_id, n_cell, stream=None):
        _check(lib().sdm_cell_sort(self._h, _ptr(cell_start), _ptr(idx), _ptr(n_live),
                                   _ptr(cell_id), int(n_cell), _stream(stream)))

    def shuffle_per_cell(self, cell_start, idx, n_live, cell_idx, cell_id, n_cell,
                         u01_by_sd=None, r=None, stream=None):
        _check(lib().sdm_shuffle_per_cell(self._h, _ptr(cell_start), _ptr(idx), _ptr(n_live),
                                          _ptr(cell_idx), _ptr(cell_id), int(n_cell),
                                          _ptr(u01_by_sd), C.byref(r) if r else None,
                                          _stream(stream)))

    def flag_pairs(self, pair_flag, cell_id, cell_idx, cell_start, idx, n_live, stream=None):
        _check(lib().sdm_flag_pairs(self._h, _ptr(pair_flag), _ptr(cell_id), _ptr(cell_idx),
                                    _ptr(cell_start), _ptr(idx), _ptr(n_live), _stream(stream)))

    def coalescence_kernel(self, pair_prob, pair_flag, volume, idx, n_live, k, stream=None):
        _check(lib().sdm_coalescence_kernel(self._h, _ptr(pair_prob), _ptr(pair_flag),
                                            _ptr(volume), _ptr(idx), _ptr(n_live), C.byref(k),
                                            _stream(stream)))

    def times_max(self, pair_prob, xi, pair_flag, idx, n_live, stream=None):
        _check(lib().sdm_times_max(self._h, _ptr(pair_prob), _ptr(xi), _ptr(pair_flag),
                                   _ptr(idx), _ptr(n_live), _stream(stream)))

    def normalize(self, pair_prob, dt, dv_per_cell, cell_id, cell_idx, cell_start, pair_flag,
                  idx, n_live, stream=None):
        _check(lib().sdm_normalize(self._h, _ptr(pair_prob), float(dt), _ptr(dv_per_cell),
                                   _ptr(cell_id), _ptr(cell_idx), _ptr(cell_start),
                                   _ptr(pair_flag), _ptr(idx), _ptr(n_live), _stream(stream)))

    def pair_rate(self, pair_prob, dt, dv_per_cell, pair_flag, volume, xi, cell_id, cell_start,
                  idx, n_live, k, stream=None):
        _check(lib().sdm_pair_rate(self._h, _ptr(pair_prob), float(dt), _ptr(dv_per_cell),
                                   _ptr(pair_flag), _ptr(volume), _ptr(xi), _ptr(cell_id),
                                   _ptr(cell_start), _ptr(idx), _ptr(n_live), C.byref(k),
                                   _stream(stream)))

    def compute_gamma(self, pair_prob, n_live, u01_by_slot=None, r=None, stream=None):
        _check(lib().sdm_compute_gamma(self._h, _ptr(pair_prob), _ptr(u01_by_slot),
                                       C.byref(r) if r else None, _ptr(n_live),
                                       _stream(stream)))

    def update_attributes(self, xi, attr, gamma, pair_flag, idx, n_live, counters=None,
                          stream=None):
        n_attr, stride = (attr.shape[0], _row_stride(attr)) if attr.dim() == 2 else (1, attr.numel())
        _check(lib().sdm_update_attributes(self._h, _ptr(xi), _ptr(attr), int(n_attr),
                                           int(stride), _ptr(gamma), _ptr(pair_flag), _ptr(idx),
                                           _ptr(n_live), _ptr(counters), _stream(stream)))

    def moments(self, M, xi, volume, idx, cell_start, n_cell, dv_per_cell=None, dv=0.0,
                stream=None):
        _check(lib().sdm_moments(self._h, _ptr(M), _ptr(xi), _ptr(volume), _ptr(idx),
                                 _ptr(cell_start), int(n_cell), _ptr(dv_per_cell), float(dv),
                                 _stream(stream)))

    def reassign(self, cell_id, n_sd, n_cell, r, stream=None):
        _check(lib().sdm_reassign(self._h, _ptr(cell_id), int(n_sd), int(n_cell), C.byref(r),
                                  _stream(stream)))

    # ------------------------------------------------ moment surrogate
    def mlp_pack(self, net, stream=None):
        _check(lib().sdm_mlp_pack(self._h, C.byref(net.c), _stream(stream)))

    def mlp_forward(self, y, x, net, cache=None, stream=None):
        _check(lib().sdm_mlp_forward(self._h, _ptr(y), _ptr(cache), _ptr(x), int(x.shape[0]),
                                     C.byref(net.c), _stream(stream)))

    def mlp_backward(self, grad, dy, x, cache, net, stream=None):
        _check(lib().sdm_mlp_backward(self._h, _ptr(grad), _ptr(dy), _ptr(x), _ptr(cache),
                                      int(x.shape[0]), C.byref(net.c), _stream(stream)))

    def mlp_mse(self, dy, loss, y, t, stream=None):
        _check(lib().sdm_mlp_mse(self._h, _ptr(dy), _ptr(loss), _ptr(y), _ptr(t),
                                 int(y.shape[0]), _stream(stream)))

    def mlp_adam(self, net, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
        opt = MlpOptC(_ptr(m), _ptr(v))
        hp = AdamHpC(lr, beta1, beta2, eps, int(t), 0)
        _check(lib().sdm_mlp_adam(self._h, C.byref(net.c), C.byref(opt), _ptr(grad),
                                  C.byref(hp), _stream(stream)))

    def hull_check(self, fallback, x, lo, hi, counters=None, stream=None):
        lo_a = (C.c_float * 5)(*[float(v) for v in lo])
        hi_a = (C.c_float * 5)(*[float(v) for v in hi])
        _check(lib().sdm_hull_check(self._h, _ptr(fallback), _ptr(counters), _ptr(x),
                                    int(x.shape[0]), lo_a, hi_a, _stream(stream)))

    def ood_check(self, fallback, x, lo, hi, occ=None, glo=None, ginv=None, counters=None,
                  stream=None):
        """Joint out-of-distribution test (box + occupancy grid of
        G = round(occ.numel() ** (1/3)) cells per axis)."""
        lo_a = (C.c_float * 5)(*[float(v) for v in lo])
        hi_a = (C.c_float * 5)(*[float(v) for v in hi])
        G = 0
        glo_a = ginv_a = None
        if occ is not None:
            G = int(round(occ.numel() ** (1.0 / 3.0)))
            glo_a = (C.c_float * 3)(*[float(v) for v in glo])
            ginv_a = (C.c_float * 3)(*[float(v) for v in ginv])
        _check(lib().sdm_ood_check(self._h, _ptr(fallback), _ptr(counters), _ptr(x),
                                   int(x.shape[0]), lo_a, hi_a, _ptr(occ), G, glo_a, ginv_a,
                                   _stream(stream)))

    def seed_from_moments(self, xi, v, M, select, n_per_cell, dv, stream=None):
        _check(lib().sdm_seed_from_moments(self._h, _ptr(xi), _ptr(v), _ptr(M), _ptr(select),
                                           int(M.shape[0]), int(n_per_cell), float(dv),
                                           _stream(stream)))

    def moments_merge(self, M, M_src, select, stream=None):
        _check(lib().sdm_moments_merge(self._h, _ptr(M), _ptr(M_src), _ptr(select),
                                       int(M.shape[0]), _stream(stream)))

    def mlp_features(self, x, M, dt, kernel_id, mean, std, stream=None):
        m_a = (C.c_float * 5)(*[float(v) for v in mean])
        s_a = (C.c_float * 5)(*[float(v) for v in std])
        _check(lib().sdm_mlp_features(self._h, _ptr(x), _ptr(M), int(M.shape[0]), float(dt),
                                      int(kernel_id), m_a, s_a, _stream(stream)))

    def mlp_apply(self, M, y, dt, mean, std, fallback=None, stream=None):
        m_a = (C.c_float * 3)(*[float(v) for v in mean])
        s_a = (C.c_float * 3)(*[float(v) for v in std])
        _check(lib().sdm_mlp_apply(self._h, _ptr(M), _ptr(y), _ptr(fallback), int(M.shape[0]),
                                   float(dt), m_a, s_a, _stream(stream)))

    # ------------------------------------------------ fused timestep
    def _state(self, st):
        s = StateC()
        s.n_sd = st.n_sd
        s.n_cell = st.n_cell
        s.n_attr = st.attr.shape[0]
        s.attr_stride = _row_stride(st.attr)
        s.xi = _ptr(st.xi)
        s.attr = _ptr(st.attr)
        s.cell_id = _ptr(st.cell_id)
        s.idx = _ptr(st.idx)
        s.n_live_dev = _ptr(st.n_live)
        s.cell_start = _ptr(st.cell_start)
        s.counters_dev = _ptr(st.counters)
        s.gamma_out = _ptr(st.gamma_out)
        return s

    @staticmethod
    def _params(st, dt, k, r, dv=None, dv_per_cell=None, step_advance=None,
                expected_per_cell=0.0, events=None):
        p = StepParamsC()
        p.dt = float(dt)
        p.dv_per_cell = _ptr(dv_per_cell)
        p.dv = float(dv) if dv is not None else 0.0
        p.kernel = k
        p.rng = r
        p.step_advance = _ptr(step_advance)
        p.expected_per_cell = float(expected_per_cell)
        if events is not None:
            for i, e in enumerate(events):
                p.events[i] = None if e is None else e.cuda_event
        return p

    def prepare_step(self, st, dt, k, r, **kw):
        s = self._state(st)
        p = self._params(st, dt, k, r, **kw)
        _check(lib().sdm_prepare_step(self._h, C.byref(s), C.byref(p)))

    def step(self, st, dt, k, r, stream=None, **kw):
        s = self._state(st)
        p = self._params(st, dt, k, r, **kw)
        _check(lib().sdm_step(self._h, C.byref(s), C.byref(p), _stream(stream)))


class Batch:
    """A batch of independent runs advanced together (sdm_batch_*).

    segments: list of (offset, n_sd, dv, kernel_id, kparams, run[, table])."""

    def __init__(self, ctx, segments):
        self.ctx = ctx
        arr = (Segment * len(segments))()
        for i, seg in enumerate(segments):
            off, n, dv, kid, kp, run = seg[:6]
            arr[i].offset, arr[i].n_sd, arr[i].dv = int(off), int(n), float(dv)
            arr[i].kernel = kernel(kid, kp, seg[6] if len(seg) > 6 else None)
            arr[i].run = int(run)
        self.n_seg = len(segments)
        self._h = C.c_void_p()
        _check(lib().sdm_batch_create(ctx.handle, C.byref(self._h), arr, self.n_seg))

    def close(self):
        if self._h:
            lib().sdm_batch_destroy(self.ctx.handle, self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, st, dt, r, stream=None, **kw):
        s = self.ctx._state(st)
        p = Context._params(st, dt, kernel(0), r, dv=1.0, **kw)
        _check(lib().sdm_batch_step(self.ctx.handle, self._h, C.byref(s), C.byref(p),
                                    _stream(stream)))

    def set_schedule(self, schedule):
        n = C.c_int32(0)
        _check(lib().sdm_batch_set_schedule(self.ctx.handle, self._h, int(schedule), C.byref(n)))
        return int(n.value)

    def n_schedules(self):
        return self.set_schedule(-1)

    def autotune(self, scratch, dt, r, steps=3, cache_path=None):
        s = self.ctx._state(scratch)
        p = Context._params(scratch, dt, kernel(0), r, dv=1.0)
        chosen = C.c_int32(-1)
        _check(lib().sdm_autotune(self.ctx.handle, self._h, C.byref(s), C.byref(p), int(steps),
                                  cache_path.encode() if cache_path else None,
                                  C.byref(chosen)))
        return int(chosen.value)


class State:
    """Device state of one run (the state listing of Sec. 3.1) as torch tensors."""

    def __init__(self, xi, attr, cell_id=None, n_cell=1, device="cuda", want_gamma=False):
        import torch
        self.n_sd = int(xi.shape[0])
        self.n_cell = int(n_cell)
        self.xi = torch.as_tensor(xi, dtype=torch.uint64).to(device).contiguous()
        a = torch.as_tensor(attr, dtype=torch.float64)
        if a.dim() == 1:
            a = a[None, :]
        self.attr = a.to(device).contiguous()
        self.cell_id = (None if cell_id is None else
                        torch.as_tensor(cell_id, dtype=torch.int32).to(device).contiguous())
        self.idx = torch.arange(self.n_sd, dtype=torch.int32, device=device)
        self.n_live = torch.tensor([self.n_sd], dtype=torch.int64, device=device)
        self.cell_start = torch.zeros(self.n_cell + 1, dtype=torch.int32, device=device)
        self.counters = torch.zeros(N_COUNTERS, dtype=torch.uint64, device=device)
        self.gamma_out = (torch.zeros(max(self.n_sd // 2, 1), dtype=torch.float64, device=device)
                          if want_gamma else None)


class Mlp:
    """Device parameters of the moment surrogate: fp32 masters (flat
    W1, b1, ..., W4, b4, W row-major [out][in]) and their packed bf16 copy."""

    def __init__(self, ctx, params, device="cuda"):
        import torch
        self.params = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous()
        assert self.params.numel() == MLP_N_PARAMS
        self.packed = torch.empty(MLP_PACKED_BYTES // 4, dtype=torch.int32, device=device)
        self.c = MlpC(_ptr(self.params), _ptr(self.packed))
        ctx.mlp_pack(self)

    @staticmethod
    def cache_for(B, device="cuda"):
        import torch
        rows = (int(B) + 15) // 16 * 16
        return torch.empty(rows * MLP_CACHE_FLOATS_PER_ROW, dtype=torch.float32, device=device)
