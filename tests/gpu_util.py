"""Helpers for the GPU tests: host<->device copies with the library's dtypes."""
import numpy as np


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    if dtype is not None:
        a = a.astype(dtype)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a.copy()).to("cuda")


def host(t, dtype=None):
    a = t.detach().cpu().numpy()
    if dtype is not None:
        a = a.view(dtype)
    return a


def zeros(n, dtype):
    import torch
    return torch.zeros(int(n), dtype=dtype, device="cuda")
