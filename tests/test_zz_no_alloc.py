"""The allocation-free Step 0 entry point (sdm_remove_if_equal_0_noalloc,
for callers that cannot allocate) gives, through the C ABI, exactly what
sdm_remove_if_equal_0 gives with a context: two calls in a row on the
library's shared fixed scratch, the second on a smaller Index."""
import numpy as np
import pytest

from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _case(n_sd, n_live, seed):
    rng = np.random.default_rng(seed)
    xi = rng.integers(1, 10, n_sd).astype(np.uint64)
    xi[rng.random(n_sd) < 0.3] = 0
    idx = rng.permutation(n_sd).astype(np.uint32)
    return idx, n_live, xi


def _with_ctx(sdm, ctx, idx, n_live, xi):
    d_idx, d_n, d_xi = dev(idx), dev(np.array([n_live], np.int64)), dev(xi)
    ctx.remove_if_equal_0(d_idx, d_n, d_xi)
    return d_idx, d_n


def _no_alloc(sdm, idx, n_live, xi):
    d_idx, d_n, d_xi = dev(idx), dev(np.array([n_live], np.int64)), dev(xi)
    sdm.remove_if_equal_0_noalloc(d_idx, d_n, d_xi)
    return d_idx, d_n


def test_no_alloc_matches_context_entry_point_twice():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as sdm
    cases = [_case(1_000_003, 999_000, 1), _case(70_001, 70_001, 2)]
    ctx = sdm.Context(1_000_003, 1, 2)
    try:
        for idx, n_live, xi in cases:
            a_idx, a_n = _no_alloc(sdm, idx, n_live, xi)
            b_idx, b_n = _with_ctx(sdm, ctx, idx, n_live, xi)
            torch.cuda.synchronize()
            n = int(host(b_n)[0])
            assert int(host(a_n)[0]) == n
            assert n == int(np.count_nonzero(xi[idx[:n_live]]))
            assert np.array_equal(host(a_idx, np.uint32)[:n], host(b_idx, np.uint32)[:n])
            # entries past the new live count are left as they were
            assert np.array_equal(host(a_idx, np.uint32)[n_live:], idx[n_live:])
    finally:
        ctx.close()


def test_no_alloc_rejects_sizes_beyond_its_scratch():
    import paper_2101_06318_amd as sdm
    lib = sdm.lib()
    big = sdm.NOALLOC_MAX_IDS + 1
    assert lib.sdm_remove_if_equal_0_noalloc(1, 1, 1, big, None) == -1
    assert b"n_sd_max" in lib.sdm_last_error()
    assert lib.sdm_remove_if_equal_0_noalloc(1, 1, 1, 0, None) == -1
    assert lib.sdm_remove_if_equal_0_noalloc(None, 1, 1, 5, None) == -1
