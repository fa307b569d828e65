"""GPU parity of the O(n) per-cell permutations (Fisher-Yates and
MergeShuffle, Sec. 3.2) against the oracle, bit for bit: the permuted
Index and the cell starts, for single cells of many sizes and for
multi-cell layouts with a scrambled incoming order."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, host, zeros

pytestmark = pytest.mark.gpu
METHODS = {"fisher_yates": 1, "merge": 2}


@pytest.fixture(scope="module")
def sdm():
    import torch
    assert torch.cuda.is_available()
    import paper_2101_06318_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(sdm):
    c = sdm.Context(40000, 20000, 1)
    yield c
    c.close()


def _check(sdm, ctx, method, idx, n_live, cid, n_cell, seed, run, step, step_dev=None):
    import torch
    d_idx = dev(idx)
    d_cs = zeros(n_cell + 1, torch.int32)
    sd = None if step_dev is None else dev(np.array([step_dev], np.uint32))
    r = sdm.rng(seed, run, step, step_dev=sd)
    ctx.shuffle_variant(METHODS[method], d_cs, d_idx, dev(np.array([n_live], np.int64)),
                        dev(cid), n_cell, r)
    torch.cuda.synchronize()
    ref_idx, ref_cs = oracle.shuffle_variant(method, idx, n_live, cid, n_cell, seed, run,
                                             step if step_dev is None else step_dev)
    assert np.array_equal(host(d_cs, np.uint32), ref_cs)
    assert np.array_equal(host(d_idx, np.uint32)[:n_live], ref_idx[:n_live])


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("n", [1, 2, 16, 17, 33, 1000, 20011])
def test_single_cell(sdm, ctx, method, n):
    idx = np.random.default_rng(n).permutation(n).astype(np.uint32)
    _check(sdm, ctx, method, idx, n, np.zeros(n, np.int32), 1, 77, 3, 5)


@pytest.mark.parametrize("method", list(METHODS))
def test_grid_cells_and_device_step(sdm, ctx, method):
    from paper_2101_06318_amd import workloads
    w = workloads.grid(seed=6, nx=16, ny=16)
    n = w["n_sd"]
    idx = np.random.default_rng(2).permutation(n).astype(np.uint32)
    _check(sdm, ctx, method, idx, n, w["cell_id"], w["n_cell"], 5, 0, 0, step_dev=41)


@pytest.mark.parametrize("method", list(METHODS))
def test_partial_index(sdm, ctx, method):
    """Only idx[0:n_live] takes part (SDs removed at Step 0 are absent)."""
    rng = np.random.default_rng(9)
    n_sd, n_cell = 30000, 9
    cid = rng.integers(0, n_cell, n_sd).astype(np.int32)
    idx = rng.permutation(n_sd).astype(np.uint32)
    _check(sdm, ctx, method, idx, 24001, cid, n_cell, 123, 7, 2)
