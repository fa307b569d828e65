"""The learned part end to end at reduced size: training pairs from replica
means of the particle method (4 x 64 grid cells, 32 realisations, 120 s),
training with the library's forward / backward / Adam kernels, and an
evaluation against a 256-member mean of 16 other cells, with the
out-of-distribution test and the particle fallback in the loop.  The
network must reduce its training loss and predict each cell's M0 and M2 at
120 s better than both baselines: a single particle run (the method without
the network) and the mean training tendency applied to every cell; M1 stays
conserved.  Everything is seeded and the GPU path is deterministic."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_pipeline_small():
    import torch
    assert torch.cuda.is_available()
    from paper_2101_06318_amd import surrogate
    ev, sur, ctx = surrogate.pipeline(torch, log=None, epochs=8, m=1,
                                      train_seeds=range(100, 104), train_nx=8, train_ny=8,
                                      train_R=32,
                                      eval_nx=4, eval_R=64, eval_launches=4, t_end=120.0)
    losses = ev["losses"]
    assert ev["train_samples"] > 25000
    assert losses[-1] < losses[0], losses
    assert ev["members"] == 256 and ev["ref_rel_se"][2] < 0.05, ev
    assert ev["fallback_fraction"] < 0.05, ev
    es, e1, ec = ev["err_surrogate"], ev["err_single_sdm"], ev["err_constant_tendency"]
    for k in (0, 2):
        assert es[k] < e1[k] and es[k] < ec[k], ev
    assert es[1] < 1e-8, ev          # M1: conserved (up to the fallback's rounding)
    assert np.all(np.isfinite(es)), ev
    ctx.close()
