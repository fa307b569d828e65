"""The learned part end to end at reduced size (32 x 32 static cells, 120 s):
training pairs from the particle method, training with the library's
forward / backward / Adam kernels, and evaluation against an 8-member SDM
ensemble.  The trained network must reduce its training loss, stay inside
its input hull almost everywhere, and be closer to the ensemble mean than a
single particle run (the method without it) for M0 and M2 while conserving
M1.  Everything is seeded and the GPU path is deterministic."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_pipeline_small():
    import torch
    assert torch.cuda.is_available()
    from paper_2101_06318_amd import surrogate
    rep, sur, ctx = surrogate.pipeline(torch, log=None, epochs=10, nx=32, eval_members=8,
                                       ensemble=False, t_end=120.0, eval_every=(1,))
    ev = rep["runs"][0]
    losses = ev["losses"]
    assert ev["train_samples"] > 50000
    assert losses[-1] < losses[0], losses
    assert ev["fallback_fraction"] < 0.01, rep
    es, e1 = ev["err_surrogate"], ev["err_single_sdm"]
    assert es[0] < e1[0] and es[2] < e1[2], rep
    assert es[1] < 1e-12 and e1[1] < 1e-12, rep          # M1 (mass) is conserved
    assert np.all(np.isfinite(es)), rep
    ctx.close()
