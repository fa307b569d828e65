"""Golovin validation (Sec. 4, eq. 7 of arXiv:2101.06318).

1. The closed-form module itself: eq. (7) integrated numerically reproduces
   the moment solutions of the additive-kernel Smoluchowski equation.
2. The oracle's SDM runs of the paper's box set-up reproduce those moments
   and the smoothed mass spectrum, within calibrated statistical bounds.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import golovin
from paper_2101_06318_amd import workloads

N0, B, VBAR = workloads.BOX_N0, workloads.GOLOVIN_B, workloads.BOX_VBAR


def test_tau_values():
    # N0 b vbar = 1.500006e-3 s^-1; 1 - tau at 1200/2400/3600 s
    assert abs(N0 * B * VBAR - 1.500006e-3) < 1e-9
    ref = {1200: 0.1652978, 2400: 0.02732336, 3600: 0.004516491}
    for t, v in ref.items():
        assert abs((1 - golovin.tau(t, N0, B, VBAR)) / v - 1) < 1e-6


@pytest.mark.parametrize("t", [600.0, 1200.0, 3600.0])
def test_eq7_moments_by_quadrature(t):
    # integrate in y = ln(v / vbar); the late-time tail reaches ~1e6 vbar
    f0 = lambda x: golovin.phi(x * VBAR, t, N0, B, VBAR) * VBAR

    def integral(k):
        g = lambda y: np.exp(y) ** (k + 1) * f0(np.exp(y))
        return sum(quad(g, a, b, limit=400, epsabs=0)[0]
                   for a, b in ((-40, -5), (-5, 0), (0, 5), (5, 10), (10, 17)))
    m0, m1, m2 = integral(0), integral(1), integral(2)
    M0, M1, M2 = golovin.moments(t, N0, B, VBAR)
    assert abs(m0 * N0 / M0 - 1) < 1e-6
    assert abs(m1 * N0 * VBAR / M1 - 1) < 1e-6       # mass conserved by eq. (7)
    assert abs(m2 * N0 * VBAR ** 2 / M2 - 1) < 1e-5


def test_eq7_reduces_to_exponential_at_start():
    v = np.linspace(0.1, 8, 50) * VBAR
    ref = np.exp(-v / VBAR) / VBAR
    got = golovin.phi(v, 1e-6, N0, B, VBAR)
    assert np.allclose(got, ref, rtol=1e-4)


def _run(oracle_mod, n_sd, seed, t_end, snap):
    w = workloads.box(n_sd, seed)
    st = dict(xi=w["xi"], attr=w["attr"], idx=np.arange(n_sd, dtype=np.uint32), n_live=n_sd)
    out = {}
    for t in range(t_end):
        st = oracle_mod.step(st["xi"], st["attr"], w["cell_id"], 1, w["dv"], st["idx"],
                             st["n_live"], dt=1.0, kernel_id=oracle_mod.KERNEL_GOLOVIN,
                             kparams=[B], seed=seed, run=0, step=t)
        if t + 1 in snap:
            out[t + 1] = dict(M=oracle_mod.moments(st["xi"], st["attr"][0], w["cell_id"],
                                                   st["idx"], st["n_live"], 1, w["dv"])[0],
                              xi=st["xi"].copy(), v=st["attr"][0].copy())
    M0 = oracle_mod.moments(w["xi"], w["attr"][0], w["cell_id"], np.arange(n_sd, dtype=np.uint32),
                            n_sd, 1, w["dv"])[0]
    return M0, out


def test_oracle_golovin_moments(oracle_mod):
    """Ensemble of 4 oracle runs (2^11 SDs, 3600 steps): M0/N0 and
    M2/M2(0) against the closed form within 3 sigma_ens/sqrt(4) plus 1 %
    (M0) or 5 % (M2); M1 conserved to 1e-12."""
    snaps = (1200, 2400, 3600)
    r0, r2 = {t: [] for t in snaps}, {t: [] for t in snaps}
    for seed in range(1, 5):
        M_init, out = _run(oracle_mod, 2048, seed, 3600, snaps)
        for t in snaps:
            M = out[t]["M"]
            r0[t].append(M[0] / N0)
            r2[t].append(M[2] / M_init[2])
            assert abs(M[1] / M_init[1] - 1) < 1e-12
    for t in snaps:
        m0, m1, m2 = golovin.moments(t, N0, B, VBAR)
        a0, a2 = np.array(r0[t]), np.array(r2[t])
        ref0, ref2 = m0 / N0, m2 / (2 * N0 * VBAR ** 2)
        assert abs(a0.mean() - ref0) < 3 * a0.std(ddof=1) / 2 + 0.01 * ref0, (t, a0, ref0)
        assert abs(a2.mean() - ref2) < 3 * a2.std(ddof=1) / 2 + 0.05 * ref2, (t, a2, ref2)


def test_oracle_golovin_spectrum(oracle_mod):
    """Smoothed dm/dlnr of 4 oracle runs (2^13 SDs) at t = 1200 s against
    eq. (7): L1 distance over the bins that hold 99 % of the analytic mass
    <= 10 % of that mass."""
    edges = golovin.radius_bins()
    specs = []
    for seed in range(1, 5):
        _, out = _run(oracle_mod, 8192, seed, 1200, (1200,))
        specs.append(golovin.sdm_spectrum(out[1200]["xi"], out[1200]["v"], workloads.BOX_DV, edges))
    sdm = golovin.smooth(np.mean(specs, axis=0))
    ana = golovin.analytic_spectrum(1200.0, N0, B, VBAR, edges)
    order = np.argsort(ana)[::-1]
    keep = order[: np.searchsorted(np.cumsum(ana[order]) / ana.sum(), 0.99) + 1]
    l1 = np.abs(sdm[keep] - ana[keep]).sum() / ana[keep].sum()
    assert l1 < 0.10, l1
