"""Golovin (additive-kernel) closed form and spectrum post-processing.

TEST INFRASTRUCTURE ONLY (validation reference for the oracle and the HIP
path).  Follows the paper's validation case (Sec. 4, eq. 7): the analytic
solution of the Smoluchowski equation for a(v1, v2) = b (v1 + v2) with an
exponential initial volume distribution of mean vbar.

Reading taken (eq. 7 integrates to 1 - tau and carries no N0): the number
density per unit volume is n(v, t) = N0 * phi(v, t), and the mass density
per unit ln r is dm/dlnr = rho_w * 3 v^2 * n(v, t) with rho_w = 1000 kg/m^3.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive

RHO_W = 1000.0


def tau(t, N0, b, vbar):
    """tau(t) = 1 - exp(-N0 b vbar t)."""
    return 1.0 - np.exp(-N0 * b * vbar * t)


def phi(v, t, N0, b, vbar):
    """Eq. (7): normalised (to 1 - tau) volume spectrum at time t > 0."""
    v = np.asarray(v, dtype=np.float64)
    T = tau(t, N0, b, vbar)
    sT = np.sqrt(T)
    return ((1.0 - T) / (v * sT) * ive(1, 2.0 * v * sT / vbar)
            * np.exp(-v * (1.0 + T - 2.0 * sT) / vbar))


def moments(t, N0, b, vbar):
    """Closed-form moments of the Golovin solution (exponential start).

    M0 = N0 (1 - tau), M1 = N0 vbar (conserved), M2 = 2 N0 vbar^2 / (1 - tau)^2,
    from dM0/dt = -b M1 M0 and dM2/dt = 2 b M1 M2 for the additive kernel.
    """
    T = tau(t, N0, b, vbar)
    return N0 * (1.0 - T), N0 * vbar, 2.0 * N0 * vbar ** 2 / (1.0 - T) ** 2


def radius_bins(n_bins=100, r_min=1e-6, r_max=1e-2):
    """Log-spaced radius bin edges (a reading: ~100 bins over 1 um .. 10 mm)."""
    return np.logspace(np.log10(r_min), np.log10(r_max), n_bins + 1)


def smooth(y, width=5, passes=2):
    """Centred running mean over `width` bins, applied `passes` times
    (Sec. 4), zero-padded to the same length."""
    k = np.ones(width) / width
    for _ in range(passes):
        y = np.convolve(y, k, mode="same")
    return y


def sdm_spectrum(xi, v, dv, edges):
    """dm/dlnr [kg/m^3 per unit ln r] of a super-droplet population."""
    xi = np.asarray(xi, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    r = np.cbrt(v * 3.0 / (4.0 * np.pi))
    mass = xi * v * RHO_W / dv
    h, _ = np.histogram(r, bins=edges, weights=mass)
    return h / np.diff(np.log(edges))


def analytic_spectrum(t, N0, b, vbar, edges):
    """dm/dlnr of eq. (7) at the geometric bin centres."""
    rc = np.sqrt(edges[:-1] * edges[1:])
    vc = 4.0 / 3.0 * np.pi * rc ** 3
    return RHO_W * 3.0 * vc ** 2 * N0 * phi(vc, t, N0, b, vbar)
