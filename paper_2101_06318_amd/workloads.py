"""Seeded synthetic inputs for the coagulation workloads.

This module only draws initial states (numpy's PCG64 generator) with the
shapes and distributions of the paper's validation case and of the
throughput workloads built on it.  It holds none of the method's
arithmetic: no shuffle, no pair probability, no collision.  Both the HIP
library's tests and the oracle's tests take their inputs from here.

Box (Sec. 4 of arXiv:2101.06318): volume 1e6 m^3, N0 = 2^23 m^-3,
exponential volume distribution with mean vbar = (4 pi / 3) (30.531 um)^3,
equal multiplicities, Golovin b = 1500 s^-1, dt = 1 s.  The paper places SDs
at quantiles within [0.001 %, 99.999 %]; here the quantile levels are drawn
at random within that range (q = 1e-5 + (1 - 2e-5) u).
"""
from __future__ import annotations

import math

import numpy as np

GOLOVIN = 0
GEOMETRIC = 1

BOX_N0 = 2.0 ** 23          # m^-3
BOX_DV = 1.0e6              # m^3
BOX_RBAR = 30.531e-6        # m
BOX_VBAR = 4.0 / 3.0 * math.pi * BOX_RBAR ** 3
GOLOVIN_B = 1500.0          # s^-1


def box(n_sd: int, seed: int, *, N0: float = BOX_N0, dv: float = BOX_DV,
        vbar: float = BOX_VBAR, b: float = GOLOVIN_B, dt: float = 1.0):
    """One well-mixed cell with the Golovin kernel (single run).

    Multiplicities are N0*dv/n_sd (an exact integer for n_sd = 2^k, k <= 23).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_sd)
    q = 1e-5 + (1.0 - 2e-5) * u
    v = -vbar * np.log1p(-q)
    total = N0 * dv
    xi0 = int(total // n_sd)
    xi = np.full(n_sd, xi0, dtype=np.uint64)
    return dict(n_sd=n_sd, n_cell=1, xi=xi, attr=v[None, :].copy(),
                cell_id=np.zeros(n_sd, np.int32), dv=np.array([dv]), dt=dt,
                kernel_id=GOLOVIN, kparams=[b, 0.0, 0.0, 0.0],
                N0=N0, vbar=vbar, b=b)


def _lognormal_volume(rng, n, median_r, sigma_g):
    r = median_r * np.exp(np.log(sigma_g) * rng.standard_normal(n))
    return 4.0 / 3.0 * math.pi * r ** 3


def grid(seed: int = 3, nx: int = 128, ny: int = 128, mean_per_cell: float = 64.0,
         n_min: int = 2, n_max: int = 512, conc: float = 1.0e8,
         dv: float = 2500.0, dt: float = 1.0, efficiency: float = 1.0):
    """2-D grid of nx*ny cells: per-cell SD count Poisson(mean) clipped to
    [n_min, n_max]; attribute row 0 = wet volume (lognormal radius, median
    10 um, sigma_g 1.5), row 1 = dry volume (lognormal radius, median
    0.04 um, sigma_g 1.4); multiplicity floor(conc*dv/n_c); geometric
    (gravitational) kernel.  SD ids are laid out cell-major.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_cell = nx * ny
    counts = np.clip(rng.poisson(mean_per_cell, n_cell), n_min, n_max).astype(np.int64)
    n_sd = int(counts.sum())
    cell_id = np.repeat(np.arange(n_cell, dtype=np.int32), counts)
    xi = np.repeat((np.floor(conc * dv / counts)).astype(np.uint64), counts)
    wet = _lognormal_volume(rng, n_sd, 10e-6, 1.5)
    dry = _lognormal_volume(rng, n_sd, 0.04e-6, 1.4)
    return dict(n_sd=n_sd, n_cell=n_cell, xi=xi, attr=np.stack([wet, dry]),
                cell_id=cell_id, dv=np.full(n_cell, dv), dt=dt,
                kernel_id=GEOMETRIC, kparams=[efficiency, 0.0, 0.0, 0.0],
                counts=counts)


def replicate_cells(w: dict, R: int, n_attr: int = 1):
    """R independent copies of every cell of the grid workload w, as one
    grid of R * n_cell cells: cell r * n_cell + c holds replica r of cell c
    (the same SDs, so with the same initial state; the particle method's
    random numbers, keyed by SD id, make the replicas independent
    realisations).  Keeps the first n_attr attribute rows."""
    n_cell = w["n_cell"]
    xi = np.tile(w["xi"], R)
    attr = np.tile(w["attr"][:n_attr], (1, R))
    cell_id = (np.tile(w["cell_id"], R) +
               np.repeat(np.arange(R, dtype=np.int64) * n_cell, w["n_sd"])).astype(np.int32)
    return dict(w, n_sd=int(xi.shape[0]), n_cell=n_cell * R, xi=xi, attr=attr,
                cell_id=cell_id, dv=np.tile(np.asarray(w["dv"], np.float64), R),
                counts=np.tile(w["counts"], R), replicas=R, base_cells=n_cell)


def with_extra_attributes(w: dict, n_attr: int, seed: int = 11):
    """The workload w with attribute rows added up to n_attr in total: row i
    >= 1 beyond w's own is a passive extensive attribute (for example the
    amount of a chemical species a droplet carries), volume times a
    lognormal per-droplet concentration (sigma_g 2, seed-drawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = w["attr"][0]
    rows = [w["attr"][i] for i in range(w["attr"].shape[0])]
    while len(rows) < n_attr:
        rows.append(v * np.exp(np.log(2.0) * rng.standard_normal(v.shape[0])))
    return dict(w, attr=np.stack(rows[:n_attr]).astype(np.float64))


def ensemble(seed: int = 4, n_runs: int = 1024, log2_min: float = 8.0,
             log2_max: float = 16.0, dt: float = 1.0, n_sd_override=None):
    """Batched ensemble of independent boxes: run r has
    n_r = round(2^(log2_min + (log2_max - log2_min) u_r)) SDs, the box
    initial state (drawn with seed*1_000_003 + r), multiplicity
    floor(N0 dV / n_r); Golovin for even r, geometric for odd r.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_runs)
    if n_sd_override is not None:
        sizes = np.asarray(n_sd_override, dtype=np.int64)
    else:
        sizes = np.rint(2.0 ** (log2_min + (log2_max - log2_min) * u)).astype(np.int64)
    runs = []
    for r in range(n_runs):
        n = int(sizes[r])
        sub = np.random.Generator(np.random.PCG64(seed * 1_000_003 + r))
        q = 1e-5 + (1.0 - 2e-5) * sub.random(n)
        v = -BOX_VBAR * np.log1p(-q)
        xi = np.full(n, int((BOX_N0 * BOX_DV) // max(n, 1)), dtype=np.uint64)
        kid = GOLOVIN if r % 2 == 0 else GEOMETRIC
        kp = [GOLOVIN_B, 0.0, 0.0, 0.0] if kid == GOLOVIN else [1.0, 0.0, 0.0, 0.0]
        runs.append(dict(n_sd=n, xi=xi, attr=v[None, :].copy(), kernel_id=kid,
                         kparams=kp, dv=BOX_DV, run=r))
    return dict(n_runs=n_runs, sizes=sizes, runs=runs, dt=dt)


def ensemble_layout(ens):
    """Concatenates the members of an ensemble into one batch state: member r
    occupies SD slots [offset_r, offset_r + n_r) with even offsets (one
    padding slot of multiplicity 0 after odd-sized members).  Returns
    (xi, attr[1, N], segments) with segments = (offset, n, dv, kernel_id,
    kparams, run)."""
    offs, off = [], 0
    for m in ens["runs"]:
        offs.append(off)
        off += m["n_sd"] + (m["n_sd"] & 1)
    n_tot = off
    xi = np.zeros(n_tot, np.uint64)
    v = np.zeros(n_tot, np.float64)
    segs = []
    for m, o in zip(ens["runs"], offs):
        n = m["n_sd"]
        xi[o:o + n] = m["xi"]
        v[o:o + n] = m["attr"][0]
        segs.append((o, n, m["dv"], m["kernel_id"], m["kparams"], m["run"]))
    return xi, v[None, :], segs



MLP_LAYERS = (5, 128, 128, 128, 3)


def mlp_init(seed: int = 7):
    """Initial parameters of the surrogate network as one flat float32
    vector (W1, b1, ..., W4, b4; W row-major [out][in]): every entry of a
    layer with fan-in f uniform in [-1/sqrt(f), 1/sqrt(f)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in zip(MLP_LAYERS[:-1], MLP_LAYERS[1:]):
        bound = 1.0 / math.sqrt(fi)
        parts.append(rng.uniform(-bound, bound, fo * fi))
        parts.append(rng.uniform(-bound, bound, fo))
    return np.concatenate(parts).astype(np.float32)
