"""Moment surrogate: training data from the particle method, training with
the library's own kernels, and its evaluation against the particle method.

The paper's outlook (arXiv:2101.06318, Sec. 5) notes that a fluid solver
coupled to the particle method needs only statistical moments of the
spectrum.  Here a network learns, per cell, the relative tendencies of the
moments M_k = sum xi v^k / dV (k = 0, 1, 2) over a step of m seconds from
the cell's moments, the step and the kernel.  What it predicts is the
expected evolution, the mean over the particle method's random
realisations: a cell replicated R times in one grid (its replicas share the
initial state; the random numbers, keyed by SD id, differ) gives that mean
with a standard error shrinking as 1/sqrt(R).

* Training data: mean trajectories (R = 512 realisations) of 32 x 32 grid
  cells (seeded), the pairs (moments at t, moments at t + m) for every t,
  about 6e5 cell-steps per network.
* Product path of one surrogate step (all in the HIP library): features,
  the joint out-of-distribution test (box plus an occupancy grid of the
  training inputs), bf16 MFMA forward pass, moment update; cells that fail
  the test fall back to the particle method (rebuilt from their moments,
  advanced by SDM steps, measured and merged back).  M1 is conserved by
  coagulation (eqs. 5-6 conserve sum xi v), so its predicted tendency is
  pinned to zero.
* Evaluation: 64 grid cells not in the training set, each replicated 4096
  times; the surrogate integrates each cell from its initial moments to
  600 s and is compared with the 4096-member mean (standard error about
  1 % in M2), beside two baselines: a single particle run and a predictor
  that applies the mean training tendency to every cell.
Data preparation (logs of the training moments, the replica means, the
standardisation statistics, the occupancy grid) and the evaluation's error
statistics are host / torch bookkeeping around those calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import Batch, Context, Mlp, State, kernel, rng, workloads

N_FEAT = 5
OCC_G = 32        # occupancy-grid cells per axis of the joint OOD test
FALLBACK_SDS = 64  # SDs per rebuilt cell


def _moments(ctx, torch, st, n_cell, dv_per_cell=None, dv=0.0):
    M = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")
    ctx.moments(M, st.xi, st.attr[0], st.idx, st.cell_start, n_cell, dv_per_cell=dv_per_cell,
                dv=dv)
    return M


def replica_means(ctx, torch, w, R, launches, seed0, n_steps, every=1, dt=1.0):
    """Every cell of the grid workload w advanced by the particle method in
    R * launches independent realisations (R replicas per launch, Philox
    seed seed0 + launch).  Returns the mean moments at steps 0, every,
    2 every, ..., n_steps ([T][n_cell][3], host float64), the standard
    error of the mean at the last of them, and one realisation's last
    moments (replica 0 of launch 0)."""
    W = workloads.replicate_cells(w, R)
    n_cell, nc = w["n_cell"], W["n_cell"]
    st = State(W["xi"], W["attr"], W["cell_id"], nc)
    xi0, a0 = st.xi.clone(), st.attr.clone()
    dvc = torch.as_tensor(W["dv"]).cuda()
    k = kernel(w["kernel_id"], w["kparams"])
    T = n_steps // every + 1
    acc = torch.zeros((T, n_cell, 3), dtype=torch.float64, device="cuda")
    acc2 = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")
    single = None
    for L in range(launches):
        st.xi.copy_(xi0)
        st.attr.copy_(a0)
        st.n_live.fill_(W["n_sd"])
        ctx.cell_sort(st.cell_start, st.idx, st.n_live, st.cell_id, nc)
        M = _moments(ctx, torch, st, nc, dvc).view(R, n_cell, 3)
        acc[0] += M.sum(0)
        for t in range(n_steps):
            ctx.step(st, dt, k, rng(seed0 + L, 0, t), dv_per_cell=dvc)
            if (t + 1) % every == 0:
                M = _moments(ctx, torch, st, nc, dvc).view(R, n_cell, 3)
                acc[(t + 1) // every] += M.sum(0)
        acc2 += (M * M).sum(0)
        if L == 0:
            single = M[0].clone()
    n = R * launches
    mean = acc / n
    var = torch.clamp(acc2 / n - mean[-1] * mean[-1], min=0.0) * (n / max(n - 1, 1))
    se = torch.sqrt(var / n)
    return mean.cpu().numpy(), se.cpu().numpy(), single.cpu().numpy()


def training_set(ctx, torch, lag, grid_seeds=range(100, 132), nx=8, ny=4, R=512, t_end=600.0,
                 dt=1.0):
    """Pairs (mean moments at step t, at step t + lag) of the nx * ny grid
    cells of every seed, t = 0 .. n_steps - lag: raw features (log M(t),
    lag dt, kernel id) and relative tendencies over lag dt.  The mean of a
    cell's M2 is carried by rare realisations with a runaway drop, so a mean
    over few realisations typically falls short of it: R is large."""
    n_steps = int(round(t_end / dt))
    X, T = [], []
    for sd in grid_seeds:
        w = workloads.grid(seed=sd, nx=nx, ny=ny)
        mean, _, _ = replica_means(ctx, torch, w, R, 1, 7000 + sd, n_steps, 1, dt)
        M0, M1 = mean[:-lag], mean[lag:]
        lm = np.log(M0)
        feat = np.concatenate([lm, np.full(lm.shape[:2] + (1,), lag * dt),
                               np.full(lm.shape[:2] + (1,), float(w["kernel_id"]))], axis=2)
        X.append(feat.reshape(-1, N_FEAT))
        T.append(((M1 - M0) / (M0 * (lag * dt))).reshape(-1, 3))
    return np.concatenate(X), np.concatenate(T)


class ParticleFallback:
    """The cells the surrogate cannot vouch for, advanced by the particle
    method instead: each selected cell is rebuilt from its moments as
    n_per_cell SDs (sdm_seed_from_moments), advanced by SDM steps as one
    run of a batch (sdm_batch_step; run id = cell index), measured
    (sdm_moments) and merged back into the moments (sdm_moments_merge).
    Unselected cells carry no live SDs, so they cost only their slots."""

    def __init__(self, n_cell, n_per_cell, dv, kernel_id, kparams, seed):
        import torch
        self.n_cell, self.n, self.dv, self.seed = n_cell, n_per_cell, float(dv), int(seed)
        segs = [(c * n_per_cell, n_per_cell, self.dv, kernel_id, list(kparams), c)
                for c in range(n_cell)]
        n_sd = n_cell * n_per_cell
        self.ctx = Context(n_sd, n_cell, 1)
        self.st = State(np.zeros(n_sd, np.uint64), np.zeros((1, n_sd)), None, n_cell)
        self.batch = Batch(self.ctx, segs)
        self.M = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")

    def advance(self, M, select, dt, steps, step0, stream=None):
        """M [n_cell][3] (device float64): the selected cells' moments after
        `steps` particle steps of dt from their rebuilt particles; Philox
        steps step0 .. step0 + steps - 1."""
        c, st = self.ctx, self.st
        c.seed_from_moments(st.xi, st.attr[0], M, select, self.n, self.dv, stream=stream)
        for t in range(steps):
            self.batch.step(st, dt, rng(self.seed, 0, step0 + t), stream=stream)
        c.moments(self.M, st.xi, st.attr[0], st.idx, st.cell_start, self.n_cell, dv=self.dv,
                  stream=stream)
        c.moments_merge(M, self.M, select, stream=stream)

    def close(self):
        self.batch.close()
        self.ctx.close()


class Surrogate:
    """Trained network plus its standardisation, box and occupancy grid."""

    def __init__(self, ctx, params, x_mean, x_std, t_mean, t_std, lo, hi, occ=None, glo=None,
                 ginv=None):
        self.ctx = ctx
        self.net = Mlp(ctx, params)
        self.x_mean, self.x_std = np.float32(x_mean), np.float32(x_std)
        self.t_mean, self.t_std = np.float32(t_mean), np.float32(t_std)
        self.lo, self.hi = np.float32(lo), np.float32(hi)
        self.occ, self.glo, self.ginv = occ, glo, ginv

    def buffers(self, torch, n):
        return dict(x=torch.zeros((n, N_FEAT), dtype=torch.float32, device="cuda"),
                    y=torch.zeros((n, 3), dtype=torch.float32, device="cuda"),
                    fb=torch.zeros(n, dtype=torch.uint8, device="cuda"))

    def step(self, torch, M, dt, kernel_id, bufs=None, counters=None, stream=None):
        """Advances the moments M [n][3] (device float64) by dt, except the
        cells that fail the out-of-distribution test (left unchanged; the
        returned mask marks them for the particle method)."""
        if bufs is None:
            bufs = self.buffers(torch, M.shape[0])
        c = self.ctx
        c.mlp_features(bufs["x"], M, dt, kernel_id, self.x_mean, self.x_std, stream=stream)
        c.ood_check(bufs["fb"], bufs["x"], self.lo, self.hi, self.occ, self.glo, self.ginv,
                    counters=counters, stream=stream)
        c.mlp_forward(bufs["y"], bufs["x"], self.net, stream=stream)
        c.mlp_apply(M, bufs["y"], dt, self.t_mean, self.t_std, fallback=bufs["fb"],
                    stream=stream)
        return bufs["fb"]


def train(ctx, torch, Xraw, Traw, epochs=20, batch=4096, lr=1e-3, seed=7, log=None):
    """Standardises, trains on the GPU (forward, MSE, backward, Adam kernels)
    and returns (Surrogate, per-epoch mean losses)."""
    # statistics as float32 values and the standardisation in float64 from
    # them: the arithmetic of sdm_mlp_features, so that inputs seen at run
    # time fall inside the box exactly where the training inputs did
    x_mean = np.float32(Xraw.mean(0))
    x_std = np.float32(Xraw.std(0))
    x_std[x_std == 0] = 1.0
    t_mean = np.float32(Traw.mean(0))
    t_std = np.float32(Traw.std(0))
    # M1 is conserved: its tendency is zero by construction (std 0 makes the
    # update ignore the network's M1 output)
    t_mean[1], t_std[1] = 0.0, 0.0
    safe = np.where(t_std > 0, t_std, 1.0).astype(np.float64)
    X = ((Xraw - x_mean.astype(np.float64)) / x_std.astype(np.float64)).astype(np.float32)
    T = ((Traw - t_mean.astype(np.float64)) / safe).astype(np.float32)
    T[:, 1] = 0.0
    lo, hi = X.min(0), X.max(0)
    occ, glo, ginv = _occupancy(X, lo, hi, OCC_G)
    sur = Surrogate(ctx, workloads.mlp_init(seed), x_mean, x_std, t_mean, t_std, lo, hi,
                    torch.from_numpy(occ.reshape(-1)).cuda(), glo, ginv)
    net = sur.net
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    n = X.shape[0]
    y = torch.zeros((batch, 3), dtype=torch.float32, device="cuda")
    dy = torch.zeros_like(y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cache = Mlp.cache_for(batch)
    grad = torch.zeros(net.params.numel(), dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    losses = []
    t = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = n // batch
        # a step size halved for the last third of the epochs
        rate = lr if ep < (2 * epochs) // 3 else lr / 4
        for i in range(nb):
            sel = perm[i * batch:(i + 1) * batch]
            xb = Xd[sel].contiguous()
            tb = Td[sel].contiguous()
            ctx.mlp_forward(y, xb, net, cache=cache)
            ctx.mlp_mse(dy, loss, y, tb)
            ctx.mlp_backward(grad, dy, xb, cache, net)
            t += 1
            ctx.mlp_adam(net, m, v, grad, t, lr=rate)
            acc += loss
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log("epoch %d loss %.5f" % (ep, losses[-1]))
    return sur, losses


def _occupancy(X, lo, hi, G):
    """Occupancy grid over the first three standardised features (the log
    moments): G cells per axis spanning [lo, hi]; cell index
    floor((x - lo) * G / (hi - lo)) in float32, clamped.  The occupied set
    is widened by one cell in every direction: the training inputs are
    trajectories, curves through the grid, whose neighbouring cells the
    network interpolates into."""
    lo3 = np.asarray(lo, np.float32)[:3]
    hi3 = np.asarray(hi, np.float32)[:3]
    span = np.where(hi3 > lo3, hi3 - lo3, np.float32(1.0)).astype(np.float32)
    ginv = (np.float32(G) / span).astype(np.float32)
    k = np.clip(np.floor((X[:, :3] - lo3) * ginv).astype(np.int64), 0, G - 1)
    occ = np.zeros((G + 2, G + 2, G + 2), np.uint8)
    occ[k[:, 0] + 1, k[:, 1] + 1, k[:, 2] + 1] = 1
    wide = np.zeros((G, G, G), np.uint8)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                wide |= occ[a:a + G, b:b + G, c:c + G]
    return wide, lo3, ginv


def evaluate(ctx, torch, sur, m, eval_seed=3, nx=8, R=256, launches=16, t_end=600.0,
             dt=1.0, fallback=True, t_mean_raw=None):
    """The surrogate (steps of m dt) against the mean of R * launches particle
    realisations of each of the nx * nx cells of a grid not used in training,
    at t_end; beside a single realisation and the constant mean tendency
    t_mean_raw (relative, per second) applied to every cell."""
    w = workloads.grid(seed=eval_seed, nx=nx, ny=nx)
    n_cell = w["n_cell"]
    n_steps = int(round(t_end / dt))
    ref, se, single = replica_means(ctx, torch, w, R, launches, 1001, n_steps, m, dt)
    M_ref = ref[-1]
    # the surrogate from each cell's initial moments (the same as every
    # replica's: ref[0])
    M = torch.as_tensor(ref[0].copy()).cuda()
    bufs = sur.buffers(torch, n_cell)
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    fb_run = (ParticleFallback(n_cell, FALLBACK_SDS, float(w["dv"][0]), w["kernel_id"],
                               w["kparams"], seed=9001) if fallback else None)
    n_sur = n_steps // m
    fb_cells = 0
    traj = [ref[0].copy()]
    for s_ in range(n_sur):
        mask = sur.step(torch, M, m * dt, w["kernel_id"], bufs, counters)
        if fb_run is not None:
            nfb = int(mask.sum().item())
            if nfb:
                fb_cells += nfb
                fb_run.advance(M, mask, dt, m, s_ * m)
        traj.append(M.cpu().numpy())
    if fb_run is not None:
        fb_run.close()
    M_sur = traj[-1]
    # the constant-tendency baseline
    M_c = ref[0].copy()
    if t_mean_raw is not None:
        for _ in range(n_sur):
            M_c = M_c * (1.0 + (m * dt) * np.asarray(t_mean_raw, np.float64))

    def rel(A):
        return (np.abs(A - M_ref) / M_ref).mean(0).tolist()

    # per-cell M2 error along the way, and the error of the domain totals
    # (free of the per-cell scatter: the surrogate's bias)
    marks = [k for k in (n_sur // 10, n_sur // 2, n_sur) if k > 0]
    along = {str(k * m * dt): float((np.abs(traj[k][:, 2] - ref[k][:, 2]) / ref[k][:, 2]).mean())
             for k in marks}
    dom = (np.abs(M_sur.sum(0) - M_ref.sum(0)) / M_ref.sum(0)).tolist()
    out = dict(err_surrogate=rel(M_sur), err_single_sdm=rel(single),
               err_m2_along=along, domain_err_surrogate=dom,
               domain_err_single_sdm=(np.abs(single.sum(0) - M_ref.sum(0)) /
                                      M_ref.sum(0)).tolist(),
               err_constant_tendency=rel(M_c) if t_mean_raw is not None else None,
               ref_rel_se=(se / M_ref).mean(0).tolist(),
               members=R * launches, cells=n_cell, t_end=t_end, dt_surrogate=m * dt,
               surrogate_steps=n_sur,
               fallback_fraction=fb_cells / float(n_cell * n_sur),
               ood_rows=int(counters[5].item()))
    # members an SDM ensemble needs for the surrogate's M2 error: the
    # single run's per-cell error falls as 1/sqrt(members)
    e_s, e_1 = out["err_surrogate"][2], out["err_single_sdm"][2]
    out["equivalent_members_m2"] = (e_1 / e_s) ** 2 if e_s > 0 else None
    return out


def pipeline(torch, log=print, epochs=20, m=1, train_seeds=range(100, 132), train_nx=8,
             train_ny=4, train_R=512, eval_nx=8, eval_R=256, eval_launches=16, t_end=600.0):
    """Training data, training and evaluation for a surrogate step of m
    seconds.  Returns (report, surrogate, context)."""
    if log is None:
        def log(_msg):
            return None
    big = max(workloads.grid(seed=s_, nx=train_nx, ny=train_ny)["n_sd"] * train_R
              for s_ in train_seeds)
    wev = workloads.grid(seed=3, nx=eval_nx, ny=eval_nx)
    big = max(big, wev["n_sd"] * eval_R) + 1024
    ctx = Context(big, 1 << 14, 2)
    X, T = training_set(ctx, torch, m, grid_seeds=train_seeds, nx=train_nx, ny=train_ny,
                        R=train_R, t_end=t_end)
    log("step %d s: %d training samples" % (m, len(X)))
    sur, losses = train(ctx, torch, X, T, epochs=epochs, log=log)
    t_mean_raw = T.mean(0)
    t_mean_raw[1] = 0.0
    ev = evaluate(ctx, torch, sur, m, nx=eval_nx, R=eval_R, launches=eval_launches,
                  t_end=t_end, t_mean_raw=t_mean_raw)
    ev.update(train_samples=int(len(X)), losses=losses)
    ev["gate_m2_5pct"] = ev["err_surrogate"][2] <= 0.05
    return ev, sur, ctx


if __name__ == "__main__":
    import argparse
    import json
    import sys
    import time

    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the moment surrogate")
    ap.add_argument("--m", type=int, default=1, help="surrogate step in seconds")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--eval-launches", type=int, default=16)
    a = ap.parse_args()
    t0 = time.time()
    rep, _, ctx = pipeline(torch, log=lambda s_: print(s_, file=sys.stderr, flush=True),
                           epochs=a.epochs, m=a.m, eval_launches=a.eval_launches)
    rep["seconds"] = round(time.time() - t0, 1)
    ctx.close()
    print(json.dumps(rep), flush=True)
