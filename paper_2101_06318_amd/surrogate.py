"""Moment surrogate: training data from the particle method, training with
the library's own kernels, and its evaluation against an SDM ensemble.

The paper's outlook (arXiv:2101.06318, Sec. 5) notes that a fluid solver
coupled to the particle method needs only statistical moments of the
spectrum.  Here a network learns, per cell, the relative tendencies of the
moments M_k = sum xi v^k / dV (k = 0, 1, 2) over one timestep from the
cell's own moments, dt and the kernel; the particle method produces its
training data, serves as its fallback outside the training inputs' box,
and measures its error.  Every arithmetic step (particle steps, moments,
features, hull test, forward, backward, loss, Adam, moment update) runs in
the HIP library; torch holds device memory and draws minibatch orders.

Workloads (seeded, synthetic), for a surrogate step of m seconds:
  * grid: 128 x 128 cells of the gravitational-kernel grid (static cells:
    every cell is an independent box), dt = 1 s over 600 s, tendencies over
    m seconds;
  * ensemble: the 1024 Golovin / gravitational boxes of 2^8..2^16 SDs,
    dt = 1 s over 600 s, tendencies over m seconds.
Evaluation: SDM on the grid with dt = 1 s for 600 s, the surrogate in steps
of m seconds; the reference is the mean over a 16-member SDM ensemble
(seeds 1001..1016) of each cell's moments; a further member (seed 1017)
gives the error of a single particle run.
"""
from __future__ import annotations

import math

import numpy as np

from . import Batch, Context, Mlp, State, kernel, rng, workloads

N_FEAT = 5


def _moments(ctx, torch, st, n_cell, dv_per_cell=None, dv=0.0):
    M = torch.zeros((n_cell, 3), dtype=torch.float64, device="cuda")
    ctx.moments(M, st.xi, st.attr[0], st.idx, st.cell_start, n_cell, dv_per_cell=dv_per_cell,
                dv=dv)
    return M


def _sorted_by_cell(ctx, st):
    """idx / cell_start of a fresh state (before its first step)."""
    ctx.cell_sort(st.cell_start, st.idx, st.n_live, st.cell_id, st.n_cell)


def grid_pairs(ctx, torch, seed, lags=(1, 10), t_end=600.0, stride=10, nx=128, dt=1.0):
    """One static-cell grid run at dt; for every lag K the pairs (moments at
    step t, moments at step t + K) for t = 0, stride, 2 stride, ... give the
    raw features (log M(t), K dt, kernel id) and the relative tendencies over
    K dt.  Returns {K: (X, T)} (host arrays)."""
    w = workloads.grid(seed=seed, nx=nx, ny=nx)
    n_cell = w["n_cell"]
    st = State(w["xi"], w["attr"], w["cell_id"], n_cell)
    dvc = torch.as_tensor(np.asarray(w["dv"], np.float64)).cuda()
    k = kernel(w["kernel_id"], w["kparams"])
    _sorted_by_cell(ctx, st)
    n_steps = int(round(t_end / dt))
    hist = [_moments(ctx, torch, st, n_cell, dvc)]
    for t in range(n_steps):
        ctx.step(st, dt, k, rng(seed, 0, t), dv_per_cell=dvc)
        hist.append(_moments(ctx, torch, st, n_cell, dvc))
    kid = torch.full((n_cell,), float(w["kernel_id"]), dtype=torch.float64, device="cuda")
    return _lag_pairs(torch, hist, kid, lags, stride, dt)


def ensemble_pairs(ctx_big, torch, seed, lags=(1, 10), t_end=600.0, stride=10, n_runs=1024,
                   dt=1.0):
    """The batched ensemble (every run a box), pairs at several lags as in
    grid_pairs; moments from the state after each step."""
    ens = workloads.ensemble(seed=seed, n_runs=n_runs)
    xi, attr, segs = workloads.ensemble_layout(ens)
    st = State(xi, attr, None, len(segs))
    ctx = Context(st.n_sd, len(segs), 1)
    b = Batch(ctx, segs)
    kid = torch.as_tensor(np.array([s_[3] for s_ in segs], np.float64)).cuda()
    n_steps = int(round(t_end / dt))
    hist = []
    for t in range(n_steps):
        b.step(st, dt, rng(seed, 0, t))
        hist.append(_moments(ctx, torch, st, len(segs), dv=workloads.BOX_DV))
    b.close()
    ctx.close()
    return _lag_pairs(torch, hist, kid, lags, stride, dt)


def _lag_pairs(torch, hist, kid, lags, stride, dt):
    out = {}
    for K in lags:
        X, T = [], []
        for t in range(0, len(hist) - K, stride):
            M, M1 = hist[t], hist[t + K]
            X.append(torch.stack([torch.log(M[:, 0]), torch.log(M[:, 1]), torch.log(M[:, 2]),
                                  torch.full_like(M[:, 0], K * dt), kid], 1).cpu().numpy())
            T.append(((M1 - M) / (M * (K * dt))).cpu().numpy())
        out[K] = (np.concatenate(X), np.concatenate(T))
    return out


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
    """Trained network plus its input / target standardisation and hull."""

    def __init__(self, ctx, params, x_mean, x_std, t_mean, t_std, lo, hi):
        self.ctx = ctx
        self.net = Mlp(ctx, params)
        self.x_mean, self.x_std = np.float32(x_mean), np.float32(x_std)
        self.t_mean, self.t_std = np.float32(t_mean), np.float32(t_std)
        self.lo, self.hi = np.float32(lo), np.float32(hi)

    def step(self, torch, M, dt, kernel_id, bufs=None, counters=None):
        """Advances the moments M [n][3] (device float64) by one timestep;
        returns the fallback mask (cells left to the particle method)."""
        n = M.shape[0]
        if bufs is None:
            bufs = dict(x=torch.zeros((n, N_FEAT), dtype=torch.float32, device="cuda"),
                        y=torch.zeros((n, 3), dtype=torch.float32, device="cuda"),
                        fb=torch.zeros(n, dtype=torch.uint8, device="cuda"))
        c = self.ctx
        c.mlp_features(bufs["x"], M, dt, kernel_id, self.x_mean, self.x_std)
        c.hull_check(bufs["fb"], bufs["x"], self.lo, self.hi, counters=counters)
        c.mlp_forward(bufs["y"], bufs["x"], self.net)
        c.mlp_apply(M, bufs["y"], dt, self.t_mean, self.t_std, fallback=bufs["fb"])
        return bufs["fb"]


def train(ctx, torch, Xraw, Traw, epochs=20, batch=4096, lr=1e-3, seed=7, log=None):
    """Standardises, trains on the GPU (forward, MSE, backward, Adam kernels)
    and returns (Surrogate, per-epoch mean losses)."""
    # statistics as float32 values and the standardisation in float64 from
    # them: the arithmetic of sdm_mlp_features, so that inputs seen at run
    # time fall inside the hull exactly where the training inputs did
    x_mean = np.float32(Xraw.mean(0))
    x_std = np.float32(Xraw.std(0))
    x_std[x_std == 0] = 1.0
    t_mean = np.float32(Traw.mean(0))
    t_std = np.float32(Traw.std(0))
    t_std[t_std == 0] = 1.0
    X = ((Xraw - x_mean.astype(np.float64)) / x_std.astype(np.float64)).astype(np.float32)
    T = ((Traw - t_mean.astype(np.float64)) / t_std.astype(np.float64)).astype(np.float32)
    lo, hi = X.min(0), X.max(0)
    sur = Surrogate(ctx, workloads.mlp_init(seed), x_mean, x_std, t_mean, t_std, lo, hi)
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
        for i in range(nb):
            sel = perm[i * batch:(i + 1) * batch]
            xb = Xd[sel].contiguous()
            tb = Td[sel].contiguous()
            ctx.mlp_forward(y, xb, net, cache=cache)
            ctx.mlp_mse(dy, loss, y, tb)
            ctx.mlp_backward(grad, dy, xb, cache, net)
            t += 1
            ctx.mlp_adam(net, m, v, grad, t, lr=lr)
            acc += loss
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log("epoch %d loss %.5f" % (ep, losses[-1]))
    return sur, losses


def evaluate(ctx, torch, sur, seeds=range(1001, 1017), held_out=1017, t_end=600.0, dt=1.0,
             nx=128, grid_seed=3, sur_every=1):
    """Surrogate vs SDM ensemble mean on the static-cell grid.  Every member
    and the surrogate start from the same initial state (grid seed); members
    differ in their Philox seed.  The surrogate takes steps of sur_every * dt;
    fallback cells take the held-out member's particle-method tendency over
    that step."""
    w = workloads.grid(seed=grid_seed, nx=nx, ny=nx)
    n_cell = w["n_cell"]
    dvc = torch.as_tensor(np.asarray(w["dv"], np.float64)).cuda()
    k = kernel(w["kernel_id"], w["kparams"])
    n_steps = int(round(t_end / dt))

    def member(seed, hook=None):
        st = State(w["xi"], w["attr"], w["cell_id"], n_cell)
        _sorted_by_cell(ctx, st)
        M = _moments(ctx, torch, st, n_cell, dvc)
        M0 = M.clone()
        for t in range(n_steps):
            ctx.step(st, dt, k, rng(seed, 0, t), dv_per_cell=dvc)
            M1 = _moments(ctx, torch, st, n_cell, dvc)
            if hook:
                hook(t, M, M1)
            M = M1
        return M0, M

    ens = []
    for s_ in seeds:
        _, Mf = member(s_)
        ens.append(Mf)
    ens = torch.stack(ens)
    M_ens = ens.mean(0)
    # standard error of the ensemble mean itself, relative, averaged over cells
    sem = (ens.std(0) / math.sqrt(ens.shape[0]) / M_ens).mean(0).cpu().numpy()

    # surrogate with the held-out member supplying fallback tendencies
    state = {}
    bufs = dict(x=torch.zeros((n_cell, N_FEAT), dtype=torch.float32, device="cuda"),
                y=torch.zeros((n_cell, 3), dtype=torch.float32, device="cuda"),
                fb=torch.zeros(n_cell, dtype=torch.uint8, device="cuda"))
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    dt_sur = sur_every * dt

    def hook(t, Mp, Mp1):
        if "M" not in state:
            state["M"] = Mp.clone()
            state["Mref"] = Mp.clone()   # the held-out member at the last surrogate step
        if (t + 1) % sur_every:
            return
        Ms = state["M"]
        before = Ms.clone()
        fb = sur.step(torch, Ms, dt_sur, w["kernel_id"], bufs, counters=counters)
        sel = fb.bool()
        if bool(sel.any()):
            Ms[sel] = before[sel] * (Mp1[sel] / state["Mref"][sel])
        state["Mref"] = Mp1.clone()

    _, M_single = member(held_out, hook)
    M_sur = state["M"]

    def rel_err(A):
        return (torch.abs(A - M_ens) / M_ens).mean(0).cpu().numpy()

    def domain_err(A):
        # error of the domain mean (the sum over cells): the surrogate's bias
        # without the per-cell sampling noise of a finite ensemble
        return (torch.abs(A.sum(0) - M_ens.sum(0)) / M_ens.sum(0)).cpu().numpy()

    fallback_frac = int(counters[5].item()) / float(n_cell * (n_steps // sur_every))
    return dict(err_surrogate=rel_err(M_sur).tolist(), err_single_sdm=rel_err(M_single).tolist(),
                domain_err_surrogate=domain_err(M_sur).tolist(),
                domain_err_single_sdm=domain_err(M_single).tolist(),
                ensemble_mean_rel_sem=sem.tolist(), fallback_fraction=fallback_frac,
                members=int(ens.shape[0]), t_end=t_end, cells=n_cell, dt_surrogate=dt_sur)


def pipeline(torch, log=print, epochs=20, nx=128, eval_members=16, ensemble=True, t_end=600.0,
             grid_seeds=(100, 101, 102), eval_every=(1, 10), stride=None):
    """For each surrogate step m dt in eval_every (dt = 1 s): pairs at lag m
    from three grid runs and the ensemble (about 3e6 cell-steps), a network
    trained on them, and its evaluation at that step.  One network per step
    size: fitted jointly over several lags, the low-noise long-lag targets
    (where runaway growth has already sped up the rates) pull the short-lag
    prediction up.  Returns (report, {m: surrogate}, context)."""
    if log is None:
        def log(_msg):
            return None
    w = workloads.grid(seed=3, nx=nx, ny=nx)
    ctx = Context(w["n_sd"] + 1024, max(w["n_cell"], 1024), 2)
    lags = tuple(eval_every)
    data = {K: ([], []) for K in lags}
    if stride is None:
        stride = max(1, int(round(t_end / 60)))
    parts = [grid_pairs(ctx, torch, seed=sd, lags=lags, t_end=t_end, stride=stride, nx=nx)
             for sd in grid_seeds]
    if ensemble:
        parts.append(ensemble_pairs(ctx, torch, seed=200, lags=lags, t_end=t_end, stride=stride))
    for part in parts:
        for K in lags:
            data[K][0].append(part[K][0])
            data[K][1].append(part[K][1])
    rep = dict(runs=[])
    surs = {}
    for K in lags:
        X = np.concatenate(data[K][0])
        T = np.concatenate(data[K][1])
        log("step %g s: %d samples" % (K, len(X)))
        sur, losses = train(ctx, torch, X, T, epochs=epochs, log=log)
        ev = evaluate(ctx, torch, sur, seeds=range(1001, 1001 + eval_members),
                      held_out=1001 + eval_members, nx=nx, t_end=t_end, sur_every=K)
        ev.update(train_samples=int(len(X)), losses=losses)
        rep["runs"].append(ev)
        surs[K] = sur
    return rep, surs, ctx


if __name__ == "__main__":
    import argparse
    import json
    import sys
    import time

    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the moment surrogate")
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--members", type=int, default=16)
    ap.add_argument("--t-end", type=float, default=600.0)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--grid-runs", type=int, default=3)
    ap.add_argument("--stride", type=int, default=None)
    a = ap.parse_args()
    t0 = time.time()
    rep, _, _ = pipeline(torch, log=lambda m: print(m, file=sys.stderr, flush=True),
                         epochs=a.epochs, nx=a.nx, eval_members=a.members,
                         ensemble=not a.no_ensemble, t_end=a.t_end,
                         grid_seeds=tuple(range(100, 100 + a.grid_runs)), stride=a.stride)
    rep["seconds"] = round(time.time() - t0, 1)
    print(json.dumps(rep), flush=True)
