"""Training and evaluation of the learned sub-step surrogate.

Orchestration only: features, targets, the network's forward and backward
passes, Adam, the surrogate step and its residual check all run in the
library's HIP kernels; torch holds the datasets on the device.

Training data comes from plain runs of the method (the kappa sub-steps): at
sampled acoustic steps the 24 features of every free solid particle are taken
between `couple` and `solid_substeps`, and the targets ((vbar - v) / (s dt),
(abar - a) / s, with the row's acceleration scale s) right after it.
"""
from __future__ import annotations

import time

import numpy as np

from . import mlp, sph

N_FEAT, N_OUT = 24, 4


def collect(scenes, steps: int, every: int = 4, warmup: int = 0, **options):
    """(X, T) device tensors of the free solid particles at every `every`-th
    acoustic step of a plain run (after `warmup` steps)."""
    import torch

    sim = sph.Simulation(scenes, **options)
    mask = torch.tensor(sim.free_mask(), device=sim.device)
    xs, ts = [], []
    for k in range(steps):
        sim.neighbor_build()
        sim.fluid_step()
        sim.couple()
        take = k >= warmup and (k - warmup) % every == 0
        if take:
            x = sim.solid_features()
        sim.solid_substeps()
        if take:
            t = sim.solid_targets()
            xs.append(x[mask])
            ts.append(t[mask])
    sim.sync()
    sim.close()
    return torch.cat(xs), torch.cat(ts)


def glorot(seed: int = 0):
    """Initial parameters: uniform Glorot weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in mlp.layer_shapes(N_FEAT, N_OUT):
        lim = np.sqrt(6.0 / (a + b))
        out.append((rng.uniform(-lim, lim, size=(a, b)).astype(np.float32), np.zeros(b, np.float32)))
    return out


def standardise(X, T):
    """Column mean and 1/std of the features, mean and std of the targets
    (constant columns get unit scale); the 56 floats sph_set_surrogate takes."""
    mx, sx = X.mean(0), X.std(0)
    mt, st = T.mean(0), T.std(0)
    sx = torch_where_small(sx)
    st = torch_where_small(st)
    stats = np.concatenate([mx.cpu().numpy(), (1.0 / sx).cpu().numpy(), mt.cpu().numpy(), st.cpu().numpy()])
    return stats.astype(np.float32), mx, sx, mt, st


def torch_where_small(s):
    import torch

    return torch.where(s > 1e-12 * s.abs().max().clamp_min(1e-30), s, torch.ones_like(s))


def fit(X, T, seconds: float = 30.0, batch: int = 8192, lr: float = 1e-3, lr_end: float = 1e-4, seed: int = 0,
        max_epochs: int = 1_000_000, log=None):
    """Train a fresh network on (X, T) with Adam on minibatches for about
    `seconds` (cosine-free exponential learning-rate decay from lr to
    lr_end).  Returns (network, stats, history)."""
    import torch

    stats, mx, sx, mt, st = standardise(X, T)
    Xs = ((X - mx) / sx).contiguous()
    Ts = ((T - mt) / st).contiguous()
    n = Xs.shape[0]
    net = mlp.Network(N_FEAT, N_OUT, max_rows=max(batch, 64))
    net.set_params(glorot(seed))
    g = torch.Generator(device=Xs.device)
    g.manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    steps_done = 0
    est_steps = None
    for epoch in range(max_epochs):
        perm = torch.randperm(n, generator=g, device=Xs.device)
        for i in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = perm[i:i + batch]
            xb, tb = Xs[idx].contiguous(), Ts[idx].contiguous()
            frac = min(1.0, (time.perf_counter() - t0) / seconds)
            rate = lr * (lr_end / lr) ** frac
            net.train_step(xb, tb, lr=rate)
            steps_done += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sub = torch.randint(0, n, (min(n, batch),), generator=g, device=Xs.device)
        loss = net.backward(Xs[sub].contiguous(), Ts[sub].contiguous())
        hist.append((epoch, el, loss))
        if log:
            log(f"epoch {epoch} {el:.1f}s train steps {steps_done} loss {loss:.4e}")
        if el >= seconds:
            break
    return net, stats, hist


def tip_history(sim, tip: int, steps: int, every: int):
    us, ts = [], []
    for _ in range(steps // every):
        sim.advance(every)
        us.append(sim.read(sph.S_U)[tip])
        ts.append(sim.scalars()["t"])
    return np.array(us), np.array(ts)


def tip_error(u, t, u_ref, t_ref):
    """max over time of |u(t) - u_ref(t)| / max |u_ref| (u interpolated to the
    reference's times)."""
    keep = t_ref <= t[-1]
    ui = np.stack([np.interp(t_ref[keep], t, u[:, k]) for k in range(u.shape[1])], axis=1)
    umax = np.linalg.norm(u_ref, axis=1).max()
    return float(np.linalg.norm(ui - u_ref[keep], axis=1).max() / max(umax, 1e-300)), float(umax)


def timed_steps_per_s(sim, steps: int):
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.advance(steps)
    e1.record(sim.stream)
    e1.synchronize()
    return steps / (e0.elapsed_time(e1) / 1e3)


def zero_network():
    """(network, stats) that predict no change over the step (vbar = v,
    abar = a): all weights and biases zero, output mean zero."""
    net = mlp.Network(N_FEAT, N_OUT, max_rows=1 << 16)
    net.set_params([(np.zeros((a, b), np.float32), np.zeros(b, np.float32)) for a, b in mlp.layer_shapes(N_FEAT, N_OUT)])
    stats = np.concatenate([np.zeros(N_FEAT), np.ones(N_FEAT), np.zeros(N_OUT), np.ones(N_OUT)]).astype(np.float32)
    return net, stats


def judge_pass_fraction(scene, net, stats, threshold: float, start: int, steps: int, **options):
    """Fraction of acoustic steps start .. start + steps of a plain run whose
    judge would pass the network: every step is a judge step (the plain
    sub-steps run and stand), so the trajectory is the plain method's and the
    count measures the network's residual on the states the method visits."""
    sim = sph.Simulation(scene, **options)
    sim.advance(start)
    sim.set_surrogate(net, stats, threshold, 1)
    sim.advance(steps)
    c = sim.surrogate_counters()
    sim.sync()
    sim.close()
    return c["judged_ok"] / max(1, c["judged_ok"] + c["judged_fail"])


def evaluate(scene, net, stats, threshold: float, steps: int, every: int = 10, timing_steps: int = 2000,
             judge_every: int = 10, plain=None, **options):
    """Plain sub-steps against the surrogate on one scene from the same start:
    tip error of the surrogate run (the plain run is the reference), the
    fraction of acoustic steps the network took (judged every `judge_every`
    steps), and steps/s of both.  plain: a (u, t, steps_per_s) result of an
    earlier plain run of the same scene, steps and sampling, to reuse."""
    tip = int(scene["tip_index"])
    if plain is None:
        p = sph.Simulation(scene, **options)
        u_p, t_p = tip_history(p, tip, steps, every)
        sps_plain = timed_steps_per_s(p, timing_steps)
        p.close()
    else:
        u_p, t_p, sps_plain = plain
    sur = sph.Simulation(scene, **options)
    sur.set_surrogate(net, stats, threshold, judge_every)
    u_s, t_s = tip_history(sur, tip, steps, every)
    c = sur.surrogate_counters()
    sps_sur = timed_steps_per_s(sur, timing_steps)
    c2 = sur.surrogate_counters()
    unstable = False
    try:
        sur.sync()
    except sph.SphError:
        unstable = True
    sur.close()
    err, umax = tip_error(u_s, t_s, u_p, t_p)
    if not np.isfinite(err):
        err, unstable = float("inf"), True
    acc = c["accepted"] / max(1, c["accepted"] + c["fallback"])
    acc_t = (c2["accepted"] - c["accepted"]) / max(1, c2["accepted"] + c2["fallback"] - c["accepted"] - c["fallback"])
    return {"threshold": threshold, "judge_every": judge_every, "tip_error": err, "tip_max_m": umax,
            "accepted_fraction": acc, "accepted_fraction_timed": acc_t, "judged_ok": c["judged_ok"],
            "judged_fail": c["judged_fail"], "unstable": unstable, "steps_per_s_plain": sps_plain,
            "steps_per_s_surrogate": sps_sur, "speedup": sps_sur / sps_plain, "eval_steps": steps,
            "timing_steps": timing_steps, "plain": (u_p, t_p, sps_plain)}
