"""Learned-corrector driver: data generation, training, threshold calibration and
evaluation, all on the GPU through the library (this module only orchestrates
calls and moves tensors).

Setting: 2D Allen-Cahn u_t = eps^2 Lap u + u - u^3 on (0,1)^2, Q1 grid of
N x N intervals, homogeneous Dirichlet data, u0 i.i.d. uniform[-0.9, 0.9]
from a seed.  The coarse step is one EIFE2 step (eq. (2.14)) of tau_c; the
reference and the fallback are `ratio` EIFE2 steps of tau_f = tau_c / ratio.
A training pair is (u_n, u_c, u_f): a state of a fine trajectory at
t_n = n tau_c, the coarse step from it, and the fine trajectory ratio steps
later.

Weights are stored as .npz (params float32, s_out, theta) with a JSON header
(the settings they were trained for).
"""
import json
import math
import os
import time

import numpy as np
import torch

from . import binding
from .binding import F_ALLEN_CAHN, Corrector, Grid
import seeded_inputs

DEFAULT = {"N": 512, "eps": 0.02, "tau_c": 0.016, "ratio": 8, "channels": 32}


def _log(msg):
    print(msg, flush=True)


def make_grids(N, eps, tau_c, ratio):
    h = [1.0 / N] * 2
    D = eps * eps
    coarse = Grid([N, N], h, D, "f32")
    coarse.set_phi(tau_c, 2)
    fine = Grid([N, N], h, D, "f32")
    fine.set_phi(tau_c / ratio, 2)
    return coarse, fine


def generate_pairs(seeds, windows, N=512, eps=0.02, tau_c=0.016, ratio=8, stride=1, stream=None):
    """Pairs from fine trajectories: for each seed, `windows` windows starting at
    t = 0, stride tau_c, 2 stride tau_c, ...  Returns three float32 CUDA tensors
    (count, N-1, N-1): u_n, u_c, u_f."""
    coarse, fine = make_grids(N, eps, tau_c, ratio)
    n = N - 1
    count = len(seeds) * windows
    un = torch.empty(count, n, n, dtype=torch.float32, device="cuda")
    uc = torch.empty_like(un)
    uf = torch.empty_like(un)
    k = 0
    t_start = time.perf_counter()
    for si, seed in enumerate(seeds):
        u = torch.tensor(seeded_inputs.uniform_field(seed, [N, N]), dtype=torch.float32, device="cuda")
        t = 0.0
        for w in range(windows):
            un[k].copy_(u)
            uc[k].copy_(u)
            coarse.step(uc[k], 1, F_ALLEN_CAHN, t, stream)
            fine.step(u, ratio, F_ALLEN_CAHN, t, stream)
            uf[k].copy_(u)
            t += tau_c
            for _ in range(stride - 1):
                fine.step(u, ratio, F_ALLEN_CAHN, t, stream)
                t += tau_c
            k += 1
        if si % 10 == 9 or si == len(seeds) - 1:
            torch.cuda.synchronize()
            _log(f"corrector data: {si + 1}/{len(seeds)} seeds, {k} pairs, {time.perf_counter() - t_start:.1f} s")
    coarse.close()
    fine.close()
    return un, uc, uf


def change_rms(un, uc):
    """Per pair: c = sqrt(mean((u_c - u_n)^2)) + 1e-30 (the library's change scale)."""
    out = []
    for i in range(0, un.shape[0], 256):
        d = (uc[i:i + 256] - un[i:i + 256]).double()
        out.append(torch.sqrt((d * d).mean(dim=(1, 2))) + 1e-30)
    return torch.cat(out)


def residual_scale(un, uc, uf, idx):
    """RMS over the pairs idx of the relative residual (u_f - u_c) / c (the
    network's output unit s_out)."""
    c = change_rms(un, uc)
    s, cnt = 0.0, 0
    for i in idx.tolist():
        d = (uf[i] - uc[i]).double() / c[i]
        s += float((d * d).sum())
        cnt += d.numel()
    return math.sqrt(s / cnt)


def window_index(seeds, windows, skip):
    """Indices of the pairs of windows >= skip (the transient before is left to the guard)."""
    return torch.tensor([s * windows + w for s in range(seeds) for w in range(skip, windows)], dtype=torch.int64)


def init_params(seed):
    """He-normal weights (fan-in 9 C_in), zero biases, a small output layer; same
    layout as the library's parameter vector."""
    rng = np.random.default_rng(seed)
    C = DEFAULT["channels"]
    parts = [rng.normal(0, math.sqrt(2.0 / 18), 9 * 2 * C), np.zeros(C)]
    for _ in range(4):
        parts += [rng.normal(0, math.sqrt(2.0 / (9 * C)), 9 * C * C), np.zeros(C)]
    parts += [rng.normal(0, 0.1 * math.sqrt(1.0 / (9 * C)), 9 * C), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == binding.CORR_PARAMS
    return p


def train(net, data, idx, epochs, batch, lr_max, lr_min=1e-5, seed=0, log_every=500):
    """Adam with a cosine learning-rate schedule over shuffled mini-batches of the pairs idx."""
    un, uc, uf = data
    count = int(idx.numel())
    idx = idx.cuda()
    steps_per_epoch = count // batch
    total = epochs * steps_per_epoch
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    step = 0
    t0 = time.perf_counter()
    hist = []
    for ep in range(epochs):
        perm = idx[torch.randperm(count, generator=gen).cuda()]
        for b in range(steps_per_epoch):
            sel = perm[b * batch:(b + 1) * batch]
            xb, cb, fb = un.index_select(0, sel), uc.index_select(0, sel), uf.index_select(0, sel)
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * step / max(1, total)))
            want = (step % log_every == 0) or step == total - 1
            loss = net.train_step(xb, cb, fb, lr, want_loss=want)
            if want:
                hist.append((step, loss))
                _log(f"corrector train: epoch {ep} step {step}/{total} lr {lr:.2e} loss {loss:.4e} "
                     f"({time.perf_counter() - t0:.1f} s)")
            step += 1
    torch.cuda.synchronize()
    return hist


def save(path, params, s_out, theta, guard, meta):
    np.savez(path, params=params.astype(np.float32), s_out=np.float64(s_out), theta=np.float64(theta),
             guard=np.float64(guard))
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(dict(meta, s_out=s_out, theta=theta, guard=guard), f, indent=1, sort_keys=True)


def load(path):
    """(params, s_out, theta, guard) of a stored corrector."""
    z = np.load(path, allow_pickle=False)
    return z["params"], float(z["s_out"]), float(z["theta"]), float(z["guard"])


def window_stats(net, data):
    """Per held-out window: indicator r, RMS coarse change ||u_c - u_n|| / sqrt(n),
    RMS error of the corrected step and of the plain coarse step against u_f."""
    un, uc, uf = data
    out = np.zeros((un.shape[0], 4))
    m = float(un[0].numel())
    for i in range(un.shape[0]):
        d = net.forward(un[i], uc[i]).double()
        ch = (uc[i] - un[i]).double()
        res = (uf[i] - uc[i]).double()
        nd, nc = float(torch.linalg.vector_norm(d)), float(torch.linalg.vector_norm(ch))
        out[i] = (nd / (nc + 1e-12), nc / math.sqrt(m), float(torch.linalg.vector_norm(res - d)) / math.sqrt(m),
                  float(torch.linalg.vector_norm(res)) / math.sqrt(m))
    return out


def calibrate_guard(data, windows, skip):
    """Guard on the RMS coarse change: between the largest change of the windows
    the network is trained for (>= skip) and the smallest of the transient
    windows (< skip) -- their geometric mean when they separate."""
    c = change_rms(data[0], data[1]).cpu().numpy()
    w = np.arange(c.size) % windows
    hi_ok, lo_tr = float(c[w >= skip].max()), float(c[w < skip].min())
    return math.sqrt(hi_ok * lo_tr) if hi_ok < lo_tr else lo_tr


def calibrate_theta(net, data, idx=None, quantile=0.999, margin=1.5):
    """Indicator r = ||delta|| / ||u_c - u_n|| over held-out pairs; theta is a
    margin above its high quantile, so that in-distribution steps pass and a
    network response well outside them falls back."""
    un, uc, _ = data
    rs = []
    for i in (range(un.shape[0]) if idx is None else idx.tolist()):
        d = net.forward(un[i], uc[i])
        num = float(torch.linalg.vector_norm(d.double()))
        den = float(torch.linalg.vector_norm((uc[i] - un[i]).double()))
        rs.append(num / (den + 1e-12))
    rs = np.array(rs)
    return float(np.quantile(rs, quantile) * margin), rs


def evaluate(net, seed, steps, theta, N=512, eps=0.02, tau_c=0.016, ratio=8, plain_ratios=(4, 2, 1), guard=None):
    """Trajectory errors against the fine reference over `steps` coarse steps.

    Returns a dict with, for the corrector and for plain EIFE2 at tau_c / r for r
    in plain_ratios: the max over t_k = k tau_c of ||u(t_k) - u_fine(t_k)||_0
    (consistent-mass L2 norm, FP64 on the device), the final-time error, and the
    wall time of the bare trajectory (no error evaluation inside)."""
    coarse, fine = make_grids(N, eps, tau_c, ratio)
    if guard is not None:
        net.set_guard(guard)
    u0 = torch.tensor(seeded_inputs.uniform_field(seed, [N, N]), dtype=torch.float32, device="cuda")
    n = N - 1
    # fine reference at the coarse times
    ref = torch.empty(steps + 1, n, n, dtype=torch.float32, device="cuda")
    u = u0.clone()
    ref[0].copy_(u)
    for k in range(steps):
        fine.step(u, ratio, F_ALLEN_CAHN, k * tau_c)
        ref[k + 1].copy_(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = u0.clone()
    fine.step(u, ratio * steps, F_ALLEN_CAHN, 0.0)
    torch.cuda.synchronize()
    fine_wall = time.perf_counter() - t0
    out = {"seed": seed, "steps": steps, "T": steps * tau_c, "theta": theta, "guard": guard, "dofs": n * n,
           "fine": {"tau": tau_c / ratio, "wall_s": fine_wall}}

    def errs(traj_fn):
        e = []
        u = u0.clone()
        for k in range(steps):
            traj_fn(u, k)
            e.append(fine.norms(u, ref[k + 1])[0])
        return max(e), e[-1], e

    # plain EIFE2 at tau_c / r
    for r in plain_ratios:
        g = Grid([N, N], [1.0 / N] * 2, eps * eps, "f32")
        g.set_phi(tau_c / r, 2)
        emax, efin, _ = errs(lambda u, k: g.step(u, r, F_ALLEN_CAHN, k * tau_c))
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, r * steps, F_ALLEN_CAHN, 0.0)
        torch.cuda.synchronize()
        out[f"plain_tau_{tau_c / r:g}"] = {"tau": tau_c / r, "max_L2": emax, "final_L2": efin,
                                           "wall_s": time.perf_counter() - t0}
        g.close()
    # corrector
    stats = {"fallbacks": 0}

    def corr_step(u, k):
        fb, _, _ = net.infer_step(coarse, fine, u, k * tau_c, ratio, theta)
        stats["fallbacks"] += int(fb)

    emax, efin, _ = errs(corr_step)
    fb_eval = stats["fallbacks"]
    u = u0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fbs = net.run(coarse, fine, u, 0.0, tau_c, steps, ratio, theta)
    torch.cuda.synchronize()
    out["corrector"] = {"tau": tau_c, "max_L2": emax, "final_L2": efin, "wall_s": time.perf_counter() - t0,
                        "fallbacks": fbs, "fallbacks_in_error_run": fb_eval}
    coarse.close()
    fine.close()
    # fine-equivalent DoF-steps/s: simulated time / tau_f fine steps per wall second
    fine_steps = steps * ratio
    for key, rec in out.items():
        if isinstance(rec, dict) and "wall_s" in rec:
            rec["fine_equiv_dof_steps_per_s"] = n * n * fine_steps / rec["wall_s"]
    return out


def compare(net, seeds, steps, theta, guard, N=512, eps=0.02, tau_c=0.016, ratio=8, bound=1e-4):
    """The corrector against plain EIFE2 at equal error over several seeds.

    The plain competitor is the largest tau_c / r (r in 1, 2, 4) whose
    max-over-time L2 error stays within `bound` on every seed; throughputs are
    fine-equivalent DoF-steps/s (simulated time / tau_f fine steps per wall
    second) of each seed's bare trajectory, averaged in time over the seeds."""
    evs = [evaluate(net, s, steps, theta, N, eps, tau_c, ratio, guard=guard) for s in seeds]
    keys = [k for k, v in evs[0].items() if isinstance(v, dict) and "max_L2" in v]
    summ = {"seeds": list(seeds), "steps": steps, "T": steps * tau_c, "bound_L2": bound, "dofs": evs[0]["dofs"],
            "tau_fine": tau_c / ratio, "tau_coarse": tau_c}
    for k in keys:
        wall = sum(e[k]["wall_s"] for e in evs)
        per_seed = [e[k]["max_L2"] for e in evs]
        summ[k] = {"tau": evs[0][k]["tau"], "max_L2": max(per_seed),
                   "max_L2_per_seed": per_seed, "seeds_within_bound": sum(x <= bound for x in per_seed),
                   "fine_equiv_dof_steps_per_s": evs[0]["dofs"] * steps * ratio * len(evs) / wall,
                   "us_per_coarse_interval": wall / (len(evs) * steps) * 1e6}
        if k == "corrector":
            summ[k]["fallbacks"] = [e[k]["fallbacks"] for e in evs]
    ok = [k for k in keys if k.startswith("plain") and summ[k]["max_L2"] <= bound]
    comp = max(ok, key=lambda k: summ[k]["tau"]) if ok else None
    summ["plain_competitor"] = comp
    if comp:
        summ["speedup_vs_competitor"] = (summ["corrector"]["fine_equiv_dof_steps_per_s"]
                                         / summ[comp]["fine_equiv_dof_steps_per_s"])
    summ["corrector_within_bound"] = summ["corrector"]["max_L2"] <= bound
    return summ
