"""Train the learned corrector on the GPU and store its weights.

    python -m paper_2209_11922_amd.train_corrector --out paper_2209_11922_amd/weights/corrector_ac512.npz

Data: fine EIFE2 trajectories (tau_f = tau_c / 8 = 0.002) of 2D Allen-Cahn,
eps = 0.02, 512^2 intervals, from seeds 0..S-1 (u0 uniform[-0.9, 0.9]); W
windows per seed.  Training: Adam with a cosine schedule on the MSE of the
scaled residual.  Threshold: calibrated on held-out seeds.  Evaluation: an
unseen seed over 500 coarse steps against the fine reference.
"""
import argparse
import json
import os
import sys
import time

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2209_11922_amd import corrector as cor  # noqa: E402
from paper_2209_11922_amd.binding import Corrector  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--eps", type=float, default=0.02)
    ap.add_argument("--seeds", type=int, default=50)
    ap.add_argument("--windows", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--val-seeds", type=int, default=2)
    ap.add_argument("--eval-seed", type=int, default=1000)
    ap.add_argument("--eval-steps", type=int, default=500)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--skip", type=int, default=3, help="first windows of each trajectory left to the guard")
    ap.add_argument("--stats", default=None, help="save per-window held-out statistics (.npy)")
    args = ap.parse_args()
    N, eps, tau_c, ratio = args.N, args.eps, 0.016, 8
    t_all = time.perf_counter()
    data = cor.generate_pairs(list(range(args.seeds)), args.windows, N, eps, tau_c, ratio)
    idx = cor.window_index(args.seeds, args.windows, args.skip)
    s_out = cor.residual_scale(*data, idx)
    cor._log(f"corrector: {idx.numel()} training pairs (windows >= {args.skip}), relative residual rms {s_out:.4e}")
    net = Corrector(N - 1, N - 1, args.batch)
    net.set_params(cor.init_params(args.init_seed))
    net.set_scale(s_out)
    hist = cor.train(net, data, idx, args.epochs, args.batch, args.lr, seed=args.init_seed)
    del data
    torch.cuda.empty_cache()
    val = cor.generate_pairs(list(range(args.seeds, args.seeds + args.val_seeds)), args.windows, N, eps, tau_c,
                             ratio)
    guard = cor.calibrate_guard(val, args.windows, args.skip)
    vidx = cor.window_index(args.val_seeds, args.windows, args.skip)
    theta, rs = cor.calibrate_theta(net, val, vidx)
    cor._log(f"corrector: theta {theta:.4e} (held-out indicator median {float(sorted(rs)[len(rs) // 2]):.3e}), "
             f"guard {guard:.4e}")
    if args.stats:
        import numpy as np
        np.save(args.stats, cor.window_stats(net, val))
    del val
    params = net.get_params()
    meta = {"N": N, "eps": eps, "tau_c": tau_c, "ratio": ratio, "seeds": args.seeds, "windows": args.windows,
            "skip": args.skip,
            "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "init_seed": args.init_seed,
            "loss_history": hist, "command": " ".join(sys.argv)}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    cor.save(args.out, params, s_out, theta, guard, meta)
    cor._log(f"corrector: weights -> {args.out} ({time.perf_counter() - t_all:.1f} s)")
    if args.eval_steps > 0:
        ev = cor.evaluate(net, args.eval_seed, args.eval_steps, theta, N, eps, tau_c, ratio, guard=guard)
        print(json.dumps(ev), flush=True)
    net.close()


if __name__ == "__main__":
    main()
