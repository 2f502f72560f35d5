"""Train the learned slope limiter on the GPU and measure what it gains over van Leer.

    python -m paper_2503_04428_amd.train_limiter [--out DIR] [--nprob 2048] [--steps 4000]

Writes DIR/mlp_limiter_weights.npy (FP32, 1249 values) and DIR/mlp_limiter_training.json (data
recipe, optimiser settings, loss history, the loss of the deployed BF16 evaluation and of van Leer
on the same samples, and the coarse-grid
L1 errors of learned vs van Leer against the restricted fine FP64 solution on held-out problems).
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="output directory (default: the package's data/)")
    ap.add_argument("--nprob", type=int, default=2048)
    ap.add_argument("--ncoarse", type=int, default=256)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-nprob", type=int, default=512)
    args = ap.parse_args(argv)

    from . import learned

    t0 = time.time()
    samples, info = learned.generate_samples(nprob=args.nprob, ncoarse=args.ncoarse, ratio=args.ratio,
                                             times=(0.02, 0.04, 0.06), seed=1000)
    print(f"samples: {info['samples']} from {args.nprob} problems ({time.time() - t0:.1f} s)", flush=True)
    base = {k: learned.baseline_loss(samples, k) for k in ("vanleer", "minmod", "centred")}
    print(f"loss of classical limiters on the samples: {base}", flush=True)
    t1 = time.time()
    w, log = learned.train(samples, steps=args.steps, batch=args.batch, lr=args.lr, seed=args.seed)
    log["deployed_full_loss"] = learned.deployed_loss(w, samples)
    print(f"trained {args.steps} steps in {time.time() - t1:.1f} s, full loss {log['final_full_loss']:.5f} "
          f"(the deployed BF16 evaluation: {log['deployed_full_loss']:.5f})", flush=True)
    t2 = time.time()
    ev = learned.coarse_error(w, nprob=args.eval_nprob, ncoarse=args.ncoarse, ratio=args.ratio, t_end=0.05,
                              seed=5000)
    print(f"held-out coarse L1 (rho, m1, m2, m3, E): learned {np.round(ev['learned_fp32'], 6).tolist()} "
          f"vanleer {np.round(ev['vanleer_fp32'], 6).tolist()} ({time.time() - t2:.1f} s)", flush=True)
    meta = {"data": info, "classical_limiter_loss": base, "training": log, "heldout_eval": ev,
            "eval": {"nprob": args.eval_nprob, "t_end": 0.05, "seed": 5000}}
    if args.out:
        os.makedirs(args.out, exist_ok=True)
        learned.save(w, meta, os.path.join(args.out, "mlp_limiter_weights.npy"),
                     os.path.join(args.out, "mlp_limiter_training.json"))
    else:
        learned.save(w, meta)
    print(json.dumps({"ratio_learned_over_vanleer": ev["ratio_learned_over_vanleer_fp32"]}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
