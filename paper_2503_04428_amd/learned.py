"""Learned slope limiter: training data from the scheme's own fine FP64 solutions, GPU training with
the library's forward/backward and Adam kernels, and the coarse-grid accuracy comparison.

Pipeline (every arithmetic step runs in libhydro.so kernels; torch only holds device buffers,
draws random batch indices and gathers rows):
  1. a batch of seeded 1D Riemann problems (problems.riemann_batch) is solved in FP64 with van Leer
     and HLLC on a grid `ratio` times finer than the target grid;
  2. at several snapshot times hx_mlp_features restricts the fine state to the coarse grid and
     emits (normalised stencil, base, target slope, weight) samples where the network applies;
  3. Adam on L = sum wt (phi a - t)^2 / sum wt with hx_mlp_grad / hx_mlp_adam (FP32 master weights);
  4. the trained network runs fused in the sweep (limiter 'mlp', BF16 matrix cores) and is compared
     with van Leer on held-out problems against the restricted fine solution.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import hydro, problems

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "data", "mlp_limiter_weights.npy")
META_PATH = os.path.join(HERE, "data", "mlp_limiter_training.json")
NPARAM = hydro.MLP_NPARAM


def init_weights(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases (phi = 1, the centred slope, before training)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(NPARAM, dtype=np.float32)

    def glorot(fan_in, fan_out, size):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=size).astype(np.float32)

    w[0:128] = glorot(4, 32, 128)
    w[160:1184] = glorot(32, 32, 1024)
    w[1216:1248] = glorot(32, 1, 32)
    return w


def load_weights(path: str = WEIGHTS_PATH) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    assert w.shape == (NPARAM,)
    return w.astype(np.float32)


def _run_to(solver, t0: float, t1: float, max_steps: int = 100000) -> tuple[float, int]:
    t, n = t0, 0
    while t < t1 * (1 - 1e-12) and n < max_steps:
        dt = min(solver.compute_dt(), t1 - t)
        solver.step(dt)
        t += dt
        n += 1
    return t, n


def generate_samples(nprob: int = 2048, ncoarse: int = 256, ratio: int = 4, times=(0.02, 0.04, 0.06),
                     seed: int = 1000, device="cuda"):
    """Training samples from fine FP64 solutions of nprob seeded Riemann problems (half of them the
    mirror images of the other half).  Returns device tensors (x, a, t, wt) with wt > 0 only."""
    import torch

    prob = problems.riemann_batch(nprob, ncoarse * ratio, seed=seed, mirror=True, precision="fp64")
    s = hydro.Solver(prob, device=device)
    s.set_state(prob.U0)
    t = 0.0
    xs, as_, ts, ws = [], [], [], []
    nsteps = 0
    for tt in times:
        t, n = _run_to(s, t, tt)
        nsteps += n
        fine = s.get_state().reshape(5, nprob, ncoarse * ratio)
        x, a, tg, wt = hydro.mlp_features(fine, ratio, prob.gamma)
        keep = wt > 0
        xs.append(x[keep])
        as_.append(a[keep])
        ts.append(tg[keep])
        ws.append(wt[keep])
    s.close()
    out = tuple(torch.cat(v).contiguous() for v in (xs, as_, ts, ws))
    return out, {"nprob": nprob, "ncoarse": ncoarse, "ratio": ratio, "times": list(times), "seed": seed,
                 "fine_steps": nsteps, "samples": int(out[0].shape[0])}


def train(samples, steps: int = 4000, batch: int = 65536, lr: float = 3e-3, lr_final: float = 1e-4, seed: int = 0,
          device="cuda", log_every: int = 500, w0=None):
    """Adam on random batches of the samples; cosine-decayed learning rate.  Returns (weights, log)."""
    import torch

    x, a, t, wt = samples
    n = x.shape[0]
    batch = min(batch, n)
    tr = hydro.MlpTrainer(init_weights(seed) if w0 is None else w0, batch, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    log = []
    for k in range(steps):
        idx = torch.randint(0, n, (batch,), device=device, generator=gen)
        tr.gradient(x[idx].contiguous(), a[idx].contiguous(), t[idx].contiguous(), wt[idx].contiguous())
        lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(steps - 1, 1)))
        tr.adam(lr=lr_k)
        if log_every and (k % log_every == 0 or k == steps - 1):
            log.append((k, float(tr.loss.item())))
    full = hydro.MlpTrainer(tr.w.cpu().numpy(), n, device=device)
    _, loss = full.gradient(x, a, t, wt)
    return tr.w.cpu().numpy(), {"steps": steps, "batch": batch, "lr": lr, "lr_final": lr_final, "seed": seed,
                                "loss_log": log, "final_full_loss": float(loss.item())}


def baseline_loss(samples, phi_rule: str = "vanleer"):
    """Loss of a classical limiter on the same samples, phi expressed per stencil (evaluation only)."""
    x, a, t, wt = samples
    r = x[:, 2] / x[:, 1]
    if phi_rule == "vanleer":
        phi = 2 * r / (1 + r)
    elif phi_rule == "minmod":
        phi = r.clamp(max=1.0)
    else:
        phi = r * 0 + 1.0
    return float(((wt * (phi * a - t) ** 2).sum() / wt.sum()).item())


def deployed_loss(weights, samples, device="cuda"):
    """Loss of the network as the sweep evaluates it (BF16 parameters, inputs and first hidden layer
    on the matrix cores, hx_mlp_eval) on the samples; training itself runs in FP32, so this is what
    the BF16 roundings change (the weighted sum is evaluation only)."""
    import torch

    x, a, t, wt = samples
    phi = hydro.mlp_eval(torch.as_tensor(np.asarray(weights, dtype=np.float32), device=device), x)
    return float(((wt * (phi * a - t) ** 2).sum() / wt.sum()).item())


def training_loss(weights, samples, device="cuda"):
    """Loss of the FP32 training forward (hx_mlp_grad) on the samples."""
    x = samples[0]
    tr = hydro.MlpTrainer(np.asarray(weights, dtype=np.float32), x.shape[0], device=device)
    _, loss = tr.gradient(*samples)
    return float(loss.item())


def coarse_error(weights, nprob: int = 256, ncoarse: int = 256, ratio: int = 4, t_end: float = 0.05,
                 seed: int = 5000, device="cuda"):
    """L1 errors of the coarse FP32 runs (learned limiter and van Leer) and the FP64 van Leer run
    against the fine FP64 solution restricted to the coarse grid, on held-out problems."""
    import torch

    fine_p = problems.riemann_batch(nprob, ncoarse * ratio, seed=seed, precision="fp64")
    f = hydro.Solver(fine_p, device=device)
    f.set_state(fine_p.U0)
    _run_to(f, 0.0, t_end)
    ref = f.get_state().reshape(5, nprob, ncoarse, ratio).mean(dim=3)
    f.close()
    out = {}
    for name, lim, prec, ng in [("learned_fp32", "mlp", "fp32", 3), ("vanleer_fp32", "vanleer", "fp32", 2),
                                ("vanleer_fp64", "vanleer", "fp64", 2)]:
        cp = problems.riemann_batch(nprob, ncoarse, seed=seed, precision=prec, limiter=lim, ng=ng)
        s = hydro.Solver(cp, device=device)
        if lim == "mlp":
            s.set_mlp(weights)
        s.set_state(cp.U0)
        _run_to(s, 0.0, t_end)
        st = s.get_state().reshape(5, nprob, ncoarse)
        s.close()
        err = (st - ref).abs().mean(dim=(1, 2)) / ref.abs().mean(dim=(1, 2)).clamp(min=1e-300)
        out[name] = err.cpu().numpy().tolist()
    out["ratio_learned_over_vanleer_fp32"] = [a / b if b > 0 else None
                                              for a, b in zip(out["learned_fp32"], out["vanleer_fp32"])]
    return out


def save(weights: np.ndarray, meta: dict, path: str = WEIGHTS_PATH, meta_path: str = META_PATH):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(weights, dtype=np.float32), allow_pickle=False)
    with open(meta_path, "w") as fh:
        json.dump(meta, fh, indent=1)
