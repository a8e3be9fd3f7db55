"""Train the learned warm start / preconditioner on pairs the FP64 MG-PCG solver generates.

Each sample: a polytrope with random index in [1, 2] and temperature contrast in [3, 30]
(Ma = 0.001, +-1% coefficient noise), a right-hand side that is white noise (zero mean) or a
smooth random-mode field with equal probability, its FP64 MG-PCG solution to 1e-10, and with
probability 1/2 a "previous pressure" input: the solution for the right-hand side perturbed by
10% white noise (else zeros).

The loss is the relative A-norm error <e, A e> / <x, A x> of the network's estimate (the norm CG
minimises): the long-wavelength part of a solution, which a network with a receptive field of
a few dozen cells cannot see, carries little A-norm energy, so the network learns the local
(short-wavelength) part of A^-1 and leaves the rest to the multigrid cycle. Every
forward/backward/Adam step runs in the library's HIP kernels (hp_nn_train_step_anorm); this
script only draws inputs and loops.

    python -m paper_1112_3507_amd.train --n 128 --samples 2000 --out paper_1112_3507_amd/weights/unet128.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (Cin, Cout) of the ten 3x3x3 convolutions in parameter order (see include/hp.h)
CONVS = [(4, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
         (48, 16), (16, 16)]


def he_uniform(seed: int) -> np.ndarray:
    """Initial parameters: weights U(-a, a), a = sqrt(6 / fan_in); zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CONVS:
        a = np.sqrt(6.0 / (27 * ci))
        parts += [rng.uniform(-a, a, size=27 * ci * co), np.zeros(co)]
    parts += [rng.uniform(-np.sqrt(6.0 / 16), np.sqrt(6.0 / 16), size=16), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def sample_stream(n, count, seed, rhs_per_set=8, log=None):
    """Yield (solver, b, p_prev or None, x): the FP64 MG-PCG handle of the sample's coefficients
    (alive while the sample is used) and device tensors."""
    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import workloads as wl
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    done = 0
    while done < count:
        idx = rng.uniform(1.0, 2.0)
        con = rng.uniform(3.0, 30.0)
        p = wl.polytrope((n, n, n), 0.001, seed=int(rng.integers(1 << 30)), contrast=con, index=idx)
        rho = torch.from_numpy(p.rho).to(dev)
        c2 = torch.from_numpy(p.c2).to(dev)
        with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
            for _ in range(min(rhs_per_set, count - done)):
                rs = int(rng.integers(1 << 30))
                b = wl.rhs_white(p.n, rs) if rng.random() < 0.5 else wl.rhs_smooth(p.n, rs)
                bt = torch.from_numpy(b).to(dev)
                x = torch.zeros_like(bt)
                s.solve(bt, x, tol=1e-10)
                prev = None
                if rng.random() < 0.5:
                    nb = b + 0.1 * np.sqrt(np.mean(b * b)) * wl.rhs_white(p.n, rs + 1)
                    prev = torch.zeros_like(bt)
                    s.solve(torch.from_numpy(nb).to(dev), prev, tol=1e-10)
                done += 1
                yield s, bt, prev, x


def train(n=128, samples=2000, lr=1e-3, seed=0, out=None, log_every=100):
    import torch
    import paper_1112_3507_amd as hp
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    net = hp.Net((n, n, n), training=True)
    net.set_params(torch.from_numpy(he_uniform(seed)).to(dev))
    # Each sample's output scale is RMS(x) / RMS(b), so the network works at unit scale; in use
    # the magnitude comes from the A-norm optimal step (hp_warm_start, learned FCG). The stored
    # out_scale is the median ratio.
    ratios = []
    losses = []
    t0 = time.time()
    for k, (solver, b, prev, x) in enumerate(sample_stream(n, samples, seed + 2)):
        ratio = float(x.norm() / b.norm())
        ratios.append(ratio)
        net.set_output_scale(ratio)
        # cosine decay to 10% of the initial rate
        rate = lr * (0.1 + 0.9 * 0.5 * (1.0 + np.cos(np.pi * k / max(samples - 1, 1))))
        losses.append(solver.train_step_anorm(net, b, x, rate, p_prev=prev))
        if log_every and (k + 1) % log_every == 0:
            print("train: %d/%d loss %.4e (last %d mean) %.1fs" % (
                k + 1, samples, np.mean(losses[-log_every:]), log_every, time.time() - t0), flush=True)
    theta = net.get_params().cpu().numpy()
    out_scale = float(np.median(ratios))
    net.close()
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        np.savez(out, theta=theta, out_scale=np.array(out_scale), n=np.array(n),
                 samples=np.array(samples), loss=np.array(losses, dtype=np.float64))
        meta = {"n": n, "samples": samples, "lr": lr, "seed": seed, "out_scale": out_scale,
                "loss_first100": float(np.mean(losses[:100])), "loss_last100": float(np.mean(losses[-100:])),
                "seconds": round(time.time() - t0, 1)}
        with open(os.path.splitext(out)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1)
    return theta, out_scale, losses


def load(path):
    """(theta float32, out_scale) from a checkpoint written by train()."""
    with np.load(path, allow_pickle=False) as z:
        return z["theta"].astype(np.float32), float(z["out_scale"])


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                                                  "unet128.npz"))
    a = ap.parse_args()
    train(a.n, a.samples, a.lr, a.seed, a.out)
