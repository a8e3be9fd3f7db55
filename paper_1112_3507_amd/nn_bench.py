"""Time the learned stage's network forward (features, ten convolutions, pooling, head, output
scaling: hp_nn_forward) on a polytrope of n^3 cells, for profiling the network kernels alone.

    python paper_1112_3507_amd/nn_bench.py --n 256 --reps 10

Prints one line per timed batch: milliseconds per forward (wall clock around `reps` forwards
after a device synchronisation) and a checksum of the output.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import train as tr
    from paper_1112_3507_amd import workloads as wl

    n = (args.n, args.n, args.n)
    p = wl.polytrope(n, 0.001, seed=5)
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rho, c2, b = d(p.rho), d(p.c2), d(wl.rhs_white(n, 6))
    net = hp.Net(n, training=False)
    net.set_params(d(tr.he_uniform(3).astype(np.float32)))
    net.set_output_scale(1e-3)
    y = torch.empty_like(b)
    for _ in range(args.warmup):
        net.forward(b, rho, c2, None, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        net.forward(b, rho, c2, None, y)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.reps
    print("network forward %dx%dx%d: %.3f ms per forward over %d (checksum %.10e)"
          % (args.n, args.n, args.n, ms, args.reps, float(y.abs().sum())), flush=True)
    net.close()


if __name__ == "__main__":
    main()
