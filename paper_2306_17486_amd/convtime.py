"""Run the network's 16-channel level pair (two stride-1 3x3 layers with ReLU)
in every variant the autotuner has -- the fused kernel at each tile height and
the two layers launched separately (each at its tuned tile) -- on one synthetic
batch, a few times each, through the library's parity hook: a fixed workload
for kernel traces and hardware-counter runs of these kernels.

    python -m paper_2306_17486_amd.convtime [--batch 64] [--size 512] [--reps 5]
"""
from __future__ import annotations

import argparse
import time

import numpy as np
import torch

from . import hh


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("convtime runs on the GPU")
    ctx = hh.Context(0)
    rng = np.random.default_rng(1)
    B, n = a.batch, a.size
    x = torch.from_numpy(rng.standard_normal((B, n, n, 16)).astype(np.float32)).to("cuda:0", torch.bfloat16)
    w1 = torch.from_numpy(rng.uniform(-1, 1, (16, 16, 3, 3)) / 12).to("cuda:0", torch.float32)
    w2 = torch.from_numpy(rng.uniform(-1, 1, (16, 16, 3, 3)) / 12).to("cuda:0", torch.float32)
    b1 = torch.zeros(16, device="cuda:0")
    b2 = torch.zeros(16, device="cuda:0")
    for code in hh.conv_variants(16, 16, 3):
        for _ in range(a.reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            hh.conv_pair_test(ctx, x, w1, b1, w2, b2, variant=code)
            dt = time.perf_counter() - t
        print(f"16-channel pair, variant {code}: {dt * 1e3:.3f} ms per call (host clock, packing included)",
              flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
