"""Run the network's 16-channel level pair (two stride-1 3x3 layers with ReLU)
in every variant the autotuner has -- the fused kernel at each tile height and
the two layers launched separately (each at its tuned tile) -- on one synthetic
batch, a few times each, through the library's parity hook: a fixed workload
for kernel traces and hardware-counter runs of these kernels.  --layer c32 /
c64 run one stride-1 32- or 64-channel layer (ReLU, bias, BF16 output only) at the size it has in
the network on a 1024^2 grid (256^2, 128^2) in each of its tile variants
instead; a comma list runs several.

    python -m paper_2306_17486_amd.convtime [--layer pair16|c32|c64] [--batch 64] [--size N] [--reps 5]
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
    ap.add_argument("--size", type=int, default=0, help="grid of the layer (default: its size at 1024^2)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--layer", default="pair16", help="pair16, c32, c64, or a comma list")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("convtime runs on the GPU")
    layers = a.layer.split(",")
    for lay in layers:
        if lay not in LAYERS:
            raise SystemExit(f"unknown layer {lay!r}; one of {', '.join(LAYERS)}")
    ctx = hh.Context(0)
    for lay in layers:
        if lay == "pair16":
            run_pair(ctx, a.batch, a.size or 512, a.reps)
        else:
            run_layer(ctx, LAYERS[lay], a.batch, a.size or SIZES[lay], a.reps)
    ctx.close()


# channels of the single stride-1 layers, and their grid in the network at 1024^2
LAYERS = {"pair16": 16, "c32": 32, "c64": 64}
SIZES = {"c32": 256, "c64": 128}


def run_layer(ctx, c, B, n, reps):
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.standard_normal((B, n, n, c)).astype(np.float32)).to("cuda:0", torch.bfloat16)
    w = torch.from_numpy(rng.uniform(-1, 1, (c, c, 3, 3)) / (3 * np.sqrt(c))).to("cuda:0", torch.float32)
    bias = torch.zeros(c, device="cuda:0")
    for code in hh.conv_variants(c, c, 0):
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            hh.conv_test(ctx, x, w, 0, False, bias=bias, relu=True, variant=code, fp32_out=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
        print(f"{c}-channel layer at {n}^2 x {B}, variant {code}: {dt * 1e3:.3f} ms per call "
              f"(host clock, packing included)", flush=True)


def run_pair(ctx, B, n, reps):
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.standard_normal((B, n, n, 16)).astype(np.float32)).to("cuda:0", torch.bfloat16)
    w1 = torch.from_numpy(rng.uniform(-1, 1, (16, 16, 3, 3)) / 12).to("cuda:0", torch.float32)
    w2 = torch.from_numpy(rng.uniform(-1, 1, (16, 16, 3, 3)) / 12).to("cuda:0", torch.float32)
    b1 = torch.zeros(16, device="cuda:0")
    b2 = torch.zeros(16, device="cuda:0")
    for code in hh.conv_variants(16, 16, 3):
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            hh.conv_pair_test(ctx, x, w1, b1, w2, b2, variant=code)
            dt = time.perf_counter() - t
        print(f"16-channel pair, variant {code}: {dt * 1e3:.3f} ms per call (host clock, packing included)",
              flush=True)


if __name__ == "__main__":
    main()
