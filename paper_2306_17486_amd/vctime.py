"""Apply the CNN+MG preconditioner (the network, then the V-cycle that starts
from the network's output) to 64 random vectors at 1024^2, four times, through
the library's parity hook: a fixed workload for kernel traces and
hardware-counter runs of the V-cycle kernels with the network's guess.

    python -m paper_2306_17486_amd.vctime [--n 1024] [--batch 64] [--reps 4]
"""
from __future__ import annotations

import argparse
import os
import time

import torch

from . import hh, inputs

NET_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "net_ms128_256_512.bin")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--reps", type=int, default=4)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("vctime runs on the GPU")
    ctx = hh.Context(0)
    k = inputs.layered_slowness(a.n, 2000)
    m = hh.Model(ctx, torch.from_numpy(k), inputs.omega_for(a.n, k))
    net = hh.Net.load(ctx, NET_FILE)
    m.attach_net(net)
    v = torch.from_numpy(inputs.random_complex((a.batch, a.n, a.n), 5)).to("cuda:0", torch.complex64)
    for i in range(a.reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        m.apply_cnn_precond(v)
        torch.cuda.synchronize()
        print(f"preconditioner application {i}: {1e3 * (time.perf_counter() - t):.2f} ms", flush=True)
    m.attach_net(None)
    net.close()
    m.close()
    ctx.close()


if __name__ == "__main__":
    main()
