#!/usr/bin/env python
"""Throughput benchmark: batched Helmholtz solves to relative residual 1e-6 at 1024^2.

Workload: one layered/blocky slowness model (seed 2000) on a 1024 x 1024 grid,
omega = 2 pi n / (10 max kappa) (10 points per wavelength), a 16-cell
absorbing layer, 64 unit point sources (seeds 3000..3063) solved together by
FGMRES(10).  A step is one whole batched solve of the 64 right-hand sides
(every iteration of every RHS until its FP64 residual is <= 1e-6), with the
slowness model, its multigrid hierarchy, its coarse factors and the
right-hand sides already resident in HBM.

Prints one JSON line.  Options:
  --gpus N (only 1 is supported: the path runs on one GPU), --steps K, --warmup W
  --precond {auto,mg,cnn_mg}: auto = CNN+MG when a trained network file exists
  --no-cpu-baseline: skip the bounded CPU oracle timing
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/s to rel. residual 1e-6 at 1024², CNN+MG vs MG-only FGMRES"
NET_FILE = os.path.join(ROOT, "paper_2306_17486_amd", "weights", "net_ms128_256.bin")

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# Algorithmic HBM bytes per grid point and right-hand side of one launch of the
# single-kernel classes (complex single = 8 B; coefficients shared by all RHS
# of the slowness model are counted once per launch, 8 B per point).
# op_dots at inner step j: z (8) + w (8) + v_0..v_j (8 (j+1)).
# ortho at inner step j:   v_0..v_j (8 (j+1)) + w read (8) + w write (8).
# vc_down (finest level):  b (8) + coarse right-hand side (8/4).
# vc_up (finest level):    b (8) + coarse correction (8/4) + z (8).


_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS",
                "NUMEXPR_NUM_THREADS", "VECLIB_MAXIMUM_THREADS", "GOTO_NUM_THREADS")


def _cpu_worker(args):
    n, seed_k, seed_b, iters = args
    for v in _THREAD_VARS:
        os.environ[v] = "1"
    import numpy as np  # noqa: F401
    from oracle import helmholtz as H
    from paper_2306_17486_amd import inputs
    k = inputs.layered_slowness(n, seed_k)
    prob = H.Problem(k, inputs.omega_for(n, k))
    b = inputs.point_source(n, seed_b)
    t = time.perf_counter()
    H.fgmres(prob.A, b, prob.mg, None, 10, 1e-6, iters)
    return (time.perf_counter() - t) / iters


def cpu_sample(n, nrhs, sample_iters):
    """Time the FP64 oracle (MG-only FGMRES) on the host cores, one RHS per
    process, `sample_iters` iterations each.  Runs before the GPU is touched
    (child processes are started from a process without GPU state)."""
    cores = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1), 16, nrhs)
    # one single-threaded process per core (children inherit this environment)
    for v in _THREAD_VARS:
        os.environ[v] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    per_it = []
    with ctx.Pool(cores) as pool:
        for v in pool.imap_unordered(_cpu_worker, [(n, 2000, 3000 + i, sample_iters) for i in range(cores)]):
            per_it.append(v)
            print(f"bench: cpu sample {len(per_it)}/{cores}: {v:.3f} s/iteration", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    return cores, sum(per_it) / len(per_it), wall


def cpu_baseline(sample, n, sample_iters, iters_per_solve):
    """solves/s of the oracle, extrapolated as cores / (s per iteration * iterations per solve)."""
    cores, s_it, wall = sample
    value = cores / (s_it * iters_per_solve)
    return {"value": value, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} RHS x {sample_iters} MG-only FGMRES iterations of the {n}^2 workload "
                      f"(one process per core, FP64 NumPy/SciPy oracle); {s_it:.3f} s/iteration, extrapolated "
                      f"to {iters_per_solve:.0f} iterations per solve; wall {wall:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--precond", choices=["auto", "mg", "cnn_mg"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--max-iters", type=int, default=10000)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {a.gpus} is not supported "
              f"(the right-hand sides shard across GPUs with no communication, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    sample = None
    if not a.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        sample = cpu_sample(a.n, a.nrhs, a.cpu_iters)

    import numpy as np
    import torch
    from paper_2306_17486_amd import hh, inputs

    n, nrhs = a.n, a.nrhs
    dev = "cuda:0"
    k = inputs.layered_slowness(n, 2000)
    omega = inputs.omega_for(n, k)
    ctx = hh.Context(0)
    model = hh.Model(ctx, torch.from_numpy(k), omega)
    b = torch.from_numpy(np.stack([inputs.point_source(n, 3000 + i) for i in range(nrhs)])).to(dev, torch.complex64)
    precond = hh.HH_PRECOND_MG
    use_cnn = a.precond == "cnn_mg" or (a.precond == "auto" and os.path.exists(NET_FILE))
    if use_cnn:
        net = hh.Net.load(ctx, NET_FILE)
        model.attach_net(net)
        precond = hh.HH_PRECOND_CNN_MG

    def one_solve():
        # a cap far above the need, so that every right-hand side reaches 1e-6
        return model.solve(b, precond=precond, max_iters=a.max_iters, want_hist=False)

    def say(msg):
        print(msg, file=sys.stderr, flush=True)

    say(f"bench: n={n} nrhs={nrhs} precond={'cnn_mg' if use_cnn else 'mg'}")
    for w in range(a.warmup):
        t = time.perf_counter()
        _, info = one_solve()
        say(f"bench: warmup {w} done in {time.perf_counter() - t:.2f} s, iterations {int(info['iters'].max())}")
    torch.cuda.synchronize()
    ctx.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for st in range(a.steps):
        x, info = one_solve()
        infos.append(info)
        say(f"bench: step {st} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_end()
    iters = np.concatenate([i["iters"] for i in infos])
    conv = np.concatenate([i["converged"] for i in infos])
    fres = np.concatenate([i["final_res"] for i in infos])
    # only right-hand sides whose FP64 residual reached 1e-6 count as solves
    value = float(conv.sum()) / elapsed

    # roofline of the dominant single-kernel class (largest summed time).
    # Algorithmic bytes = (sum over RHS of their iterations) x N x bytes per point
    # and RHS, plus the shared coefficients (8 B per point) once per launch.
    # Inactive right-hand sides exit at once and are not counted.
    N = n * n
    mean_it = float(iters.mean())
    rhs_iters = float(iters.sum())
    mean_jp1 = (10 + 1) / 2.0  # mean (j + 1) over full FGMRES(10) cycles
    mc = n // 4  # coarsest grid of the 3-level hierarchy
    per_pt = {"op_dots": 16 + 8 * mean_jp1, "ortho": 16 + 8 * mean_jp1, "vc_down": 8 + 2, "vc_up": 8 + 2 + 8,
              # coarse solve per RHS: b read twice, y written and read, x written (5 coarse vectors)
              "vc_coarse": 5 * 8 * mc * mc / N}
    # per launch, shared by all RHS: coefficients; for the coarse solve the m
    # Schur inverses (m^2 complex each) streamed once per sweep
    coef_pt = {"op_dots": 8, "ortho": 0, "vc_down": 8, "vc_up": 8, "vc_coarse": 2 * mc ** 3 * 8 / N}
    ranked = sorted(((v[0], kname) for kname, v in prof.items()), reverse=True)
    dom = next((kname for _, kname in ranked if kname in per_pt), None)
    roof = None
    if dom:
        ms, cnt = prof[dom]
        total_bytes = rhs_iters * N * per_pt[dom] + cnt * N * coef_pt[dom]
        ach = total_bytes / (ms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(ms / cnt * 1e3, 1),
                "algorithmic_bytes_per_launch": int(total_bytes / cnt),
                "bytes_per_point_per_rhs": per_pt[dom]}
    kt = {kname: {"ms": round(v[0], 2), "launches": v[1]} for kname, v in prof.items()}

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if not use_cnn else "bf16+c64+f64",
        "data": "synthetic",
        "config": {"workload": f"{n}^2 layered slowness (seed 2000), {nrhs} unit point sources (seeds 3000..), "
                               f"FGMRES(10) rtol 1e-6, " + ("CNN+MG" if use_cnn else "MG-only") + " preconditioner",
                   "n": n, "nrhs": nrhs, "precond": "cnn_mg" if use_cnn else "mg"},
        "iterations": {"mean": mean_it, "min": int(iters.min()), "max": int(iters.max())},
        "all_converged": bool(conv.all()),
        "converged": f"{int(conv.sum())}/{conv.size}",
        "max_final_rel_residual": float(fres.max()),
        "roofline": roof,
        "kernel_ms": kt,
    }
    if sample is not None:
        out["cpu_baseline"] = cpu_baseline(sample, n, a.cpu_iters, mean_it)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
