"""Writes tests/golden/oracle_1024_layered2000.json: what the FP64 oracle alone
gives on the benchmark workload (1024 x 1024 grid, layered slowness seed 2000,
omega for 10 points per wavelength, unit point sources 3000 + r), for a few of
its right-hand sides:

* x* = A^{-1} b by the sparse direct solve (the exact discrete solution);
* MG-only FGMRES(10) to relative residual 1e-6: iterations, final residual and
  the distance to x*;
* the two-phase CNN+MG FGMRES(10) with the shipped network (3 MG-only
  iterations, then CNN+MG; the preconditioners judge each other per cycle):
  the same figures.

At rtol 1e-6 the distance to x* depends on which residual is left, not only on
its size (reading C17 of the design notes); these figures are the oracle's own
floor, the values the GPU solve is compared with.  Nothing here comes from the
GPU library: only oracle/, the seeded input generators and the network file.

Run from the repository root:
  python tests/golden/make_oracle_1024.py
      (right-hand sides 0 and 21, both preconditioners; about 15 minutes on 4 cores)
  python tests/golden/make_oracle_1024.py --rhs 1 --kinds mg --max-iters 12000 \
      --out tests/golden/oracle_1024_layered2000_mg_rhs1.json
      (the MG-only solve of source 1, which the GPU solve stops at its 10000-iteration
      cap: about 45 minutes on one core)
Single-threaded processes, one per job."""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 1024
SEED_KAPPA = 2000
RHS = (0, 21)
NET_FILE = os.path.join(ROOT, "paper_2306_17486_amd", "weights", "net_ms128_256_512.bin")
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_1024_layered2000.json")


def _problem():
    from oracle import helmholtz as H
    from paper_2306_17486_amd import inputs
    k = inputs.layered_slowness(N, SEED_KAPPA)
    return H.Problem(k, inputs.omega_for(N, k))


def _job(args):
    kind, r, max_iters = args
    import numpy as np
    from oracle import cnn as C
    from oracle import helmholtz as H
    from oracle import solver as S
    from paper_2306_17486_amd import inputs, netfile
    prob = _problem()
    b = inputs.point_source(N, 3000 + r)
    t = time.perf_counter()
    if kind == "mg":
        x, its, _, rel = H.solve_mg(prob, b, rtol=1e-6, max_iters=max_iters)
        extra = {}
    else:
        flat, ch = netfile.read_params(NET_FILE)
        netp = S.NetPrecond(C.Net(netfile.unflatten_params(flat, ch)), prob)
        st = {}
        x, its, _, rel = S.solve_two_phase(prob, netp, b, rtol=1e-6, max_iters=max_iters, stats=st)
        extra = st
    dt = time.perf_counter() - t
    res = float(np.linalg.norm(b - prob.A(x)) / np.linalg.norm(b))
    print(f"{kind} rhs {r}: {its} iterations, residual {res:.3e}, {dt:.0f} s", flush=True)
    return kind, r, x, int(its), res, dt, extra


def main():
    import numpy as np
    from oracle import helmholtz as H
    from paper_2306_17486_amd import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--rhs", default=",".join(str(r) for r in RHS))
    ap.add_argument("--kinds", default="cnn_mg,mg")
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    rhs = tuple(int(v) for v in a.rhs.split(","))
    jobs = [(kind, r, a.max_iters) for r in rhs for kind in a.kinds.split(",")]
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(jobs)) as pool:
        pend = pool.map_async(_job, jobs)
        prob = _problem()
        B = np.stack([inputs.point_source(N, 3000 + r) for r in rhs])
        t = time.perf_counter()
        X = H.exact_solve(prob, B)
        print(f"direct solve {time.perf_counter() - t:.0f} s", flush=True)
        results = pend.get()
    out = {"workload": f"{N}^2 layered slowness seed {SEED_KAPPA}, omega = 2 pi n / 10, unit point sources "
                       "3000 + r, FGMRES(10), rtol 1e-6 on the FP64 true residual",
           "max_iters": a.max_iters,
           "reference": "x* by the oracle's sparse direct solve (SuperLU, FP64)",
           "network": os.path.basename(NET_FILE), "rhs": {}}
    for kind, r, x, its, res, dt, extra in results:
        q = rhs.index(r)
        err = float(np.linalg.norm(x - X[q]) / np.linalg.norm(X[q]))
        d = out["rhs"].setdefault(str(r), {})
        d[kind] = dict({"iterations": its, "rel_residual": res, "rel_error_vs_exact": err,
                        "seconds": round(dt, 1)}, **extra)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
