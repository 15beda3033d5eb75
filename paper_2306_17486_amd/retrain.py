"""Solve-time re-training on an out-of-distribution slowness model (Sec. 5.4):
once the medium is known, the trained network is optimised for a short time
on pairs that the multigrid method generates on that medium at half the size
(300 pairs, 30 epochs over them), then used at the full size.  Every step runs
in the library's kernels (hh_gen_training_pairs, hh_train_step).

    python -m paper_2306_17486_amd.retrain --family salt --n 1024 --seed 5 \\
        --net paper_2306_17486_amd/weights/net_ms128_256_512.bin --out retrained.bin

The half-size medium keeps the squared slowness on average: kappa_h^2 is the
mean of kappa^2 over 2 x 2 cells; omega follows the 10-points-per-wavelength
rule on each grid.  The paper's media (Marmousi, SEG/EAGE salt, Overthrust)
are not available: inputs.OOD_FAMILIES are synthetic stand-ins with their
kinds of structure, on square grids."""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import hh, inputs
from .train import GAMMA0


def half_size(kappa: np.ndarray) -> np.ndarray:
    n = kappa.shape[0]
    m = n // 2
    return np.sqrt((kappa.reshape(m, 2, m, 2) ** 2).mean(axis=(1, 3)))


def retrain(ctx, net, kappa: np.ndarray, npairs: int = 300, epochs: int = 30, batch: int = 30, lr: float = 1e-4,
            seed: int = 0, kmin: int = 2, kmax: int = 8, log=None) -> dict:
    """Optimise `net` in place on `npairs` pairs (eq. 20) of the half-size medium."""
    dev = f"cuda:{ctx.device}"
    kh = half_size(kappa)
    nh = kh.shape[0]
    if npairs % batch:
        raise ValueError("npairs must be a multiple of batch")
    # the training step takes one slowness model per sample (its encoder
    # gradient is per sample): the medium repeated `batch` times
    m = hh.Model(ctx, torch.from_numpy(np.repeat(kh[None], batch, axis=0)), inputs.omega_for(nh, kh),
                 gamma0=GAMMA0)
    rng = np.random.default_rng(seed)
    t0 = time.time()
    es, rs = [], []
    for b0 in range(0, npairs, batch):
        x = torch.from_numpy(inputs.random_complex((batch, nh, nh), seed * 1000 + b0)).to(dev, torch.complex64)
        e, r = m.training_pairs(x, rng.integers(kmin, kmax + 1, batch).tolist())
        es.append(e)
        rs.append(r)
    E, R = torch.cat(es), torch.cat(rs)
    t_pairs = time.time() - t0
    losses = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(npairs)).to(dev)
        el = []
        for b0 in range(0, npairs, batch):
            idx = perm[b0:b0 + batch]
            el.append(net.train_step(m, R[idx].contiguous(), E[idx].contiguous(), lr=lr, max_grad_norm=0.0))
        losses.append(float(np.mean(el)))
        if log and (ep + 1) % 5 == 0:
            log(f"[retrain] epoch {ep + 1}/{epochs} loss {losses[-1]:.4e}")
    t_train = time.time() - t0
    m.close()
    return {"half_size": nh, "pairs": npairs, "epochs": epochs, "batch": batch, "lr": lr,
            "pair_seconds": round(t_pairs, 2), "train_seconds": round(t_train, 2), "epoch_loss": losses}


def iterations(ctx, kappa: np.ndarray, nets: dict, nsrc: int = 4, seed: int = 3500, max_iters: int = 4000) -> dict:
    """FGMRES(10) iterations to 1e-6 for nsrc point sources on the medium:
    MG-only and CNN+MG with each network of `nets`."""
    dev = f"cuda:{ctx.device}"
    n = kappa.shape[0]
    m = hh.Model(ctx, torch.from_numpy(kappa), inputs.omega_for(n, kappa))
    b = torch.from_numpy(np.stack([inputs.point_source(n, seed + i) for i in range(nsrc)])).to(dev, torch.complex64)
    out = {}
    _, info = m.solve(b, max_iters=max_iters, precond=hh.HH_PRECOND_MG, want_hist=False)
    out["mg"] = info["iters"].tolist()
    for name, net in nets.items():
        m.attach_net(net)
        _, info = m.solve(b, max_iters=max_iters, precond=hh.HH_PRECOND_CNN_MG, want_hist=False)
        out[name] = info["iters"].tolist()
        out[name + "_converged"] = int(info["converged"].sum())
        m.attach_net(None)
    m.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--family", choices=sorted(inputs.OOD_FAMILIES), default="salt")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--net", required=True)
    ap.add_argument("--pairs", type=int, default=300)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--nsrc", type=int, default=4)
    ap.add_argument("--out", default="")
    ap.add_argument("--json", default="")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("re-training runs on the GPU")
    ctx = hh.Context(0)
    kappa = inputs.OOD_FAMILIES[a.family](a.n, a.seed)
    before = hh.Net.load(ctx, a.net)
    net = hh.Net.load(ctx, a.net)
    rep = retrain(ctx, net, kappa, npairs=a.pairs, epochs=a.epochs, lr=a.lr, seed=a.seed, log=print)
    its = iterations(ctx, kappa, {"cnn_pretrained": before, "cnn_retrained": net}, nsrc=a.nsrc)
    rep.update(family=a.family, n=a.n, seed=a.seed, iterations=its)
    print(json.dumps(rep), flush=True)
    if a.out:
        net.save(a.out)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rep, f)
    before.close()
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
