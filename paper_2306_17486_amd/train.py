"""Multiscale training of the encoder-solver network on pairs that the
multigrid-preconditioned solver itself generates (Sec. 4.3, eq. 19-20), run on
the GPU through the C ABI (every forward, backward and optimiser step is a
library kernel).

* Data (eq. 20): per sample a fresh slowness model (alternating Gaussian random
  field / layered family), a random vector x, b = A x on the training operator
  (global damping 0.05, Sec. 5.1), k ~ U{2..8} MG-preconditioned FGMRES
  iterations from zero giving x_k; e = x - x_k, r = b - A x_k.
* Loss (eq. 19): mean over the batch of || P(Net(r / rms r)) - e / (h^2 rms r) ||^2.
* Multiscale schedule (Sec. 4.3, Sec. 5.3): blocks of steps alternate between
  the grid sizes (128, 256 and optionally 512) in the proportions of the
  paper's epoch lengths, 16:10:4; Adam, learning rate divided by 10 for the
  last quarter of the steps.  Below n = 512 the coarsest level keeps the size
  of the level above it, so only 512 trains the stride-2 coarsest layers that
  larger grids use.
* Gradient clipping: the global gradient norm is clipped to `clip` times the
  median of the recent norms, so one outlier batch (the switch to a new grid
  size, a rare hard medium) cannot undo what the network has learned.
* Validation: fixed held-out pairs per size, evaluated without updates.
* Evaluation: FGMRES iterations to 1e-6 with MG-only, with the untrained
  network and with the trained one, on held-out media at several sizes.

    python -m paper_2306_17486_amd.train --steps 2000 --out paper_2306_17486_amd/weights/net_ms128_256.bin
"""
from __future__ import annotations

import argparse
import json
import os
import queue
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import hh, inputs

SIZE_WEIGHT = {128: 16, 256: 10, 512: 4, 1024: 2}  # relative number of steps per grid size (Sec. 5.3 epoch lengths; 1024 optional)
GAMMA0 = 0.05                     # global damping of the training operators (Sec. 5.1)
TRAIN_SEED0 = 100_000             # slowness seeds of the training stream: TRAIN_SEED0 + step * batch + j
VAL_SEED0 = 9000                  # held-out validation media and vectors
EVAL_KAPPA_SEED0 = 1000           # held-out media of the iteration-count evaluation
EVAL_SOURCE_SEED0 = 3000


def _log(*a):
    print(*a, flush=True)


def family_of(j: int) -> str:
    return "grf" if j % 2 == 0 else "layered"


def kappa_batch(n: int, seeds, pool=None) -> np.ndarray:
    """Slowness models of the given seeds; `pool` (an executor) draws them in
    parallel (NumPy's FFTs and generators release the GIL)."""
    one = lambda s: inputs.slowness(n, int(s), family_of(int(s)))
    ks = list(pool.map(one, seeds)) if pool is not None else [one(s) for s in seeds]
    return np.stack(ks).astype(np.float32)


def schedule(steps: int, block: int, sizes=(128, 256)) -> list[int]:
    """Grid size of every block of `block` steps: each block goes to the size
    that is furthest behind its share of the SIZE_WEIGHT ratio."""
    done = {n: 0 for n in sizes}
    out = []
    for _ in range((steps + block - 1) // block):
        n = min(sizes, key=lambda s: (done[s] / SIZE_WEIGHT[s], -SIZE_WEIGHT[s]))
        done[n] += 1
        out.append(n)
    return out


def learning_rate(step: int, steps: int, lr: float, drop_frac: float = 0.75) -> float:
    return lr if step < int(drop_frac * steps) else lr / 10.0


class KappaPrefetch:
    """Draws the next batches of slowness models on host threads while the GPU
    trains on the current one."""

    def __init__(self, plan, batch: int, depth: int = 3, step0: int = 0, fresh=None):
        self.q: queue.Queue = queue.Queue(maxsize=depth)
        self.plan, self.batch, self.step0 = plan, batch, step0
        self.fresh = fresh if fresh is not None else [True] * len(plan)
        self.t = threading.Thread(target=self._run, daemon=True)
        self.t.start()

    def _run(self):
        with ThreadPoolExecutor(8) as pool:
            for step, n in enumerate(self.plan):
                if not self.fresh[step]:  # the previous step's media are used again
                    self.q.put((step, n, None))
                    continue
                seeds = TRAIN_SEED0 + (self.step0 + step) * self.batch + np.arange(self.batch)
                self.q.put((step, n, kappa_batch(n, seeds, pool)))

    def get(self):
        return self.q.get()


def make_val_set(ctx, sizes, nval: int, batch: int, dev):
    """Held-out (model, r, e) batches per size, generated once and kept on the GPU."""
    out = {}
    for n in sizes:
        om = inputs.omega_for(n)
        rng = np.random.default_rng(VAL_SEED0 + n)
        items = []
        for b0 in range(0, nval, batch):
            seeds = VAL_SEED0 + b0 + np.arange(batch)
            m = hh.Model(ctx, torch.from_numpy(kappa_batch(n, seeds)), om, gamma0=GAMMA0)
            x = torch.from_numpy(inputs.random_complex((batch, n, n), VAL_SEED0 + 7 * n + b0)).to(dev)
            e, r = m.training_pairs(x, rng.integers(2, 9, batch).tolist())
            items.append((m, r, e))
        out[n] = items
    return out


def val_loss(net, items) -> float:
    return float(np.mean([net.eval_loss(m, r, e) for m, r, e in items]))


class GradClip:
    """Clip threshold = factor x the median of the last `window` gradient norms
    (no clipping until `warmup` norms have been seen, or with factor 0)."""

    def __init__(self, factor: float, window: int = 200, warmup: int = 20):
        self.factor, self.window, self.warmup = factor, window, warmup
        self.norms: list[float] = []

    def threshold(self) -> float:
        if self.factor <= 0 or len(self.norms) < self.warmup:
            return 0.0
        return self.factor * float(np.median(self.norms[-self.window:]))

    def record(self, norm: float):
        self.norms.append(norm)


def train(ctx, net, steps: int, batch: int, lr: float, block: int, val_every: int, nval: int, seed: int,
          sizes=(128, 256), clip: float = 2.0, step0: int = 0, reuse: int = 1, reuse_from: int = 1024):
    """`steps` steps; with `step0` > 0 (a continued run) the training stream's
    media are those of steps step0 .. step0 + steps - 1, so no sample repeats.
    At grid sizes >= `reuse_from` one batch of media (and its factorised
    coarsest operators) serves `reuse` consecutive steps of a block, each with
    fresh random vectors: setting up 32 media at 1024^2 costs several training
    steps."""
    dev = f"cuda:{ctx.device}"
    plan_blocks = schedule(steps, block, sizes)
    plan = [plan_blocks[s // block] for s in range(steps)]
    fresh = [plan[s] < reuse_from or (s % block) % max(1, reuse) == 0 for s in range(steps)]
    omegas = {n: inputs.omega_for(n) for n in sizes}
    _log(f"[train] {steps} steps, batch {batch}, blocks of {block}: " +
         ", ".join(f"{n}^2 x {plan.count(n)}" for n in sizes))
    t0 = time.time()
    val = make_val_set(ctx, sizes, nval, batch, dev)
    _log(f"[train] validation set ({nval} pairs per size) in {time.time() - t0:.1f} s")
    hist = {"step": [], "size": [], "loss": [], "lr": [], "grad_norm": [], "clipped": [], "val_step": [],
            "val": {str(n): [] for n in sizes}}
    clipper = GradClip(clip)

    def do_val(step):
        hist["val_step"].append(step)
        vs = {}
        for n in sizes:
            vs[n] = val_loss(net, val[n])
            hist["val"][str(n)].append(vs[n])
        _log(f"[val] step {step}: " + ", ".join(f"{n}^2 {vs[n]:.4e}" for n in sizes))

    do_val(0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    pre = KappaPrefetch(plan, batch, step0=step0, fresh=fresh)
    t0 = time.time()
    run = {n: [] for n in sizes}
    m = None
    for step in range(steps):
        s, n, kap = pre.get()
        assert s == step and n == plan[step]
        if kap is not None:
            if m is not None:
                m.close()
            m = hh.Model(ctx, torch.from_numpy(kap), omegas[n], gamma0=GAMMA0)
        x = torch.view_as_complex(torch.randn((batch, n, n, 2), generator=gen, device=dev))
        e, r = m.training_pairs(x, rng.integers(2, 9, batch).tolist())
        cur_lr = learning_rate(step, steps, lr)
        thr = clipper.threshold()
        loss = net.train_step(m, r, e, lr=cur_lr, max_grad_norm=thr)
        clipper.record(net.last_grad_norm)
        if not np.isfinite(loss):
            raise RuntimeError(f"training loss is not finite at step {step}")
        hist["step"].append(step)
        hist["size"].append(n)
        hist["loss"].append(loss)
        hist["lr"].append(cur_lr)
        hist["grad_norm"].append(net.last_grad_norm)
        hist["clipped"].append(bool(thr > 0 and net.last_grad_norm > thr))
        run[n].append(loss)
        if (step + 1) % 50 == 0:
            el = time.time() - t0
            _log(f"[train] step {step + 1}/{steps} {n}^2 lr {cur_lr:.0e} loss(50) "
                 f"{np.mean(hist['loss'][-50:]):.4e} |g| {np.median(hist['grad_norm'][-50:]):.3e} "
                 f"clipped {sum(hist['clipped'][-50:])}  {el:.0f} s ({el / (step + 1) * 1e3:.0f} ms/step)")
        if (step + 1) % val_every == 0 or step + 1 == steps:
            do_val(step + 1)
    if m is not None:
        m.close()
    hist["seconds"] = time.time() - t0
    hist["steps_per_s"] = steps / hist["seconds"]
    return hist


def evaluate(ctx, nets: dict, sizes=(128, 256, 512), nk: int = 16, max_iters: int = 2000):
    """FGMRES(10) iterations to relative residual 1e-6 for nk held-out Gaussian
    random field media (one point source each): MG-only and two-phase CNN+MG
    with each network of `nets`."""
    dev = f"cuda:{ctx.device}"
    res = {}
    for n in sizes:
        kap = np.stack([inputs.grf_slowness(n, EVAL_KAPPA_SEED0 + i) for i in range(nk)]).astype(np.float32)
        om = inputs.omega_for(n)
        m = hh.Model(ctx, torch.from_numpy(kap), om)
        b = torch.from_numpy(np.stack([inputs.point_source(n, EVAL_SOURCE_SEED0 + i) for i in range(nk)])).to(dev)
        inst = list(range(nk))
        row = {}
        _, info = m.solve(b, inst=inst, max_iters=max_iters, precond=hh.HH_PRECOND_MG, want_hist=False)
        row["mg"] = info["iters"].tolist()
        row["mg_converged"] = int(info["converged"].sum())
        for name, net in nets.items():
            m.attach_net(net)
            _, info = m.solve(b, inst=inst, max_iters=max_iters, precond=hh.HH_PRECOND_CNN_MG, want_hist=False)
            row[name] = info["iters"].tolist()
            row[name + "_converged"] = int(info["converged"].sum())
        m.attach_net(None)
        m.close()
        res[str(n)] = row
        _log(f"[eval] {n}^2: mean iterations MG-only {np.mean(row['mg']):.1f}" +
             "".join(f", {k} {np.mean(row[k]):.1f}" for k in nets))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--block", type=int, default=100, help="steps per multiscale block")
    ap.add_argument("--val-every", type=int, default=250)
    ap.add_argument("--nval", type=int, default=256, help="validation pairs per size")
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--clip", type=float, default=2.0, help="clip at this multiple of the median gradient norm")
    ap.add_argument("--init-seed", type=int, default=0, help="seed of the initial parameters")
    ap.add_argument("--sizes", type=str, default="128,256", help="training grid sizes (128, 256, 512, 1024)")
    ap.add_argument("--eval-sizes", type=str, default="128,256,512")
    ap.add_argument("--eval-media", type=int, default=16)
    ap.add_argument("--eval-large", type=str, default="1024", help="sizes evaluated on fewer media")
    ap.add_argument("--eval-large-media", type=int, default=4)
    ap.add_argument("--eval-large-max-iters", type=int, default=8000)
    ap.add_argument("--out", type=str, default=os.path.join(os.path.dirname(__file__), "weights",
                                                          "net_ms128_256.bin"))
    ap.add_argument("--init-from", type=str, default="",
                    help="continue from this network file (parameters and Adam moments)")
    ap.add_argument("--step0", type=int, default=0,
                    help="steps already taken by --init-from: the training stream continues after them")
    ap.add_argument("--gen-seed", type=int, default=None, help="seed of the random vectors (default: --seed)")
    ap.add_argument("--explicit", action="store_true",
                    help="train the explicit U-Net (the coarsest level convolves with the kernels, Sec. 5.2)")
    ap.add_argument("--reuse", type=int, default=1,
                    help="steps that share one batch of media at sizes >= --reuse-from")
    ap.add_argument("--reuse-from", type=int, default=1024)
    ap.add_argument("--light", action="store_true",
                    help="train the lightweight network (inverted bottlenecks, batch norm, softplus; Sec. 4.4)")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("training runs on the GPU")
    ctx = hh.Context(0)
    init = inputs.init_light_params(args.init_seed) if args.light else inputs.init_net_params(args.init_seed)
    net = (hh.Net.load(ctx, args.init_from) if args.init_from
           else hh.Net(ctx, init, explicit=args.explicit, light=args.light))
    sizes = tuple(int(s) for s in args.sizes.split(","))
    if any(s not in SIZE_WEIGHT for s in sizes):
        sys.exit(f"training sizes must be among {sorted(SIZE_WEIGHT)}")
    seed = args.seed + args.step0 if args.gen_seed is None else args.gen_seed
    hist = train(ctx, net, args.steps, args.batch, args.lr, args.block, args.val_every, args.nval, seed,
                 sizes=sizes, clip=args.clip, step0=args.step0, reuse=args.reuse, reuse_from=args.reuse_from)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    _log(f"[train] saved {args.out} after {hist['seconds']:.0f} s ({hist['steps_per_s']:.2f} steps/s)")
    if net.light != args.light:
        init = inputs.init_light_params(args.init_seed) if net.light else inputs.init_net_params(args.init_seed)
    untrained = hh.Net(ctx, init, explicit=net.explicit, light=net.light)
    nets = {"cnn_untrained": untrained, "cnn_trained": net}
    ev = evaluate(ctx, nets, sizes=tuple(int(s) for s in args.eval_sizes.split(",") if s), nk=args.eval_media)
    ev.update(evaluate(ctx, nets, sizes=tuple(int(s) for s in args.eval_large.split(",") if s),
                       nk=args.eval_large_media, max_iters=args.eval_large_max_iters))
    rep = dict(args=vars(args), history=hist, evaluation=ev)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rep, f)
    _log("[train] done")


if __name__ == "__main__":
    main()
