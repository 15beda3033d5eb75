"""FP64 CPU oracle of the preconditioner composition, the two-phase solve and the
method-generated training data.

TEST INFRASTRUCTURE ONLY (see ``oracle/helmholtz.py``).
"""
from __future__ import annotations

import numpy as np

from . import cnn as C
from . import helmholtz as H


class NetPrecond:
    """Network part of the preconditioner for one slowness model: the encoder is
    applied once and its features reused for every application (Sec. 4.1)."""

    def __init__(self, net: C.Net, prob: H.Problem):
        self.net, self.prob = net, prob
        self.h = prob.h
        kin = C.kappa_features(prob.k2w2, prob.gamma, prob.h)
        self.enc, _ = net.encode(kin)
        self.nc = C.coarsest_size(prob.n)
        self.Ghat = None if net.explicit else C.green_hat(net.p["implicit_K"], self.nc)[0]

    def __call__(self, r: np.ndarray) -> np.ndarray:
        """e = s * Net(h^2 r / s), s = rms(h^2 r) (single right-hand side)."""
        s = C.residual_scale(r[None], self.h)[0]
        if s == 0.0:
            return np.zeros_like(r)
        rin = C.to_channels(self.h * self.h * r[None] / s)
        out, _ = self.net.solve(rin, self.enc, self.Ghat)
        return s * C.from_channels(out)[0]


def cnn_mg_precond(prob: H.Problem, netp: NetPrecond, v: np.ndarray) -> np.ndarray:
    """CNN+MG preconditioner: the network's error estimate is the initial guess of
    the shifted-Laplacian V-cycle on the same right-hand side (Sec. 4.1)."""
    return prob.hier.vcycle(v, netp(v))


def solve_two_phase(prob: H.Problem, netp: NetPrecond, b: np.ndarray, rtol=1e-6, max_iters=2000,
                    warm_iters=3, restart=10, fallback=True, probe_ratio=0.5, stats=None):
    """Sec. 4.1: a few MG-only FGMRES iterations, then FGMRES(restart) with the
    CNN+MG preconditioner from that iterate.  Iterations of both phases count.

    With ``fallback`` the two preconditioners judge each other, one restart
    cycle at a time (the reading of the method used here; the paper gives no
    rule): a cycle whose true residual ratio (end / start) exceeds
    probe_ratio is followed by one cycle with the other preconditioner
    (CNN+MG <-> MG-only).  If that probe cycle reduces the residual more, its
    preconditioner takes over; otherwise the previous one resumes, and the
    number of cycles before the next probe may run doubles (2, 4, 8, ...; a
    switch resets it).  ``stats`` (a dict, optional) receives ``probes`` and
    ``mg_cycles`` (cycles after the warm start run with MG-only).

    A network application with a non-finite result ends its cycle at once:
    that cycle's directions are dropped (x keeps its value from the cycle's
    start; the applications made count as iterations) and the right-hand side
    continues with MG-only (the failure rule of the library)."""
    x, its, hist, rel = H.fgmres(prob.A, b, prob.mg, None, restart, rtol, warm_iters)
    apps = [0]

    class _NonFinite(Exception):
        pass

    def cnn(v):
        apps[0] += 1
        z = cnn_mg_precond(prob, netp, v)
        if not np.all(np.isfinite(z)):
            raise _NonFinite()
        return z

    cur, probing, q_base, wait, gap, probes, mg_cycles = "cnn", False, None, 0, 0, 0, 0
    cnn_off = False
    while rel > rtol and its < max_iters:
        if cur == "mg":
            mg_cycles += 1
        rel0 = rel
        if cur == "cnn":
            apps[0] = 0
            try:
                x, its, h, rel = H.fgmres(prob.A, b, cnn, x, restart, rtol, max_iters, iters_done=its, cycles=1)
            except _NonFinite:
                its += apps[0]
                hist = hist + [rel0] * apps[0]
                cur, cnn_off, probing = "mg", True, False
                continue
        else:
            x, its, h, rel = H.fgmres(prob.A, b, prob.mg, x, restart, rtol, max_iters, iters_done=its, cycles=1)
        hist = hist + h[1:]
        if cnn_off:
            continue
        q = rel / rel0
        other = "mg" if cur == "cnn" else "cnn"
        if probing:
            probing = False
            if q < q_base:
                gap, wait = 0, 0
            else:
                gap = 2 * gap if gap > 0 else 2
                wait = gap
                cur = other
        else:
            q_base = q
            if fallback and q > probe_ratio and wait <= 0:
                probing = True
                probes += 1
                cur = other
            elif wait > 0:
                wait -= 1
    if stats is not None:
        stats["probes"] = probes
        stats["mg_cycles"] = mg_cycles
    return x, its, hist, rel


def training_pair(prob: H.Problem, x: np.ndarray, k: int):
    """Eq. 20: b = A x, x~ = k iterations of MG-preconditioned FGMRES from 0,
    e = x - x~, r = b - A x~ (= A e).  ``x`` is the random vector (an input)."""
    b = prob.A(x)
    xt, its, _, _ = H.fgmres(prob.A, b, prob.mg, None, 10, 0.0, k)
    e = x - xt
    r = b - prob.A(xt)
    return e, r
