"""The multi-step elimination chains of the reduced coarse solve, checked as
algebra on the host: for random block recurrences, the schedule the kernels
follow -- per level l the forward / backward combines, the chain over the kept
indices 2^l (i+1) - 1 with the product factors, then the fills from the deepest
level up -- reproduces the plain two-ended chains exactly (to rounding), for
every length of the reduced system and depths 0..3.  (The GPU tests check the
kernels themselves against the oracle's coarse solve.)"""
import numpy as np
import pytest


def _plain(M, P, R, g, Pp, Rp):
    p = M // 2
    y = {}
    for j in range(p):
        y[j] = g[j] + (P[j] @ y[j - 1] if j > 0 else 0)
    for j in range(M - 1, p, -1):
        y[j] = g[j] + (P[j] @ y[j + 1] if j < M - 1 else 0)

    def mid(ends):
        v = g[p].copy()
        if p >= 1:
            v = v + Pp @ ends[0]
        if p + 1 <= M - 1:
            v = v + Rp @ ends[1]
        return v

    x = {p: mid([y.get(p - 1), y.get(p + 1)])}
    for j in range(p - 1, -1, -1):
        x[j] = y[j] + R[j] @ x[j + 1]
    for j in range(p + 1, M):
        x[j] = y[j] + R[j] @ x[j - 1]
    return y, x, mid


def _multistep(M, D, P, R, g, mid):
    p = M // 2
    nst = [p, M - 1 - p]
    n_at = lambda l, e: nst[e] >> l
    base = lambda l, i: ((i + 1) << l) - 1
    rowf = lambda e, s: s if e == 0 else M - 1 - s
    rowb = lambda e, s: p - 1 - s if e == 0 else p + 1 + s
    FL = {}

    def mat(l, dr, e, i):  # dr 0: forward factor A_l(i), 1: backward B_l(i)
        if l == 0:
            return P[rowf(e, i)] if dr == 0 else R[rowb(e, i)]
        return FL[(l, dr, e, i)]

    for l in range(1, D + 1):  # the products, each level from the previous one
        for dr in (0, 1):
            for e in (0, 1):
                for i in range(n_at(l, e)):
                    if dr == 0 and i < 1:
                        continue
                    FL[(l, dr, e, i)] = mat(l - 1, dr, e, 2 * i + 1) @ mat(l - 1, dr, e, 2 * i)
    X, hw, E = {}, {}, [None, None]

    def src(l, dr, row):
        if l == 0:
            return g[row] if dr == 0 else X[row]
        return hw[row]

    def phase(kind, l):  # 4/6 combine, 5/7 fill (forward / backward), level l >= 1
        dr = 0 if kind in (4, 5) else 1
        rowfn = rowf if dr == 0 else rowb
        out = {}
        for e in (0, 1):
            for i in range(n_at(l - 1, e)):
                if (i % 2 == 1) != (kind in (4, 6)):
                    continue
                si = base(l - 1, i)
                r = rowfn(e, si)
                if kind in (4, 6):
                    rp = rowfn(e, base(l - 1, i - 1))
                    out[("h", r)] = src(l - 1, dr, r) + mat(l - 1, dr, e, i) @ src(l - 1, dr, rp)
                elif dr == 0:
                    v = src(l - 1, 0, r) + (mat(l - 1, 0, e, i) @ X[rowfn(e, base(l - 1, i - 1))] if i > 0 else 0)
                    if si == nst[e] - 1:
                        E[e] = v
                    out[("x", r)] = v
                else:
                    rp = p if i == 0 else rowfn(e, base(l - 1, i - 1))
                    out[("x", r)] = src(l - 1, 1, r) + mat(l - 1, 1, e, i) @ X[rp]
        for (kk, r), v in out.items():
            (hw if kk == "h" else X)[r] = v

    def chain(dr):
        for e in (0, 1):
            prev = None if dr == 0 else X[p]
            for i in range(n_at(D, e)):
                si = base(D, i)
                r = (rowf if dr == 0 else rowb)(e, si)
                has = dr == 1 or i > 0
                v = src(D, dr, r) + (mat(D, dr, e, i) @ prev if has else 0)
                X[r] = v
                prev = v
                if dr == 0 and si == nst[e] - 1:
                    E[e] = v

    for l in range(1, D + 1):
        phase(4, l)
    chain(0)
    for l in range(D, 0, -1):
        phase(5, l)
    y = {j: X[j] for j in range(M) if j != p}
    for l in range(1, D + 1):
        phase(6, l)
    X[p] = mid(E)
    chain(1)
    for l in range(D, 0, -1):
        phase(7, l)
    return y, X


@pytest.mark.parametrize("D", [0, 1, 2, 3])
def test_multistep_chains_reproduce_the_plain_chains(D):
    rng = np.random.default_rng(7 + D)
    d = 3
    rn = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)) * 0.3
    for M in range(1, 48):
        P = {j: rn(d, d) for j in range(M)}
        R = {j: rn(d, d) for j in range(M)}
        g = {j: rn(d) for j in range(M)}
        Pp, Rp = rn(d, d), rn(d, d)
        y_ref, x_ref, mid = _plain(M, P, R, g, Pp, Rp)
        y, x = _multistep(M, D, P, R, g, mid)
        for j in y_ref:
            assert np.allclose(y[j], y_ref[j], rtol=1e-12, atol=1e-12), (M, D, "y", j)
        for j in x_ref:
            assert np.allclose(x[j], x_ref[j], rtol=1e-12, atol=1e-12), (M, D, "x", j)
