"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws random numbers and shapes them into problem inputs
(slowness models, sources, random vectors, initial network weights).  It holds
none of the solver's or the network's arithmetic.

The paper draws its slowness models from image datasets (CIFAR-10, OpenFWI,
STL-10; Sec. 4.3, "Slowness Model Datasets") that are resized, smoothed and
normalised to [0.25, 1].  Those datasets are not available, so two synthetic
families with the same value range stand in for them:

* ``grf_slowness``: a smooth Gaussian random field (correlation length 0.1 of
  the unit square), the analogue of the smoothed natural images;
* ``layered_slowness``: piecewise-constant tilted layers with optional blocks,
  the analogue of the layered OpenFWI-style media.
"""
from __future__ import annotations

import math

import numpy as np

KAPPA_MIN = 0.25
KAPPA_MAX = 1.0


def _minmax(f: np.ndarray, lo: float = KAPPA_MIN, hi: float = KAPPA_MAX) -> np.ndarray:
    fmin, fmax = float(f.min()), float(f.max())
    if fmax - fmin <= 0.0:
        return np.full_like(f, hi)
    return lo + (hi - lo) * (f - fmin) / (fmax - fmin)


def _fp32_exact(k: np.ndarray) -> np.ndarray:
    """Round to the nearest float32 and return float64.

    The library takes the slowness in FP32; rounding here hands the CPU checker
    and the library the same medium, so both assemble the same operator.
    """
    return np.asarray(k, dtype=np.float32).astype(np.float64)


def grf_slowness(n: int, seed: int, corr: float = 0.1) -> np.ndarray:
    """Gaussian random field on an n x n grid mapped to [0.25, 1] (float64
    holding float32-representable values).

    White noise is smoothed by a periodic Gaussian filter of standard deviation
    ``corr * n`` cells (applied in Fourier space), then min-max normalised.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n))
    sigma = corr * n
    fy = np.fft.fftfreq(n)[:, None]
    fx = np.fft.rfftfreq(n)[None, :]
    filt = np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    field = np.fft.irfft2(np.fft.rfft2(white) * filt, s=(n, n))
    return _fp32_exact(_minmax(field))


def layered_slowness(n: int, seed: int) -> np.ndarray:
    """Layered / blocky slowness on an n x n grid with values in [0.25, 1]
    (float64 holding float32-representable values).

    4-10 layers separated by tilted straight interfaces y = a_k + t_k (x - 1/2)
    with t_k ~ U(-0.3, 0.3); every layer gets a value ~ U[0.25, 1].  With
    probability 1/2, 1-3 axis-aligned blocks of random value are painted on top.
    """
    rng = np.random.default_rng(seed)
    nlayers = int(rng.integers(4, 11))
    offsets = np.sort(rng.uniform(0.0, 1.0, nlayers - 1))
    tilts = rng.uniform(-0.3, 0.3, nlayers - 1)
    values = rng.uniform(KAPPA_MIN, KAPPA_MAX, nlayers)
    c = (np.arange(n) + 0.5) / n
    y = c[:, None]
    x = c[None, :]
    idx = np.zeros((n, n), dtype=np.int64)
    for a, t in zip(offsets, tilts):
        idx += (y > a + t * (x - 0.5)).astype(np.int64)
    kappa = values[idx]
    if rng.uniform() < 0.5:
        for _ in range(int(rng.integers(1, 4))):
            x0, x1 = np.sort(rng.uniform(0.0, 1.0, 2))
            y0, y1 = np.sort(rng.uniform(0.0, 1.0, 2))
            v = rng.uniform(KAPPA_MIN, KAPPA_MAX)
            mask = (y >= y0) & (y <= y1) & (x >= x0) & (x <= x1)
            kappa = np.where(mask, v, kappa)
    return _fp32_exact(kappa)


def slowness(n: int, seed: int, family: str) -> np.ndarray:
    if family == "grf":
        return grf_slowness(n, seed)
    if family == "layered":
        return layered_slowness(n, seed)
    raise ValueError(f"unknown slowness family {family!r}")


def omega_for(n: int, kappa: np.ndarray | None = None, ppw: float = 10.0) -> float:
    """Angular frequency giving ``ppw`` points per wavelength at the largest slowness.

    The ten-points-per-wavelength rule bounds omega * kappa * h by 2 pi / 10 (Sec. 3.1).
    With h = 1/n this sets omega = 2 pi n / (ppw * max kappa).
    """
    kmax = KAPPA_MAX if kappa is None else float(np.max(kappa))
    return 2.0 * math.pi * n / (ppw * kmax)


def point_source_cells(n: int, seed: int, count: int = 1, margin: int = 16) -> list[tuple[int, int]]:
    """Seeded interior cells (row, col) at distance >= ``margin`` from every edge."""
    rng = np.random.default_rng(seed)
    lo, hi = margin, n - margin
    if hi <= lo:
        lo, hi = 0, n
    return [(int(rng.integers(lo, hi)), int(rng.integers(lo, hi))) for _ in range(count)]


def point_source(n: int, seed: int, margin: int = 16) -> np.ndarray:
    """A unit point source (value 1 at one seeded interior cell), complex128 n x n."""
    (i, j), = point_source_cells(n, seed, 1, margin)
    b = np.zeros((n, n), dtype=np.complex128)
    b[i, j] = 1.0
    return b


def random_complex(shape, seed: int) -> np.ndarray:
    """Standard circular complex Gaussian draws: real and imaginary parts iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# Network description and seeded initial weights.
# ---------------------------------------------------------------------------

def net_layers(ch=(16, 32, 64, 64)):
    """Layer list of the encoder-solver network (name, kind, cin, cout).

    kind: 'c' = 3x3 conv stride 1, 'd' = 3x3 conv stride 2 (downsample),
    't' = 3x3 transposed conv stride 2 (upsample), 'd4'/'t4' = the coarsest
    down/up pair whose stride is 2 for n >= 512 and 1 below (Sec. 5.3).
    Convolution weights are stored (cout, cin, 3, 3); transposed-convolution
    weights (cin, cout, 3, 3).
    """
    c1, c2, c3, c4 = ch
    L = []
    # encoder: strided conv + two conv/act modules per level
    L += [("enc1_d", "d", 2, c1), ("enc1_c1", "c", c1, c1), ("enc1_c2", "c", c1, c1)]
    L += [("enc2_d", "d", c1, c2), ("enc2_c1", "c", c2, c2), ("enc2_c2", "c", c2, c2)]
    L += [("enc3_d", "d", c2, c3), ("enc3_c1", "c", c3, c3), ("enc3_c2", "c", c3, c3)]
    # solver down path
    L += [("s1_d", "d", 2, c1), ("s1_c1", "c", c1, c1), ("s1_c2", "c", c1, c1)]
    L += [("s2_d", "d", c1, c2), ("s2_c1", "c", c2, c2), ("s2_c2", "c", c2, c2)]
    L += [("s3_d", "d", c2, c3), ("s3_c1", "c", c3, c3), ("s3_c2", "c", c3, c3)]
    L += [("s4_d", "d4", c3, c4), ("s4_c1", "c", c4, c4), ("s4_c2", "c", c4, c4)]
    # solver up path
    L += [("u3_t", "t4", c4, c3), ("u3_c1", "c", c3, c3), ("u3_c2", "c", c3, c3)]
    L += [("u2_t", "t", c3, c2), ("u2_c1", "c", c2, c2), ("u2_c2", "c", c2, c2)]
    L += [("u1_t", "t", c2, c1), ("u1_c1", "c", c1, c1), ("u1_c2", "c", c1, c1)]
    L += [("out", "c", c1, 2)]
    return L


def init_net_params(seed: int, ch=(16, 32, 64, 64)) -> dict[str, np.ndarray]:
    """Seeded initial weights (float64): uniform(+-1/sqrt(fan_in)) for every
    conv weight and bias (PyTorch's default Kaiming-uniform rule), and the
    implicit-layer kernels set to L + iI with L the 5-point Laplacian
    (Sec. 5.3).  ``implicit_K`` has shape (channels/2, 3, 3) complex.
    """
    rng = np.random.default_rng(seed)
    p: dict[str, np.ndarray] = {}
    for name, kind, cin, cout in net_layers(ch):
        if kind in ("t", "t4"):
            fan_in = cout * 9  # PyTorch computes ConvTranspose fan-in from weight dim 1
            shape = (cin, cout, 3, 3)
        else:
            fan_in = cin * 9
            shape = (cout, cin, 3, 3)
        bound = 1.0 / math.sqrt(fan_in)
        p[name + ".w"] = rng.uniform(-bound, bound, shape)
        p[name + ".b"] = rng.uniform(-bound, bound, (cout,))
    lap = np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])
    nk = ch[3] // 2
    p["implicit_K"] = np.broadcast_to(lap + 1j * np.array([[0, 0, 0], [0, 1.0, 0], [0, 0, 0]]),
                                      (nk, 3, 3)).astype(np.complex128).copy()
    return p


# ---------------------------------------------------------------------------
# Out-of-distribution media (stand-ins for the paper's Marmousi, SEG/EAGE salt
# dome and Overthrust velocity models, which are not available here).  Each
# builds a velocity model v (km/s) and returns kappa = 1/v normalised to a
# largest value of 1 (the normalisation of Sec. 5.4), on a square n x n grid.
# ---------------------------------------------------------------------------

def _kappa_from_velocity(v: np.ndarray) -> np.ndarray:
    k = 1.0 / v
    return _fp32_exact(k / k.max())


def salt_slowness(n: int, seed: int) -> np.ndarray:
    """Sediments whose velocity grows with depth (1.5 -> 4 km/s, mild layering)
    around a salt body (4.5 km/s) with a rough dome-shaped top and steep flanks."""
    rng = np.random.default_rng(seed)
    c = (np.arange(n) + 0.5) / n
    y, x = c[:, None], c[None, :]
    nl = int(rng.integers(12, 20))
    tops = np.sort(rng.uniform(0.0, 1.0, nl))
    dips = rng.uniform(-0.08, 0.08, nl)
    layer = np.zeros((n, n), dtype=np.int64)
    for a, t in zip(tops, dips):
        layer += (y > a + t * (x - 0.5)).astype(np.int64)
    v = 1.5 + 2.5 * (layer / nl) ** 0.8 + rng.uniform(-0.15, 0.15, nl + 1)[layer]
    # salt: top y = y0 - h exp(-((x - xc)/w)^2) + small roughness, flanks down to the bottom
    xc, w, y0, h = rng.uniform(0.35, 0.65), rng.uniform(0.12, 0.22), rng.uniform(0.55, 0.7), rng.uniform(0.2, 0.35)
    kx = np.arange(1, 6)
    rough = (rng.uniform(-0.02, 0.02, 5)[:, None] * np.sin(2 * np.pi * kx[:, None] * x[0][None, :])).sum(0)
    top = y0 - h * np.exp(-((x[0] - xc) / w) ** 2) + rough
    inside = (y > top[None, :]) & (np.abs(x - xc) < 1.6 * w * np.sqrt(np.maximum(0.0, 1.0 - (y - top[None, :]) * 0.3)))
    v = np.where(inside, 4.5, v)
    return _kappa_from_velocity(v)


def faulted_slowness(n: int, seed: int) -> np.ndarray:
    """Many thin dipping layers (velocity 1.5 -> 4.5 km/s with depth and random
    contrasts) cut by two normal faults that offset them (a Marmousi-like
    structure)."""
    rng = np.random.default_rng(seed)
    c = (np.arange(n) + 0.5) / n
    y, x = c[:, None], c[None, :]
    nl = int(rng.integers(25, 40))
    tops = np.sort(rng.uniform(0.0, 1.0, nl))
    vals = 1.5 + 3.0 * np.sort(rng.uniform(0.0, 1.0, nl + 1)) + rng.uniform(-0.3, 0.3, nl + 1)
    vals = np.clip(vals, 1.5, 4.5)
    yy = y + 0.15 * (x - 0.5)  # regional dip
    for _ in range(2):  # faults: x = x0 + s (y - 0.5); the hanging wall drops by d
        x0, s, d = rng.uniform(0.25, 0.75), rng.uniform(-0.4, 0.4), rng.uniform(0.03, 0.08)
        yy = yy - d * (x > x0 + s * (y - 0.5))
    layer = np.zeros((n, n), dtype=np.int64)
    for a in tops:
        layer += (yy > a).astype(np.int64)
    return _kappa_from_velocity(vals[layer])


def folded_slowness(n: int, seed: int) -> np.ndarray:
    """Folded layers (an anticline and a syncline) with a thrust fault that
    repeats part of the sequence (an Overthrust-like structure)."""
    rng = np.random.default_rng(seed)
    c = (np.arange(n) + 0.5) / n
    y, x = c[:, None], c[None, :]
    nl = int(rng.integers(10, 18))
    tops = np.sort(rng.uniform(0.05, 1.0, nl))
    vals = np.clip(2.0 + 4.0 * np.sort(rng.uniform(0.0, 1.0, nl + 1)) + rng.uniform(-0.4, 0.4, nl + 1), 2.0, 6.0)
    amp, per, ph = rng.uniform(0.05, 0.12), rng.uniform(0.6, 1.2), rng.uniform(0.0, 2 * np.pi)
    yy = y - amp * np.sin(2 * np.pi * x / per + ph) * (1.0 - 0.5 * y)
    # thrust: above the plane y = y0 + s (x - 0.5) the block is pushed up by d
    y0, s, d = rng.uniform(0.35, 0.6), rng.uniform(0.5, 1.0), rng.uniform(0.08, 0.15)
    yy = np.where(y < y0 + s * (x - 0.5), yy + d, yy)
    layer = np.zeros((n, n), dtype=np.int64)
    for a in tops:
        layer += (yy > a).astype(np.int64)
    return _kappa_from_velocity(vals[layer])


OOD_FAMILIES = {"salt": salt_slowness, "faulted": faulted_slowness, "folded": folded_slowness}


# ---------------------------------------------------------------------------
# The paper's lightweight network (Sec. 4.4, Sec. 5.3): modules of a 3x3
# convolution, batch normalisation and softplus; inverted bottlenecks (1x1
# expansion by LIGHT_EXPAND, depthwise 3x3, 1x1 shrink, sum with the module's
# input) on the first three solver levels.
# ---------------------------------------------------------------------------
LIGHT_EXPAND = 6


def net_layers_light(ch=(16, 32, 64, 64), t: int = LIGHT_EXPAND):
    """Layer list of the lightweight encoder-solver network (name, kind, cin, cout).

    kinds: 'd' 3x3 stride-2 conv, 'd4' the coarsest down conv (stride 2 from
    n = 512, else 1), 'cb' 3x3 conv + batch norm + softplus, 'e' 1x1 expansion
    + batch norm + softplus, 'w' depthwise 3x3 + batch norm + softplus (cin =
    cout channels), 's' 1x1 shrink + batch norm (added to the bottleneck's
    input), 't' / 't4' 3x3 stride-2 transposed conv, 'c' the 3x3 projection.
    Layers followed by batch norm have no bias (the normalisation removes it).
    """
    c1, c2, c3, c4 = ch
    L = []
    for lvl, (ci, co) in enumerate(((2, c1), (c1, c2), (c2, c3)), start=1):
        L += [(f"enc{lvl}_d", "d", ci, co), (f"enc{lvl}_c1", "cb", co, co), (f"enc{lvl}_c2", "cb", co, co)]
    for lvl, (ci, co) in enumerate(((2, c1), (c1, c2), (c2, c3)), start=1):
        L += [(f"s{lvl}_d", "d", ci, co), (f"s{lvl}_e", "e", co, t * co), (f"s{lvl}_w", "w", t * co, t * co),
              (f"s{lvl}_s", "s", t * co, co)]
    L += [("s4_d", "d4", c3, c4), ("s4_c1", "cb", c4, c4), ("s4_c2", "cb", c4, c4)]
    L += [("u3_t", "t4", c4, c3), ("u3_c1", "cb", c3, c3), ("u3_c2", "cb", c3, c3)]
    L += [("u2_t", "t", c3, c2), ("u2_c1", "cb", c2, c2), ("u2_c2", "cb", c2, c2)]
    L += [("u1_t", "t", c2, c1), ("u1_c1", "cb", c1, c1), ("u1_c2", "cb", c1, c1)]
    L += [("out", "c", c1, 2)]
    return L


def light_has_bn(kind: str) -> bool:
    return kind in ("cb", "e", "w", "s")


def init_light_params(seed: int, ch=(16, 32, 64, 64), t: int = LIGHT_EXPAND) -> dict[str, np.ndarray]:
    """Seeded initial parameters of the lightweight network (float64): Kaiming-
    uniform weights (bound 1/sqrt(fan_in)), biases likewise where the layer has
    one, batch-norm scale 1 and shift 0 with running mean 0 and variance 1, and
    the implicit kernels L + iI."""
    rng = np.random.default_rng(seed)
    p: dict[str, np.ndarray] = {}
    for name, kind, cin, cout in net_layers_light(ch, t):
        if kind in ("t", "t4"):
            shape, fan_in = (cin, cout, 3, 3), cout * 9
        elif kind in ("e", "s"):
            shape, fan_in = (cout, cin), cin
        elif kind == "w":
            shape, fan_in = (cout, 3, 3), 9
        else:
            shape, fan_in = (cout, cin, 3, 3), cin * 9
        bound = 1.0 / math.sqrt(fan_in)
        p[name + ".w"] = rng.uniform(-bound, bound, shape)
        if light_has_bn(kind):
            p[name + ".g"] = np.ones(cout)
            p[name + ".be"] = np.zeros(cout)
            p[name + ".rm"] = np.zeros(cout)
            p[name + ".rv"] = np.ones(cout)
        else:
            p[name + ".b"] = rng.uniform(-bound, bound, (cout,))
    lap = np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])
    nk = ch[3] // 2
    p["implicit_K"] = np.broadcast_to(lap + 1j * np.array([[0, 0, 0], [0, 1.0, 0], [0, 0, 0]]),
                                      (nk, 3, 3)).astype(np.complex128).copy()
    return p
