"""The network's flat FP32 parameter vector and its file format, in plain
NumPy (no GPU library needed).

Parameter order (the layout of include/hh.h): for every layer of
inputs.net_layers in order, the weights ((cout, cin, 3, 3) for convolutions,
(cin, cout, 3, 3) for transposed convolutions) then the biases; then the
complex 3x3 implicit-layer kernels as (re, im) pairs.

File: 8-byte magic "HHNET002", int32 channels[4], int32 coarsest-layer kind
(0 implicit, 1 explicit), int64 parameter count, int64 optimiser step, int32
has_optimiser_state, FP32 parameters, then (when present) the FP32 Adam first
and second moments.  Files with magic "HHNET001" have no kind field (implicit)."""
from __future__ import annotations

import numpy as np

from . import inputs

MAGIC = b"HHNET002"
MAGIC1 = b"HHNET001"

NET_LAYER_NAMES = [name for name, _, _, _ in inputs.net_layers((16, 32, 64, 64))]


def flatten_params(p: dict, ch=(16, 32, 64, 64)) -> np.ndarray:
    """Named parameters (weights, biases, complex implicit kernels) -> the flat FP32 vector."""
    parts = []
    for name, _, _, _ in inputs.net_layers(ch):
        parts.append(np.asarray(p[name + ".w"], dtype=np.float64).ravel())
        parts.append(np.asarray(p[name + ".b"], dtype=np.float64).ravel())
    K = np.asarray(p["implicit_K"])
    parts.append(np.stack([K.real, K.imag], axis=-1).ravel())
    return np.concatenate(parts).astype(np.float32)


def unflatten_params(flat: np.ndarray, ch=(16, 32, 64, 64)) -> dict:
    """The flat FP32 vector -> named FP64 parameters."""
    out = {}
    off = 0
    for name, kind, cin, cout in inputs.net_layers(ch):
        shape = (cin, cout, 3, 3) if kind in ("t", "t4") else (cout, cin, 3, 3)
        sz = int(np.prod(shape))
        out[name + ".w"] = flat[off:off + sz].reshape(shape).astype(np.float64)
        off += sz
        out[name + ".b"] = flat[off:off + cout].astype(np.float64)
        off += cout
    nk = ch[3] // 2
    k = flat[off:off + nk * 18].reshape(nk, 3, 3, 2).astype(np.float64)
    out["implicit_K"] = k[..., 0] + 1j * k[..., 1]
    return out


def read_header(path: str) -> dict:
    """{'ch': channels, 'explicit': bool} of a network file."""
    with open(path, "rb") as f:
        magic = f.read(8)
        if magic not in (MAGIC, MAGIC1):
            raise ValueError(f"{path} is not a network file")
        ch = tuple(int(c) for c in np.frombuffer(f.read(16), dtype=np.int32))
        explicit = bool(np.frombuffer(f.read(4), dtype=np.int32)[0]) if magic == MAGIC else False
    return {"ch": ch, "explicit": explicit}


def read_params(path: str) -> tuple[np.ndarray, tuple[int, ...]]:
    """(flat FP32 parameters, channels) of a network file."""
    with open(path, "rb") as f:
        magic = f.read(8)
        if magic not in (MAGIC, MAGIC1):
            raise ValueError(f"{path} is not a network file")
        ch = tuple(int(c) for c in np.frombuffer(f.read(16), dtype=np.int32))
        if magic == MAGIC:
            f.read(4)  # coarsest-layer kind
        npar = int(np.frombuffer(f.read(8), dtype=np.int64)[0])
        f.read(8 + 4)  # optimiser step, has_optimiser_state
        flat = np.frombuffer(f.read(4 * npar), dtype=np.float32)
    if flat.size != npar:
        raise ValueError(f"{path}: truncated")
    return flat.copy(), ch
