"""The network's flat FP32 parameter vector and its file format, in plain
NumPy (no GPU library needed).

Parameter order (the layout of include/hh.h): for every layer of
inputs.net_layers in order, the weights ((cout, cin, 3, 3) for convolutions,
(cin, cout, 3, 3) for transposed convolutions) then the biases; then the
complex 3x3 implicit-layer kernels as (re, im) pairs.

The lightweight network (inputs.net_layers_light): per layer the weights
((cout, cin, 3, 3), (cin, cout, 3, 3) for transposed, (cout, cin) for 1x1,
(cout, 3, 3) for depthwise), then for batch-normalised layers the scale,
shift, running mean and running variance, otherwise the biases; then the
implicit kernels.

File: 8-byte magic "HHNET002", int32 channels[4], int32 flags (bit 0: explicit
coarsest layer, bit 1: lightweight network), int64 parameter count, int64
optimiser step, int32 has_optimiser_state, FP32 parameters, then (when
present) the FP32 Adam first and second moments.  Files with magic "HHNET001"
have no flags field (the implicit U-Net)."""
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


def _light_shape(kind: str, cin: int, cout: int) -> tuple[int, ...]:
    if kind in ("t", "t4"):
        return (cin, cout, 3, 3)
    if kind in ("e", "s"):
        return (cout, cin)
    if kind == "w":
        return (cout, 3, 3)
    return (cout, cin, 3, 3)


def flatten_light_params(p: dict, ch=(16, 32, 64, 64)) -> np.ndarray:
    """Named parameters of the lightweight network -> the flat FP32 vector."""
    parts = []
    for name, kind, _, _ in inputs.net_layers_light(ch):
        parts.append(np.asarray(p[name + ".w"], dtype=np.float64).ravel())
        keys = (".g", ".be", ".rm", ".rv") if inputs.light_has_bn(kind) else (".b",)
        for k in keys:
            parts.append(np.asarray(p[name + k], dtype=np.float64).ravel())
    K = np.asarray(p["implicit_K"])
    parts.append(np.stack([K.real, K.imag], axis=-1).ravel())
    return np.concatenate(parts).astype(np.float32)


def unflatten_light_params(flat: np.ndarray, ch=(16, 32, 64, 64)) -> dict:
    """The lightweight network's flat FP32 vector -> named FP64 parameters."""
    out = {}
    off = 0
    for name, kind, cin, cout in inputs.net_layers_light(ch):
        shape = _light_shape(kind, cin, cout)
        sz = int(np.prod(shape))
        out[name + ".w"] = flat[off:off + sz].reshape(shape).astype(np.float64)
        off += sz
        keys = (".g", ".be", ".rm", ".rv") if inputs.light_has_bn(kind) else (".b",)
        for k in keys:
            out[name + k] = flat[off:off + cout].astype(np.float64)
            off += cout
    nk = ch[3] // 2
    k = flat[off:off + nk * 18].reshape(nk, 3, 3, 2).astype(np.float64)
    out["implicit_K"] = k[..., 0] + 1j * k[..., 1]
    return out


def read_header(path: str) -> dict:
    """{'ch': channels, 'explicit': bool, 'light': bool} of a network file."""
    with open(path, "rb") as f:
        magic = f.read(8)
        if magic not in (MAGIC, MAGIC1):
            raise ValueError(f"{path} is not a network file")
        ch = tuple(int(c) for c in np.frombuffer(f.read(16), dtype=np.int32))
        flags = int(np.frombuffer(f.read(4), dtype=np.int32)[0]) if magic == MAGIC else 0
    return {"ch": ch, "explicit": bool(flags & 1), "light": bool(flags & 2)}


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
