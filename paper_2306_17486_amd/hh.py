"""Thin ctypes binding of libhh (include/hh.h).

Functions named ``hh_*`` mirror the C entry points one to one and only marshal
arguments.  The small ``Context`` / ``Model`` / ``Net`` wrappers take torch
tensors, pass their device pointers and return results; every numerical step
runs in the library's HIP kernels.  There is no fallback: if ``libhh.so`` is
missing or cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhh.so")

HH_OK = 0
HH_NOT_CONVERGED = 1
HH_ERR_ARG = -1
HH_ERR_HIP = -2
HH_ERR_NOMEM = -3
HH_ERR_STATE = -4
HH_ERR_BREAKDOWN = -5
HH_PRECOND_MG = 0
HH_PRECOND_CNN_MG = 1


class HHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libhh error {status}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_17486_amd.build`")
_lib = C.CDLL(LIB_PATH)


class hh_model_desc(C.Structure):
    _fields_ = [("n", C.c_int), ("omega", C.c_double), ("abl_width", C.c_int), ("abl_gamma_max", C.c_double),
                ("gamma0", C.c_double), ("sl_beta", C.c_double), ("levels", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("jacobi_w", C.c_double), ("coarse_reduce", C.c_int),
                ("coarse_iters", C.c_int)]


class hh_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("rtol", C.c_double), ("precond", C.c_int),
                ("warm_mg_iters", C.c_int), ("use_x0", C.c_int), ("fixed_iters", C.c_int), ("fallback", C.c_int),
                ("probe_ratio", C.c_double), ("graph", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_IP = C.POINTER(C.c_int)
_DP = C.POINTER(C.c_double)


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


hh_version = _sig("hh_version", C.c_char_p)
hh_last_error = _sig("hh_last_error", C.c_char_p)
hh_ctx_create = _sig("hh_ctx_create", _I, _I, _P, ALLOC_FN, FREE_FN, _P, C.POINTER(_P))
hh_ctx_destroy = _sig("hh_ctx_destroy", _I, _P)
hh_model_desc_default = _sig("hh_model_desc_default", None, C.POINTER(hh_model_desc))
hh_model_create = _sig("hh_model_create", _I, _P, C.POINTER(hh_model_desc), _I, _P, C.POINTER(_P))
hh_model_destroy = _sig("hh_model_destroy", _I, _P)
hh_solve_opts_default = _sig("hh_solve_opts_default", None, C.POINTER(hh_solve_opts))
hh_solve = _sig("hh_solve", _I, _P, _P, _I, _IP, _P, _P, C.POINTER(hh_solve_opts), _DP, _IP, _IP, _DP, _IP, _IP)
hh_solve_batch = _sig("hh_solve_batch", _I, _P, _I, _P, _IP, _P, _P, _P, C.POINTER(hh_solve_opts), _P, _P, _P, _P,
                      _P)
hh_apply_operator = _sig("hh_apply_operator", _I, _P, _I, _D, _I, _IP, _P, _P)
hh_apply_vcycle = _sig("hh_apply_vcycle", _I, _P, _I, _IP, _P, _P, _P)
class hh_net_desc(C.Structure):
    _fields_ = [("ch", C.c_int * 4), ("explicit_coarse", C.c_int), ("arch", C.c_int)]


HH_ARCH_UNET, HH_ARCH_LIGHT = 0, 1


_FP = C.POINTER(C.c_float)
hh_net_create = _sig("hh_net_create", _I, _P, C.POINTER(hh_net_desc), _FP, C.POINTER(_P))
hh_net_destroy = _sig("hh_net_destroy", _I, _P)
hh_net_num_params = _sig("hh_net_num_params", C.c_size_t, _P)
hh_net_get_params = _sig("hh_net_get_params", _I, _P, _FP)
hh_net_set_params = _sig("hh_net_set_params", _I, _P, _FP)
hh_net_save = _sig("hh_net_save", _I, _P, C.c_char_p)
hh_net_load = _sig("hh_net_load", _I, _P, C.c_char_p, C.POINTER(_P))
hh_model_attach_net = _sig("hh_model_attach_net", _I, _P, _P)
hh_net_forward = _sig("hh_net_forward", _I, _P, _I, _IP, _P, _P)
hh_apply_cnn_precond = _sig("hh_apply_cnn_precond", _I, _P, _I, _IP, _P, _P)
hh_conv_test = _sig("hh_conv_test", _I, _P, _I, _I, _I, _I, _I, _I, _P, _P, _I, _P, _P, _I, _P, _P, _IP, _I)
hh_conv_pair_test = _sig("hh_conv_pair_test", _I, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _P, _IP, _I)
hh_conv_variants = _sig("hh_conv_variants", _I, _I, _I, _I, _IP, _I)
hh_conv_tuned_variant = _sig("hh_conv_tuned_variant", _I, _I, _I, _I, _I, _I, _I, _I)
hh_conv_force_variant = _sig("hh_conv_force_variant", _I, _I, _I, _I, _I)
hh_implicit_test = _sig("hh_implicit_test", _I, _P, _I, _I, _P, _P, _I)
hh_implicit_ggrad_test = _sig("hh_implicit_ggrad_test", _I, _P, _I, _I, _I, _P, _P, _P)
hh_pointwise_test = _sig("hh_pointwise_test", _I, _P, _I, _I, C.c_size_t, _P, _P, _P, _P, _I, _P, _P)
hh_depthwise_test = _sig("hh_depthwise_test", _I, _P, _I, _I, _I, _I, _P, _P, _P, _I, _I, _P, _P)
hh_wgrad_test = _sig("hh_wgrad_test", _I, _P, _I, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P)
hh_gen_training_pairs = _sig("hh_gen_training_pairs", _I, _P, _P, _I, _P, _IP, _P, _P)
hh_residual_norms = _sig("hh_residual_norms", _I, _P, _P, _I, _IP, _P, _P, _DP)
hh_residual_norms_noalloc = _sig("hh_residual_norms_noalloc", _I, _P, _P, _I, _IP, _P, _P, _DP)
hh_vcycle_tuned_height = _sig("hh_vcycle_tuned_height", _I, _I, _I, _I, _I, _I)
hh_vcycle_force_height = _sig("hh_vcycle_force_height", _I, _I, _I, _I)
hh_model_set_coarse_group = _sig("hh_model_set_coarse_group", _I, _P, _I)
hh_model_coarse_group = _sig("hh_model_coarse_group", _I, _P, _I)
hh_train_step = _sig("hh_train_step", _I, _P, _P, _P, _I, _P, _P, _D, _D, _DP, _DP)
hh_eval_loss = _sig("hh_eval_loss", _I, _P, _P, _P, _I, _P, _P, _DP)
hh_net_get_grads = _sig("hh_net_get_grads", _I, _P, _FP)
hh_profile_begin = _sig("hh_profile_begin", _I, _P, _I)
hh_profile_end = _sig("hh_profile_end", _I, _P, _DP, C.POINTER(C.c_longlong))
HH_K_NUM_CLASSES = 11

# kernel classes for hh_profile_begin
HH_K_OPERATOR, HH_K_VC_DOWN, HH_K_VC_UP, HH_K_VC_COARSE, HH_K_VC_MID, HH_K_OP_DOTS, HH_K_ORTHO, HH_K_SMALL, \
    HH_K_RESTART, HH_K_CONV, HH_K_NET_OTHER = range(11)
KERNEL_CLASS_NAMES = ["operator", "vc_down", "vc_up", "vc_coarse", "vc_mid", "op_dots", "ortho", "small",
                      "restart", "conv", "net_other"]


def check(status: int, allow=(HH_OK,)) -> int:
    if status in allow:
        return status
    raise HHError(status, (hh_last_error() or b"").decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous and on the GPU"
    return C.c_void_p(t.data_ptr())


def _int_array(vals):
    if vals is None:
        return None
    a = (C.c_int * len(vals))(*[int(v) for v in vals])
    return a


# ---------------------------------------------------------------------------
# torch-facing wrappers
# ---------------------------------------------------------------------------

class Context:
    """A libhh context on one device and torch's current stream; device memory
    comes from torch's caching allocator through the allocator callbacks."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        self.stream = stream or torch.cuda.current_stream(device)
        dev = device

        def _alloc(nbytes, user):
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        h = C.c_void_p()
        check(hh_ctx_create(device, C.c_void_p(self.stream.cuda_stream), self._alloc, self._free, None, C.byref(h)))
        self.handle = h
        # models and networks of this context: released before the context is
        self._children = weakref.WeakSet()

    def close(self):
        """Release the context, after every model and network still open on it
        (their workspaces go back through this context's allocator)."""
        if getattr(self, "handle", None):
            for c in list(getattr(self, "_children", ())):
                c.close()
            hh_ctx_destroy(self.handle)
            self.handle = None

    def profile_begin(self, cls: int = HH_K_NUM_CLASSES):
        check(hh_profile_begin(self.handle, cls))

    def profile_end(self):
        """{class name: (total kernel ms, timed launches)} since profile_begin."""
        ms = (C.c_double * HH_K_NUM_CLASSES)()
        cnt = (C.c_longlong * HH_K_NUM_CLASSES)()
        check(hh_profile_end(self.handle, ms, cnt))
        return {KERNEL_CLASS_NAMES[k]: (ms[k], cnt[k]) for k in range(HH_K_NUM_CLASSES) if cnt[k]}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def model_desc(n: int, omega: float, **kw) -> hh_model_desc:
    d = hh_model_desc()
    hh_model_desc_default(C.byref(d))
    d.n = n
    d.omega = omega
    for k, v in kw.items():
        setattr(d, k, v)
    return d


class Model:
    """Slowness model(s) on an n x n grid: kappa is a (ninst, n, n) or (n, n) tensor."""

    def __init__(self, ctx: Context, kappa: torch.Tensor, omega: float, **desc_kw):
        k = kappa.to(device=f"cuda:{ctx.device}", dtype=torch.float32).contiguous()
        if k.dim() == 2:
            k = k[None]
        self.ctx, self.n, self.ninst = ctx, k.shape[-1], k.shape[0]
        self.desc = model_desc(self.n, omega, **desc_kw)
        h = C.c_void_p()
        check(hh_model_create(ctx.handle, C.byref(self.desc), self.ninst, _ptr(k), C.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:  # a closed context has already released this model
                hh_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parity-test building blocks --------------------------------------
    def apply_operator(self, x: torch.Tensor, level: int = 0, shift: float = 0.0, inst=None) -> torch.Tensor:
        x = x.to(torch.complex64).contiguous()
        y = torch.empty_like(x)
        nrhs = x.shape[0]
        check(hh_apply_operator(self.handle, level, shift, nrhs, _int_array(inst), _ptr(x), _ptr(y)))
        return y

    def apply_vcycle(self, b: torch.Tensor, x0: torch.Tensor | None = None, inst=None) -> torch.Tensor:
        b = b.to(torch.complex64).contiguous()
        x0 = None if x0 is None else x0.to(torch.complex64).contiguous()
        x = torch.empty_like(b)
        check(hh_apply_vcycle(self.handle, b.shape[0], _int_array(inst), _ptr(b), _ptr(x0), _ptr(x)))
        return x

    def residual_norms(self, b: torch.Tensor, x: torch.Tensor, inst=None) -> np.ndarray:
        """||b - A x|| / ||b|| (FP64) of solutions x (complex128) for right-hand sides b."""
        b = b.to(torch.complex64).contiguous()
        x = x.to(torch.complex128).contiguous()
        out = np.zeros(b.shape[0])
        check(hh_residual_norms(self.ctx.handle, self.handle, b.shape[0], _int_array(inst), _ptr(b), _ptr(x),
                                out.ctypes.data_as(_DP)))
        return out

    def residual_norms_noalloc(self, b: torch.Tensor, x: torch.Tensor, inst=None) -> np.ndarray:
        """residual_norms through the entry point that allocates nothing (b complex64
        and x complex128, contiguous, as given: no conversion here either)."""
        assert b.dtype == torch.complex64 and x.dtype == torch.complex128
        assert b.is_contiguous() and x.is_contiguous()
        out = np.zeros(b.shape[0])
        check(hh_residual_norms_noalloc(self.ctx.handle, self.handle, b.shape[0], _int_array(inst), _ptr(b),
                                        _ptr(x), out.ctypes.data_as(_DP)))
        return out

    def set_coarse_group(self, R: int):
        """Fix the coarse solve's right-hand sides per workgroup (1, 2, 4, 8) or autotune (0)."""
        check(hh_model_set_coarse_group(self.handle, R))

    def coarse_group(self, nact: int) -> int:
        return hh_model_coarse_group(self.handle, nact)

    def attach_net(self, net: "Net | None"):
        check(hh_model_attach_net(self.handle, net.handle if net is not None else None))
        self.net = net

    def training_pairs(self, x: torch.Tensor, kiters):
        """(e, r) of eq. 20 for random vectors x (one per slowness model of the model)."""
        x = x.to(torch.complex64).contiguous()
        e = torch.empty_like(x)
        r = torch.empty_like(x)
        check(hh_gen_training_pairs(self.ctx.handle, self.handle, x.shape[0], _ptr(x), _int_array(kiters), _ptr(e),
                                    _ptr(r)))
        return e, r

    def apply_cnn_precond(self, v: torch.Tensor, inst=None) -> torch.Tensor:
        """z = V(v; Net(v)), one application of the CNN+MG preconditioner."""
        v = v.to(torch.complex64).contiguous()
        z = torch.empty_like(v)
        check(hh_apply_cnn_precond(self.handle, v.shape[0], _int_array(inst), _ptr(v), _ptr(z)))
        return z

    def net_forward(self, r: torch.Tensor, inst=None) -> torch.Tensor:
        r = r.to(torch.complex64).contiguous()
        e = torch.empty_like(r)
        check(hh_net_forward(self.handle, r.shape[0], _int_array(inst), _ptr(r), _ptr(e)))
        return e

    # -- solve --------------------------------------------------------------
    def solve(self, b: torch.Tensor, x0: torch.Tensor | None = None, inst=None, restart=10, max_iters=2000,
              rtol=1e-6, precond=HH_PRECOND_MG, warm_mg_iters=3, fixed_iters=0, want_hist=True, fallback=True,
              probe_ratio=0.5, graph=True):
        """Returns (x complex128 tensor, info dict with iters, converged, final_res, hist)."""
        b = b.to(torch.complex64).contiguous()
        nrhs = b.shape[0]
        if x0 is not None:
            x = x0.to(torch.complex128).contiguous().clone()
        else:
            x = torch.empty(b.shape, dtype=torch.complex128, device=b.device)
        o = hh_solve_opts()
        hh_solve_opts_default(C.byref(o))
        o.restart, o.max_iters, o.rtol, o.precond = restart, max_iters, rtol, precond
        o.warm_mg_iters, o.use_x0, o.fixed_iters = warm_mg_iters, int(x0 is not None), fixed_iters
        o.fallback, o.probe_ratio, o.graph = int(fallback), probe_ratio, int(graph)
        hl = (fixed_iters if fixed_iters > 0 else max_iters) + 1
        hist = np.zeros((nrhs, hl)) if want_hist else None
        iters = np.zeros(nrhs, dtype=np.int32)
        conv = np.zeros(nrhs, dtype=np.int32)
        fres = np.zeros(nrhs)
        mgc = np.zeros(nrhs, dtype=np.int32)
        cnnit = np.zeros(nrhs, dtype=np.int32)
        st = hh_solve(self.ctx.handle, self.handle, nrhs, _int_array(inst), _ptr(b), _ptr(x), C.byref(o),
                      hist.ctypes.data_as(_DP) if hist is not None else None, iters.ctypes.data_as(_IP),
                      conv.ctypes.data_as(_IP), fres.ctypes.data_as(_DP), mgc.ctypes.data_as(_IP),
                      cnnit.ctypes.data_as(_IP))
        check(st, allow=(HH_OK, HH_NOT_CONVERGED))
        return x, dict(iters=iters, converged=conv.astype(bool), final_res=fres, hist=hist, status=st,
                       mg_cycles=mgc, cnn_iters=cnnit)


def _ptr_array(ctype, items):
    arr = (ctype * len(items))(*items)
    return arr, C.cast(arr, C.c_void_p)


def solve_batch(ctx: Context, models, bs, insts=None, restart=10, max_iters=2000, rtol=1e-6, precond=HH_PRECOND_MG,
                warm_mg_iters=3, fallback=True, probe_ratio=0.5, graph=True):
    """Several models (any sizes) solved in one interleaved launch sequence
    (hh_solve_batch).  bs[i]: right-hand sides of models[i]; insts[i]: optional
    RHS -> instance map.  Returns [(x complex128 tensor, info dict)] per model."""
    nm = len(models)
    bs = [b.to(torch.complex64).contiguous() for b in bs]
    xs = [torch.empty(b.shape, dtype=torch.complex128, device=b.device) for b in bs]
    o = hh_solve_opts()
    hh_solve_opts_default(C.byref(o))
    o.restart, o.max_iters, o.rtol, o.precond = restart, max_iters, rtol, precond
    o.warm_mg_iters, o.fallback, o.probe_ratio, o.graph = warm_mg_iters, int(fallback), probe_ratio, int(graph)
    nr = [b.shape[0] for b in bs]
    out = {k: [np.zeros(n, dtype=np.int32) for n in nr] for k in ("iters", "converged", "mg_cycles", "cnn_iters")}
    fres = [np.zeros(n) for n in nr]
    inst_arrays = [_int_array(insts[i]) if insts is not None and insts[i] is not None else None for i in range(nm)]
    keep = []

    def ints(lst):
        a, p = _ptr_array(_IP, [x.ctypes.data_as(_IP) for x in lst])
        keep.append(a)
        return p

    ma, mp = _ptr_array(C.c_void_p, [m.handle for m in models])
    ia, ip = _ptr_array(_IP, [C.cast(a, _IP) if a is not None else None for a in inst_arrays])
    ba, bp = _ptr_array(C.c_void_p, [b.data_ptr() for b in bs])
    xa, xp = _ptr_array(C.c_void_p, [x.data_ptr() for x in xs])
    fa, fp = _ptr_array(_DP, [f.ctypes.data_as(_DP) for f in fres])
    st = hh_solve_batch(ctx.handle, nm, mp, (C.c_int * nm)(*nr), ip, bp, xp, C.byref(o), ints(out["iters"]),
                        ints(out["converged"]), fp, ints(out["mg_cycles"]), ints(out["cnn_iters"]))
    check(st, allow=(HH_OK, HH_NOT_CONVERGED))
    return [(xs[i], dict(iters=out["iters"][i], converged=out["converged"][i].astype(bool), final_res=fres[i],
                         status=st, mg_cycles=out["mg_cycles"][i], cnn_iters=out["cnn_iters"][i]))
            for i in range(nm)]


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

from .netfile import (NET_LAYER_NAMES, flatten_light_params, flatten_params, read_header, read_params,  # noqa: E402,F401
                      unflatten_light_params, unflatten_params)


class Net:
    """Encoder-solver network on the device (FP32 master parameters)."""

    def __init__(self, ctx: Context, params: dict | np.ndarray | None = None, ch=(16, 32, 64, 64), _handle=None,
                 explicit: bool = False, light: bool = False):
        """explicit: the coarsest level convolves with the learned kernels
        instead of applying their Green's functions; light: the lightweight
        network (inverted bottlenecks, batch normalisation, softplus)."""
        self.ctx = ctx
        self.ch = tuple(ch)
        self.explicit = bool(explicit)
        self.light = bool(light)
        if _handle is not None:
            self.handle = _handle
            ctx._children.add(self)
            return
        d = hh_net_desc()
        for i in range(4):
            d.ch[i] = ch[i]
        d.explicit_coarse = int(self.explicit)
        d.arch = HH_ARCH_LIGHT if self.light else HH_ARCH_UNET
        flat = None
        if params is not None:
            if isinstance(params, np.ndarray):
                flat = params
            else:
                flat = flatten_light_params(params, ch) if self.light else flatten_params(params, ch)
            flat = np.ascontiguousarray(flat, dtype=np.float32)
        h = C.c_void_p()
        check(hh_net_create(ctx.handle, C.byref(d), flat.ctypes.data_as(_FP) if flat is not None else None,
                            C.byref(h)))
        self.handle = h
        ctx._children.add(self)
        if flat is not None:
            assert flat.size == self.num_params(), (flat.size, self.num_params())

    @classmethod
    def load(cls, ctx: Context, path: str) -> "Net":
        h = C.c_void_p()
        check(hh_net_load(ctx.handle, path.encode(), C.byref(h)))
        hd = read_header(path)
        return cls(ctx, ch=hd["ch"], _handle=h, explicit=hd["explicit"], light=hd["light"])

    def save(self, path: str):
        check(hh_net_save(self.handle, path.encode()))

    def num_params(self) -> int:
        return int(hh_net_num_params(self.handle))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.num_params(), dtype=np.float32)
        check(hh_net_get_params(self.handle, a.ctypes.data_as(_FP)))
        return a

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.num_params()
        check(hh_net_set_params(self.handle, a.ctypes.data_as(_FP)))

    def get_grads(self) -> np.ndarray:
        a = np.zeros(self.num_params(), dtype=np.float32)
        check(hh_net_get_grads(self.handle, a.ctypes.data_as(_FP)))
        return a

    def unflatten(self, flat: np.ndarray) -> dict:
        """Named FP64 parameters (or gradients) of a flat vector of this network."""
        return unflatten_light_params(flat, self.ch) if self.light else unflatten_params(flat, self.ch)

    def train_step(self, model: "Model", r: torch.Tensor, e: torch.Tensor, lr: float,
                   max_grad_norm: float = 0.0) -> float:
        """One training step; returns the loss (the gradient norm is kept in last_grad_norm)."""
        r = r.to(torch.complex64).contiguous()
        e = e.to(torch.complex64).contiguous()
        loss, gnorm = C.c_double(), C.c_double()
        check(hh_train_step(self.ctx.handle, self.handle, model.handle, r.shape[0], _ptr(r), _ptr(e), lr,
                            max_grad_norm, C.byref(loss), C.byref(gnorm)))
        self.last_grad_norm = gnorm.value
        return loss.value

    def eval_loss(self, model: "Model", r: torch.Tensor, e: torch.Tensor) -> float:
        """Loss of hh_train_step without the backward pass or an update."""
        r = r.to(torch.complex64).contiguous()
        e = e.to(torch.complex64).contiguous()
        loss = C.c_double()
        check(hh_eval_loss(self.ctx.handle, self.handle, model.handle, r.shape[0], _ptr(r), _ptr(e), C.byref(loss)))
        return loss.value

    def implicit_test(self, x_bf16: torch.Tensor, nc: int, adjoint=False) -> torch.Tensor:
        y = torch.empty_like(x_bf16)
        check(hh_implicit_test(self.handle, nc, x_bf16.shape[0], _ptr(x_bf16), _ptr(y), int(adjoint)))
        return y

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:
                hh_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conv_variants(cin: int, cout: int, mode: int) -> list[int]:
    """Kernel variant codes of a convolution shape (the first is the untuned default)."""
    codes = (C.c_int * 16)()
    nv = hh_conv_variants(cin, cout, mode, codes, 16)
    return [int(codes[i]) for i in range(nv)]


def conv_tuned_variant(device: int, cin: int, cout: int, mode: int, Hout: int, Wout: int, B: int) -> int:
    """The autotuner's choice for a key (0: not tuned yet)."""
    return int(hh_conv_tuned_variant(device, cin, cout, mode, Hout, Wout, B))


def conv_force_variant(cin: int, cout: int, mode: int, code: int):
    """Use one variant for every launch of a shape (0: autotune again)."""
    check(hh_conv_force_variant(cin, cout, mode, code))


def conv_test(ctx: Context, x_bf16: torch.Tensor, w: torch.Tensor, mode: int, flipped: bool, bias=None, skip=None,
              relu=False, active=None, fill=None, act=None, variant: int = 0, fp32_out: bool = True):
    """One convolution through the library's MFMA kernel; returns (y bf16, y fp32),
    y fp32 None with fp32_out=False (the FP32 copy not written, as in the network).
    act: 0 none, 1 ReLU, 2 softplus (default: 1 if relu else 0); variant: a
    kernel variant code (0: the autotuned choice).
    active: optional per-batch-entry flags (0 = skipped, output left as filled);
    fill: initial value of both outputs (default: uninitialised)."""
    B, H, W_, cin = x_bf16.shape
    cout = w.shape[1] if flipped else w.shape[0]
    Ho = H // 2 if mode == 1 else (2 * H if mode == 2 else H)
    Wo = W_ // 2 if mode == 1 else (2 * W_ if mode == 2 else W_)
    y = torch.empty((B, Ho, Wo, cout), dtype=torch.bfloat16, device=x_bf16.device)
    yf = torch.empty((B, Ho, Wo, cout), dtype=torch.float32, device=x_bf16.device) if fp32_out else None
    if fill is not None:
        y.fill_(fill)
        if yf is not None:
            yf.fill_(fill)
    # keep every converted tensor referenced until the call returns: the library
    # allocates through torch's caching allocator and could otherwise reuse them
    w = w.to(torch.float32).contiguous()
    bias = bias.to(torch.float32).contiguous() if bias is not None else None
    skip = skip.contiguous() if skip is not None else None
    check(hh_conv_test(ctx.handle, cin, cout, mode, B, H, W_, _ptr(x_bf16), _ptr(w), int(flipped), _ptr(bias),
                       _ptr(skip), int(act if act is not None else (1 if relu else 0)), _ptr(y), _ptr(yf),
                       _int_array(active), int(variant)))
    return y, yf


def conv_pair_test(ctx: Context, x_bf16: torch.Tensor, w1: torch.Tensor, b1, w2: torch.Tensor, b2, active=None,
                   fill=None, variant: int = 0):
    """Two fused stride-1 16-channel ReLU layers (mode 3); returns (y, mid) BF16,
    mid written by the unfused variant 1 only.  fill: initial value of both."""
    B, H, W_, _ = x_bf16.shape
    y = torch.empty((B, H, W_, 16), dtype=torch.bfloat16, device=x_bf16.device)
    mid = torch.empty_like(y)
    if fill is not None:
        y.fill_(fill)
        mid.fill_(fill)
    x_bf16 = x_bf16.contiguous()
    w1, w2 = w1.to(torch.float32).contiguous(), w2.to(torch.float32).contiguous()
    b1 = b1.to(torch.float32).contiguous() if b1 is not None else None
    b2 = b2.to(torch.float32).contiguous() if b2 is not None else None
    check(hh_conv_pair_test(ctx.handle, B, H, W_, _ptr(x_bf16), _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2), _ptr(mid),
                            _ptr(y), _int_array(active), int(variant)))
    return y, mid


def wgrad_test(ctx: Context, a_bf16: torch.Tensor, x_bf16: torch.Tensor, mode: int) -> torch.Tensor:
    """Weight-gradient kernel: (ca, cx, 3, 3) FP32 sums of a (x) shifted x over pixels."""
    B, Ho, Wo, ca = a_bf16.shape
    _, Hi, Wi, cx = x_bf16.shape
    a_bf16, x_bf16 = a_bf16.contiguous(), x_bf16.contiguous()
    out = torch.empty((ca, cx, 3, 3), dtype=torch.float32, device=a_bf16.device)
    check(hh_wgrad_test(ctx.handle, ca, cx, mode, B, Ho, Wo, Hi, Wi, _ptr(a_bf16), _ptr(x_bf16), _ptr(out)))
    return out


def pointwise_test(ctx: Context, x_bf16: torch.Tensor, w: torch.Tensor, bias=None, res=None, act: int = 0):
    """The lightweight network's 1x1 convolution: x [..., cin] BF16, w (cout, cin); returns (y bf16, y fp32)."""
    cin = x_bf16.shape[-1]
    cout = w.shape[0]
    npix = x_bf16.numel() // cin
    y = torch.empty(x_bf16.shape[:-1] + (cout,), dtype=torch.bfloat16, device=x_bf16.device)
    yf = torch.empty(y.shape, dtype=torch.float32, device=x_bf16.device)
    w = w.to(torch.float32).contiguous()
    bias = bias.to(torch.float32).contiguous() if bias is not None else None
    res = res.contiguous() if res is not None else None
    x_bf16 = x_bf16.contiguous()
    check(hh_pointwise_test(ctx.handle, cin, cout, npix, _ptr(x_bf16), _ptr(w), _ptr(bias), _ptr(res), int(act),
                            _ptr(y), _ptr(yf)))
    return y, yf


def depthwise_test(ctx: Context, x_bf16: torch.Tensor, w: torch.Tensor, bias=None, act: int = 0, flip=False):
    """The lightweight network's depthwise 3x3 convolution: x [B][H][W][C] BF16, w (C, 3, 3)."""
    B, H, W_, Cc = x_bf16.shape
    y = torch.empty_like(x_bf16)
    yf = torch.empty(x_bf16.shape, dtype=torch.float32, device=x_bf16.device)
    w = w.to(torch.float32).contiguous()
    bias = bias.to(torch.float32).contiguous() if bias is not None else None
    x_bf16 = x_bf16.contiguous()
    check(hh_depthwise_test(ctx.handle, Cc, B, H, W_, _ptr(x_bf16), _ptr(w), _ptr(bias), int(act), int(flip),
                            _ptr(y), _ptr(yf)))
    return y, yf


def implicit_ggrad_test(ctx: Context, z_bf16: torch.Tensor, gy_bf16: torch.Tensor) -> torch.Tensor:
    """Gradient of the implicit layer's transformed Green's functions for BF16
    NHWC z, gy [B][nc][nc][2 nk]: complex128 [nk][2nc][2nc]."""
    B, nc, _, ch = z_bf16.shape
    out = torch.empty((ch // 2, 2 * nc, 2 * nc), dtype=torch.complex128, device=z_bf16.device)
    z_bf16, gy_bf16 = z_bf16.contiguous(), gy_bf16.contiguous()
    check(hh_implicit_ggrad_test(ctx.handle, ch // 2, nc, B, _ptr(z_bf16), _ptr(gy_bf16), _ptr(out)))
    return out


def vcycle_tuned_height(device: int, kernel: int, mode: int, n: int, nrhs: int) -> int:
    """The V-cycle tile height the autotuner chose for a key (0: not tuned yet)."""
    return int(hh_vcycle_tuned_height(device, kernel, mode, n, nrhs))


def vcycle_force_height(kernel: int, mode: int, height: int):
    """Use one tile height for a V-cycle kernel and mode (0: autotune again)."""
    check(hh_vcycle_force_height(kernel, mode, height))
