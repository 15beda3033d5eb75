"""The C-ABI library loads without a GPU and exports every function include/hh.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hh.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(hh_[a-z0-9_]+)\s*\(", txt)
    # typedef'd callback types are not functions
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_header_declares_core_entry_points():
    d = _declared()
    for n in ("hh_ctx_create", "hh_model_create", "hh_solve", "hh_apply_operator", "hh_apply_vcycle"):
        assert n in d


def test_library_exports_every_declared_symbol():
    from paper_2306_17486_amd import hh
    missing = [n for n in _declared() if not hasattr(hh._lib, n)]
    assert not missing, missing
    assert b"gfx950" in hh.hh_version()


def test_binding_names_match_the_header():
    from paper_2306_17486_amd import hh
    for n in _declared():
        assert hasattr(hh, n), n


def test_defaults_without_gpu():
    from paper_2306_17486_amd import hh
    import ctypes as C
    d = hh.hh_model_desc()
    hh.hh_model_desc_default(C.byref(d))
    assert (d.abl_width, d.levels, d.nu_pre, d.nu_post) == (16, 3, 1, 1)
    assert d.sl_beta == 0.5 and d.jacobi_w == 0.8 and d.abl_gamma_max == 1.0 and d.coarse_reduce == 4
    assert d.coarse_iters == 0
    o = hh.hh_solve_opts()
    hh.hh_solve_opts_default(C.byref(o))
    assert (o.restart, o.max_iters, o.warm_mg_iters) == (10, 2000, 3) and o.rtol == 1e-6
    assert o.fallback == 1 and o.probe_ratio == 0.5 and o.graph == 1


def test_argument_errors_are_reported_without_gpu():
    from paper_2306_17486_amd import hh
    import ctypes as C
    st = hh.hh_model_create(None, None, 1, None, None)
    assert st == hh.HH_ERR_ARG
    assert b"null pointer" in hh.hh_last_error()
    o = hh.hh_solve_opts()
    hh.hh_solve_opts_default(C.byref(o))
    assert hh.hh_solve_batch(None, 1, None, None, None, None, None, C.byref(o), None, None, None, None,
                             None) == hh.HH_ERR_ARG


def test_parameter_vector_round_trip_and_size():
    import numpy as np
    from paper_2306_17486_amd import inputs, netfile
    p = inputs.init_net_params(3)
    flat = netfile.flatten_params(p)
    assert flat.dtype == np.float32 and flat.size == 509522
    q = netfile.unflatten_params(flat)
    assert set(q) == set(p)
    for k in p:
        assert np.allclose(q[k], np.asarray(p[k]).astype(np.complex64 if np.iscomplexobj(p[k]) else np.float32))


def test_shipped_network_file_reads_without_gpu():
    import numpy as np
    from paper_2306_17486_amd import netfile
    path = os.path.join(ROOT, "paper_2306_17486_amd", "weights", "net_ms128_256_512.bin")
    flat, ch = netfile.read_params(path)
    assert ch == (16, 32, 64, 64) and flat.size == 509522
    assert np.isfinite(flat).all()
