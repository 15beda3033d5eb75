"""The residual-norm entry point that allocates nothing (its partial sums in
the library's fixed per-GPU scratch array) against hh_residual_norms, through
the C ABI: two calls in a row, the second on a smaller input, so the second
reuses the scratch the first one left behind."""
import sys

import numpy as np
import pytest
import torch

from paper_2306_17486_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(hh, ctx, n, ninst, nrhs, seed):
    ks = np.stack([inputs.slowness(n, seed + i, "grf" if i % 2 == 0 else "layered") for i in range(ninst)])
    m = hh.Model(ctx, torch.from_numpy(ks), inputs.omega_for(n))
    b = torch.from_numpy(inputs.random_complex((nrhs, n, n), seed + 10)).to("cuda:0", torch.complex64)
    # solutions that leave residuals of very different sizes per right-hand side
    x = torch.from_numpy(inputs.random_complex((nrhs, n, n), seed + 11) * 1e-3
                         * np.logspace(-3, 0, nrhs)[:, None, None]).to("cuda:0", torch.complex128)
    inst = [r % ninst for r in range(nrhs)] if ninst > 1 else None
    return m, b, x, inst


def test_residual_norms_noalloc_matches():
    from paper_2306_17486_amd import hh
    ctx = hh.Context(0)
    for n, ninst, nrhs, seed in ((256, 3, 7, 500), (128, 1, 2, 600)):  # the second call is smaller
        _say(f"no-alloc residual norms: n={n} media={ninst} nrhs={nrhs}")
        m, b, x, inst = _case(hh, ctx, n, ninst, nrhs, seed)
        ref = m.residual_norms(b, x, inst=inst)
        got = m.residual_norms_noalloc(b, x, inst=inst)
        _say(f"  ref {ref}\n  got {got}")
        # FP64 sums in a different order: agreement to a few FP64 roundings
        assert np.all(np.abs(got - ref) <= 1e-12 * ref), np.abs(got - ref) / ref
        m.close()
    ctx.close()


def test_residual_norms_noalloc_rejects_beyond_its_limits():
    from paper_2306_17486_amd import hh
    ctx = hh.Context(0)
    m, b, x, _ = _case(hh, ctx, 64, 1, 1, 700)
    big = torch.zeros((257, 64, 64), dtype=torch.complex64, device="cuda:0")
    bigx = torch.zeros((257, 64, 64), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(hh.HHError) as e:
        m.residual_norms_noalloc(big, bigx)
    assert e.value.status == hh.HH_ERR_ARG
    m.close()
    ctx.close()
