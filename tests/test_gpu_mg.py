"""GPU parity of the operator, the V-cycle and MG-only FGMRES against the FP64 oracle.

Called through the C ABI (ctypes binding).  Sizes span several tiles and a
ragged tail (n = 100 is not a multiple of the 64 x 16 tiles)."""
import sys

import numpy as np
import pytest
import torch

from oracle import helmholtz as H
from paper_2306_17486_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hh():
    from paper_2306_17486_amd import hh as _hh
    return _hh


@pytest.fixture(scope="module")
def ctx(hh):
    return hh.Context(0)


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _dev(a, dtype=torch.complex64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


@pytest.mark.parametrize("n,family", [(128, "grf"), (100, "layered")])
def test_operator_all_levels(hh, ctx, n, family):
    _say(f"operator parity n={n} {family}")
    k = inputs.slowness(n, 11, family)
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    m = hh.Model(ctx, torch.from_numpy(k), om)
    for lvl, L in enumerate(prob.hier.levels):
        x = inputs.random_complex((2, L.n, L.n), 20 + lvl)
        for shift in (0.0, 0.5):
            y = m.apply_operator(_dev(x), level=lvl, shift=shift).cpu().numpy()
            ref = np.stack([H.apply_op(x[i], L.k2w2, L.gamma, L.h, shift) for i in range(2)])
            assert _rel(y, ref) <= 2e-6, (lvl, shift, _rel(y, ref))
            # elementwise, so that one wrong edge row or absorbing-layer band cannot
            # hide in the global norm
            emax = float(np.abs(y - ref).max() / np.abs(ref).max())
            _say(f"  level {lvl} shift {shift}: global {_rel(y, ref):.2e}, elementwise {emax:.2e}")
            assert emax <= 2e-5, (lvl, shift, emax)


def test_operator_complex_symmetry(hh, ctx):
    n = 96
    _say("operator bilinear symmetry")
    k = inputs.grf_slowness(n, 3)
    m = hh.Model(ctx, torch.from_numpy(k), inputs.omega_for(n, k))
    x = inputs.random_complex((1, n, n), 1)
    y = inputs.random_complex((1, n, n), 2)
    Ax = m.apply_operator(_dev(x)).cpu().numpy().astype(np.complex128)
    Ay = m.apply_operator(_dev(y)).cpu().numpy().astype(np.complex128)
    lhs, rhs = np.sum(y * Ax), np.sum(x * Ay)
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


@pytest.mark.parametrize("n,family,with_x0,reduce", [(128, "grf", False, 1), (100, "layered", False, 1),
                                                     (128, "layered", True, 1), (100, "grf", True, 1),
                                                     (100, "layered", False, 0), (128, "grf", True, 0),
                                                     (128, "grf", True, 2), (100, "layered", False, 2),
                                                     (116, "grf", False, 2), (128, "layered", False, 3),
                                                     (116, "grf", True, 3), (100, "grf", False, 4),
                                                     (128, "grf", False, 4), (200, "grf", False, 1),
                                                     (232, "layered", True, 4), (128, "grf", False, 5),
                                                     (232, "layered", True, 5), (512, "grf", True, 5),
                                                     (400, "layered", False, 4), (400, "grf", True, 0)])
def test_vcycle_parity(hh, ctx, n, family, with_x0, reduce):
    _say(f"vcycle parity n={n} {family} x0={with_x0} reduced coarse factorisation {reduce}")
    k = inputs.slowness(n, 12, family)
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    m = hh.Model(ctx, torch.from_numpy(k), om, coarse_reduce=reduce)
    b = inputs.random_complex((3, n, n), 5)
    x0 = inputs.random_complex((3, n, n), 6) * 1e-4 if with_x0 else None
    z = m.apply_vcycle(_dev(b), None if x0 is None else _dev(x0)).cpu().numpy()
    ref = np.stack([prob.hier.vcycle(b[i], None if x0 is None else x0[i]) for i in range(3)])
    assert _rel(z, ref) <= 2e-5, _rel(z, ref)
    emax = float(np.abs(z - ref).max() / np.abs(ref).max())
    _say(f"  global {_rel(z, ref):.2e}, elementwise {emax:.2e}")
    assert emax <= 2e-4, emax


@pytest.mark.parametrize("n,reduce", [(64, 4), (200, 4), (200, 1), (232, 0)])
def test_vcycle_multi_instance(hh, ctx, n, reduce):
    # two media in one model: each medium's coarse factors (tile-parallel
    # factorisation over both media at once; at 200^2 and 232^2 the coarsest
    # grid spans two 32-wide tiles, the second ragged) against its own oracle
    _say(f"vcycle two slowness models at n={n}, reduced coarse factorisation {reduce}")
    ks = [inputs.grf_slowness(n, 1), inputs.layered_slowness(n, 2)]
    om = inputs.omega_for(n)
    m = hh.Model(ctx, torch.from_numpy(np.stack(ks)), om, coarse_reduce=reduce)
    b = inputs.random_complex((4, n, n), 7)
    inst = [1, 0, 0, 1]
    z = m.apply_vcycle(_dev(b), inst=inst).cpu().numpy()
    probs = [H.Problem(k, om) for k in ks]
    for r in range(4):
        ref = probs[inst[r]].hier.vcycle(b[r])
        assert _rel(z[r], ref) <= 2e-5
        assert float(np.abs(z[r] - ref).max() / np.abs(ref).max()) <= 2e-4


def test_fgmres_mg_config1(hh, ctx):
    """128^2 GRF (seed 1000), one unit point source (seed 3000), FGMRES(10) + SL V-cycle,
    rtol 1e-6: iteration count within 2 of the oracle, solution within 1e-5 of the
    exact discrete solution, FP64 residual <= 1e-6 recomputed here."""
    n = 128
    _say("fgmres config 1")
    k = inputs.grf_slowness(n, 1000)
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    b = inputs.point_source(n, 3000)
    xo, its_o, _, _ = H.solve_mg(prob, b)
    xs = H.exact_solve(prob, b)
    m = hh.Model(ctx, torch.from_numpy(k), om)
    x, info = m.solve(_dev(b[None]))
    x = x.cpu().numpy()[0]
    _say("gpu iters", info["iters"][0], "oracle", its_o, "final", info["final_res"][0])
    assert info["converged"][0]
    assert abs(int(info["iters"][0]) - its_o) <= 2
    assert np.linalg.norm(b - prob.A(x)) / np.linalg.norm(b) <= 1e-6
    assert _rel(x, xs) <= 1e-5
    h = info["hist"][0]
    assert h[0] == pytest.approx(1.0) and h[info["iters"][0] + 1:].max() == -1.0


def test_fgmres_batch_instances_and_edge_cases(hh, ctx):
    n = 64
    _say("fgmres batch with two models, a zero rhs and an iteration cap")
    ks = [inputs.grf_slowness(n, 4), inputs.layered_slowness(n, 5)]
    om = inputs.omega_for(n)
    m = hh.Model(ctx, torch.from_numpy(np.stack(ks)), om)
    b = np.stack([inputs.point_source(n, 30), inputs.point_source(n, 31), np.zeros((n, n)),
                  inputs.random_complex((n, n), 32)])
    inst = [0, 1, 0, 1]
    x, info = m.solve(_dev(b), inst=inst)
    x = x.cpu().numpy()
    for r in (0, 1, 3):
        prob = H.Problem(ks[inst[r]], om)
        assert info["converged"][r]
        assert np.linalg.norm(b[r] - prob.A(x[r])) / np.linalg.norm(b[r]) <= 1e-6
        _, its_o, _, _ = H.solve_mg(prob, b[r])
        assert abs(int(info["iters"][r]) - its_o) <= 2
    assert info["converged"][2] and info["iters"][2] == 0 and np.abs(x[2]).max() == 0.0
    # iteration cap
    x, info = m.solve(_dev(b[:2]), inst=inst[:2], max_iters=5)
    assert info["status"] == hh.HH_NOT_CONVERGED
    assert list(info["iters"]) == [5, 5] and not info["converged"].any()


def test_fgmres_fixed_iterations_match_oracle(hh, ctx):
    """fixed_iters = k reproduces eq. 20's x~ (k MG-preconditioned iterations from 0)."""
    n = 64
    _say("fgmres fixed iterations")
    k = inputs.layered_slowness(n, 8)
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om, gamma0=0.05)
    m = hh.Model(ctx, torch.from_numpy(k), om, gamma0=0.05)
    xr = inputs.random_complex((n, n), 9)
    b = prob.A(xr)
    for kk in (2, 5, 8):
        xo, _, _, _ = H.fgmres(prob.A, b, prob.mg, None, 10, 0.0, kk)
        x, info = m.solve(_dev(b[None]), fixed_iters=kk)
        assert info["iters"][0] == kk
        assert _rel(x.cpu().numpy()[0], xo) <= 1e-4


def test_bad_arguments_raise(hh, ctx):
    with pytest.raises(hh.HHError):
        hh.Model(ctx, torch.ones(30, 30), 10.0)  # 30 not divisible by 4
    k = torch.from_numpy(inputs.grf_slowness(32, 1))
    m = hh.Model(ctx, k, 20.0)
    with pytest.raises(hh.HHError):
        m.solve(_dev(np.zeros((1, 32, 32))), restart=40)
    with pytest.raises(hh.HHError):
        m.solve(_dev(np.zeros((1, 32, 32))), precond=hh.HH_PRECOND_CNN_MG)


# (reduced factorisation?, variant): plain factorisation -- chain R, split 100 RS + R
# (RS rows of each Schur inverse per workgroup); reduced factorisation (one level of
# cyclic reduction) -- 1000 + R, and with split chains 10000 + 100 RS + R
COARSE_VARIANTS = [(0, 1), (0, 2), (0, 4), (0, 8), (0, 801), (0, 808), (0, 1601), (0, 1604), (0, 3202), (0, 3208),
                   (1, 1001), (1, 1002), (1, 1004), (1, 1008), (1, 10801), (1, 10808), (1, 11602), (1, 13201),
                   (1, 13208), (2, 1001), (2, 1002), (2, 1004), (2, 1008), (2, 10801), (2, 10808), (2, 11602),
                   (2, 13201), (2, 13208), (3, 1001), (3, 1004), (3, 1008), (3, 10808), (3, 13201), (4, 1002),
                   (4, 1008), (4, 11602), (5, 1001), (5, 13201)]


@pytest.mark.parametrize("reduce,R", COARSE_VARIANTS)
def test_coarse_group_sizes_vcycle_parity(hh, ctx, reduce, R):
    # 11 right-hand sides: full groups and a ragged last group for every R; one
    # and two slowness models (grouping order padded per model); coarse grids of
    # 32 and 16 points (split slices with and without empty rows)
    n = 128
    _say(f"coarse solve variant {R} (reduced factorisation {reduce})")
    k = inputs.slowness(n, 13, "layered")
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    m = hh.Model(ctx, torch.from_numpy(k), om, coarse_reduce=reduce)
    m.set_coarse_group(R)
    assert m.coarse_group(11) == R
    b = inputs.random_complex((11, n, n), 17)
    z = m.apply_vcycle(_dev(b)).cpu().numpy()
    ref = np.stack([prob.hier.vcycle(b[i]) for i in range(11)])
    assert _rel(z, ref) <= 2e-5, _rel(z, ref)
    ks = [inputs.grf_slowness(64, 1), inputs.layered_slowness(64, 2)]
    m2 = hh.Model(ctx, torch.from_numpy(np.stack(ks)), inputs.omega_for(64), coarse_reduce=reduce)
    m2.set_coarse_group(R)
    inst = [1, 0, 0, 1, 1, 0, 1]
    b2 = inputs.random_complex((7, 64, 64), 18)
    z2 = m2.apply_vcycle(_dev(b2), inst=inst).cpu().numpy()
    for r in range(7):
        assert _rel(z2[r], H.Problem(ks[inst[r]], inputs.omega_for(64)).hier.vcycle(b2[r])) <= 2e-5


@pytest.mark.parametrize("reduce,R", [(1, 1001), (1, 1002), (1, 1004), (2, 1001), (2, 1002), (2, 1004),
                                     (2, 1008), (2, 13201), (3, 1001), (3, 1002), (3, 13201), (4, 1001),
                                     (5, 1001), (5, 1004), (5, 13201)])
def test_coarse_prefetching_chains_vcycle_parity(hh, ctx, reduce, R):
    # a 128 x 128 coarsest grid: the chains with R <= 4 prefetch each step's factor
    # during the previous step (whole chunk pairs of columns per thread)
    n = 512
    _say(f"coarse solve variant {R} (reduced factorisation {reduce}) at n={n}")
    k = inputs.slowness(n, 14, "grf")
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    m = hh.Model(ctx, torch.from_numpy(k), om, coarse_reduce=reduce)
    m.set_coarse_group(R)
    b = inputs.random_complex((5, n, n), 19)
    z = m.apply_vcycle(_dev(b)).cpu().numpy()
    ref = np.stack([prob.hier.vcycle(b[i]) for i in range(5)])
    assert _rel(z, ref) <= 2e-5, _rel(z, ref)


def test_coarse_autotuner_and_compaction_in_solves(hh, ctx):
    # right-hand sides that converge at different iterations leave ragged active
    # sets: the packed coarse solve must still give every RHS the oracle's count.
    # RHS 2 finishes a restart cycle before the others: its returned solution must
    # not change after its convergence test (regression: finished RHS once took
    # their last correction again in every later cycle)
    n = 64
    _say("coarse autotuner and active packing")
    k = inputs.grf_slowness(n, 40)
    om = inputs.omega_for(n, k)
    prob = H.Problem(k, om)
    b = np.stack([inputs.point_source(n, 60 + i) for i in range(6)] + [inputs.random_complex((n, n), 66)])
    its_o = [H.solve_mg(prob, b[r])[1] for r in range(7)]
    bad = []
    for reduce, R in ((1, 0), (1, 1001), (1, 1008), (1, 11601), (0, 0), (0, 1), (0, 802), (0, 1608), (2, 0),
                      (2, 1002), (2, 13201), (3, 0), (3, 1001), (4, 0), (5, 0), (5, 1002)):
        m = hh.Model(ctx, torch.from_numpy(k), om, coarse_reduce=reduce)
        m.set_coarse_group(R)
        xd, info = m.solve(_dev(b))
        lib = m.residual_norms(_dev(b), xd)
        x = xd.cpu().numpy()
        for r in range(7):
            res = np.linalg.norm(b[r] - prob.A(x[r])) / np.linalg.norm(b[r])
            # the library applies A with FP32 coefficients: on these solutions that
            # operator differs from the FP64 one by about 4e-8 of ||b||
            assert abs(lib[r] - res) <= 1e-7
            assert abs(info["final_res"][r] - res) <= 1e-7
            _say(f"  reduce={reduce} R={R} rhs {r}: iters {info['iters'][r]} (oracle {its_o[r]}) gpu residual "
                 f"{info['final_res'][r]:.3e} host residual {res:.3e}")
            if not (info["converged"][r] and res <= 1e-6 and abs(int(info["iters"][r]) - its_o[r]) <= 2):
                bad.append((reduce, R, r))
        if R == 0:
            split = tuple(100 * rs + r for rs in (8, 16, 32) for r in (1, 2, 4, 8))
            assert m.coarse_group(7) in ((1001, 1002, 1004, 1008) + tuple(10000 + c for c in split) if reduce else
                                         (1, 2, 4, 8, 801, 802, 804, 808, 1601, 1602, 1604, 1608, 3201, 3202, 3204,
                                          3208))
    assert not bad, bad


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_vcycle_tile_heights_bit_identical(hh, ctx, mode):
    # every tile height the V-cycle autotuner can pick computes each point the
    # same way: bit-identical outputs (ragged size 100: partial tiles), and the
    # default against the oracle
    n = 100 if mode != 2 else 128
    heights = {0: ([4, 8, 16], [8, 16, 32]), 1: ([4, 8], [8, 16, 32]), 2: ([2, 4, 8], [4, 8, 16])}[mode]
    _say(f"vcycle tile heights, mode {mode}: down {heights[0]}, up {heights[1]}")
    k = inputs.slowness(n, 13, "layered")
    om = inputs.omega_for(n, k)
    m = hh.Model(ctx, torch.from_numpy(k), om)
    b = _dev(inputs.random_complex((3, n, n), 8))
    net = None
    if mode == 2:
        net = hh.Net(ctx, inputs.init_net_params(21))
        m.attach_net(net)
        run = lambda: m.apply_cnn_precond(b)  # noqa: E731
    else:
        x0 = _dev(inputs.random_complex((3, n, n), 9) * 1e-4) if mode == 1 else None
        run = lambda: m.apply_vcycle(b, x0)  # noqa: E731
    ref = run()
    try:
        for hd in heights[0]:
            for hu in heights[1]:
                hh.vcycle_force_height(0, mode, hd)
                hh.vcycle_force_height(1, mode, hu)
                assert torch.equal(run(), ref), (hd, hu)
    finally:
        hh.vcycle_force_height(0, mode, 0)
        hh.vcycle_force_height(1, mode, 0)
    with pytest.raises(hh.HHError):
        hh.vcycle_force_height(0, mode, 3)
    # the first launch of each key was tuned
    assert hh.vcycle_tuned_height(0, 0, mode, n, 3) in heights[0]
    assert hh.vcycle_tuned_height(0, 1, mode, n, 3) in heights[1]
    if mode == 0:
        prob = H.Problem(k, om)
        bb = b.cpu().numpy()
        refo = np.stack([prob.hier.vcycle(bb[i]) for i in range(3)])
        assert _rel(ref.cpu().numpy(), refo) <= 2e-5
    if net is not None:
        m.attach_net(None)
        net.close()
    m.close()
