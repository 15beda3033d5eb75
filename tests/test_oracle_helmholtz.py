"""Pins of the FP64 oracle's operator, transfers, V-cycle and FGMRES against
facts the paper and the mathematics fix (not against the oracle itself)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import helmholtz as H
from paper_2306_17486_amd import inputs


def _problem(n, seed=7, omega_scale=1.0, family="grf", gamma0=0.0):
    k = inputs.slowness(n, seed, family)
    return H.Problem(k, inputs.omega_for(n, k) * omega_scale, gamma0=gamma0)


# --- absorbing layer (Sec. 3.1) --------------------------------------------

def test_abl_profile_endpoints():
    g = H.abl_gamma(64, width=16, gamma_max=1.0)
    assert g[0, 32] == 1.0 and g[32, 0] == 1.0 and g[63, 40] == 1.0
    assert g[16, 32] == 0.0 and g[32, 32] == 0.0
    # quadratic ramp: d = 8 -> ((16-8)/16)^2 = 1/4
    assert g[8, 32] == pytest.approx(0.25)
    # symmetric under flips
    assert np.array_equal(g, g[::-1, :]) and np.array_equal(g, g.T)


# --- operator (eqs. 1-3) ----------------------------------------------------

def test_matrix_free_equals_assembled():
    P = _problem(24)
    u = inputs.random_complex((24, 24), 1)
    for shift in (0.0, 0.5):
        A = P.matrix(shift)
        y1 = (A @ u.ravel()).reshape(24, 24)
        y2 = H.apply_op(u, P.k2w2, P.gamma, P.h, shift)
        assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(y1).max()


def test_stencil_entries_brute_force():
    # eq. 3 written out entry by entry for one interior and one corner cell
    n = 8
    P = _problem(n, omega_scale=0.5)
    A = P.matrix().toarray()
    h = P.h
    i, j = 2, 3
    r = i * n + j
    m = P.k2w2[i, j] * (1 - 1j * P.gamma[i, j])
    assert A[r, r] == pytest.approx(4 / h ** 2 - m)
    for q in ((i - 1) * n + j, (i + 1) * n + j, i * n + j - 1, i * n + j + 1):
        assert A[r, q] == pytest.approx(-1 / h ** 2)
    assert np.count_nonzero(A[r]) == 5
    assert np.count_nonzero(A[0]) == 3  # corner: two ghosts are zero (Dirichlet)


def test_complex_symmetric_not_hermitian():
    P = _problem(20)
    A = P.matrix()
    assert abs(A - A.T).max() == 0.0
    assert abs(A - A.conj().T).max() > 0.0
    x = inputs.random_complex((20, 20), 2)
    y = inputs.random_complex((20, 20), 3)
    lhs = np.sum(y * P.A(x))
    rhs = np.sum(x * P.A(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_frequency_closed_form_spectrum():
    # omega = 0: A is the zero-ghost Laplacian; its eigenpairs are known in closed form.
    n = 16
    h = 1.0 / n
    z = np.zeros((n, n))
    idx = np.arange(n)
    for p, q in ((1, 1), (3, 5), (n, n - 2)):
        v = np.outer(np.sin(p * math.pi * (idx + 1) / (n + 1)), np.sin(q * math.pi * (idx + 1) / (n + 1)))
        lam = 4 / h ** 2 * (math.sin(p * math.pi / (2 * (n + 1))) ** 2 + math.sin(q * math.pi / (2 * (n + 1))) ** 2)
        Av = H.apply_op(v.astype(complex), z, z, h)
        assert np.abs(Av - lam * v).max() <= 1e-9 * lam


# --- transfers (eq. 8) ------------------------------------------------------

def test_prolongation_is_bilinear_interpolation():
    c = inputs.random_complex((6, 6), 4)
    f = H.prolong(c)
    cp = np.zeros((7, 7), dtype=complex)
    cp[:6, :6] = c  # zero ghost beyond the high edge
    for I in range(6):
        for J in range(6):
            assert f[2 * I, 2 * J] == pytest.approx(c[I, J])
            assert f[2 * I + 1, 2 * J] == pytest.approx((cp[I, J] + cp[I + 1, J]) / 2)
            assert f[2 * I, 2 * J + 1] == pytest.approx((cp[I, J] + cp[I, J + 1]) / 2)
            assert f[2 * I + 1, 2 * J + 1] == pytest.approx(
                (cp[I, J] + cp[I + 1, J] + cp[I, J + 1] + cp[I + 1, J + 1]) / 4)


def test_restriction_weights_and_adjointness():
    f = np.zeros((8, 8))
    f[4, 6] = 1.0  # fine 2I = 4, 2J = 6 -> coarse (2, 3) gets 4/16
    R = H.restrict_fw(f)
    assert R[2, 3] == pytest.approx(0.25) and R.sum() == pytest.approx(0.25)
    f[:] = 0
    f[5, 6] = 1.0  # odd row: shared by coarse rows 2 and 3 with weight 2/16
    R = H.restrict_fw(f)
    assert R[2, 3] == pytest.approx(0.125) and R[3, 3] == pytest.approx(0.125)
    # constants are preserved away from the edges
    Rc = H.restrict_fw(np.ones((16, 16)))
    assert np.allclose(Rc[1:, 1:], 1.0)
    # P = 4 R^T (dot-product test)
    c = inputs.random_complex((8, 8), 5)
    g = inputs.random_complex((16, 16), 6)
    assert np.vdot(H.prolong(c), g) == pytest.approx(4 * np.vdot(c, H.restrict_fw(g)))


def test_coefficient_restriction_keeps_constants_at_edges():
    c = np.full((16, 16), 0.7)
    assert np.allclose(H.restrict_coeff(c), 0.7)


def test_coefficient_restriction_hand_computed():
    # reading C5: full weighting (1/16)[1 2 1; 2 4 2; 1 2 1] centred on fine
    # (2I, 2J), the field padded by replicating its edge cells.  On c = 4i + j
    # (4 x 4) the edge rows/columns carry weights 3/4 (edge) and 1/4 (next):
    #   out[0,0] = (9 c00 + 3 c01 + 3 c10 + c11) / 16 = (0 + 3 + 12 + 5) / 16
    #   out[0,1] = 3/4 (c01/4 + c02/2 + c03/4) + 1/4 (c11/4 + c12/2 + c13/4) = 3/4 * 2 + 1/4 * 6
    #   out[1,0] = 3/4 (c10/4 + c20/2 + c30/4) + 1/4 (c11/4 + c21/2 + c31/4) = 3/4 * 8 + 1/4 * 9
    #   out[1,1] = interior weights on a linear field: c22 = 10
    c = np.array([[4.0 * i + j for j in range(4)] for i in range(4)])
    assert np.allclose(H.restrict_coeff(c), [[1.25, 3.0], [8.25, 10.0]], rtol=0, atol=1e-15)
    # injection would give [[0, 2], [8, 10]], zero padding 15/16 at (0, 0)
    # interior weights on a quadratic: (1/4)(2I-1)^2 + (1/2)(2I)^2 + (1/4)(2I+1)^2 = 4 I^2 + 1/2
    q = np.array([[float(i * i) for j in range(8)] for i in range(8)])
    out = H.restrict_coeff(q)
    assert np.allclose(out[1:, :], np.array([4.0 * I * I + 0.5 for I in range(1, 4)])[:, None], rtol=0, atol=1e-13)


# --- relaxation -------------------------------------------------------------

def test_jacobi_matches_assembled_diagonal():
    P = _problem(16)
    A = P.matrix(H.SL_BETA).toarray()
    d = np.diag(A).reshape(16, 16)
    x = inputs.random_complex((16, 16), 8)
    b = inputs.random_complex((16, 16), 9)
    ref = x + 0.8 * (b - (A @ x.ravel()).reshape(16, 16)) / d
    assert np.abs(P.hier.jacobi(0, x, b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_jacobi_smoothing_factor_closed_form():
    # damped Jacobi symbol 1 - w (1 - (cos t1 + cos t2)/2); max over high frequencies
    w = 0.8
    t = np.linspace(-math.pi, math.pi, 257)
    T1, T2 = np.meshgrid(t, t)
    high = (np.abs(T1) >= math.pi / 2) | (np.abs(T2) >= math.pi / 2)
    s = np.abs(1 - w * (1 - (np.cos(T1) + np.cos(T2)) / 2))
    assert s[high].max() == pytest.approx(max(abs(1 - 2 * w), abs(1 - w / 2)), abs=1e-12)


def _lfa_two_grid(w=0.8, nu1=1, nu2=1, m=64):
    """Two-grid local Fourier analysis for the 5-point Laplacian (h = 1):
    damped Jacobi, full weighting, bilinear interpolation, rediscretised 2h operator."""
    rho = 0.0
    for t1 in (np.arange(m) + 0.5) / m * math.pi - math.pi / 2:
        for t2 in (np.arange(m) + 0.5) / m * math.pi - math.pi / 2:
            harm = [(t1, t2), (t1 + math.pi, t2), (t1, t2 + math.pi), (t1 + math.pi, t2 + math.pi)]
            Ah = np.array([4 - 2 * math.cos(a) - 2 * math.cos(b) for a, b in harm])
            S = np.diag(1 - w * Ah / 4)
            Rr = np.array([(1 + math.cos(a)) * (1 + math.cos(b)) / 4 for a, b in harm])
            AH = (4 - 2 * math.cos(2 * t1) - 2 * math.cos(2 * t2)) / 4
            K = np.eye(4) - np.outer(Rr, Rr) * Ah[None, :] / AH
            M = np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)
            rho = max(rho, max(abs(np.linalg.eigvals(M))))
    return rho


def test_vcycle_contraction_matches_two_grid_lfa():
    """omega = 0 Laplacian.  With n even, coarse cell I sits on fine cell 2I, so the
    coarse Dirichlet ghost of the low edge lands one fine cell beyond the fine
    ghost.  A huge mass on fine row/column 0 moves the low-edge boundary onto fine
    index 0, which makes fine and coarse boundaries coincide; the same oracle code
    must then contract at the textbook two-grid LFA rate."""
    lfa = _lfa_two_grid()
    assert 0.3 < lfa < 0.4
    n = 64
    k2w2 = np.zeros((n, n))
    k2w2[0, :] = -1e12
    k2w2[:, 0] = -1e12
    g = np.zeros((n, n))
    for levels in (2, 3):
        hier = H.Hierarchy(k2w2, g, levels)
        rng = np.random.default_rng(0)
        e = rng.standard_normal((n, n)) + 0j
        e[0, :] = 0
        e[:, 0] = 0
        for _ in range(40):
            e_new = e - hier.vcycle(H.apply_op(e, k2w2, g, 1.0 / n, 0.0))
            ratio = np.linalg.norm(e_new) / np.linalg.norm(e)
            e = e_new / np.linalg.norm(e_new)
        assert abs(ratio - lfa) < 0.03, (levels, ratio, lfa)


def test_vcycle_is_a_stable_preconditioner_with_even_grid_alignment():
    """Without the boundary shift (the alignment the solver uses), the omega = 0
    V-cycle is not a convergent stationary iteration on its own (the low-edge
    mode), but all the other modes still contract; FGMRES absorbs the rest."""
    n = 32
    P = H.Problem(np.ones((n, n)), 0.0)
    N = n * n
    E = np.zeros((N, N), dtype=complex)
    for c in range(N):
        e = np.zeros(N, dtype=complex)
        e[c] = 1.0
        e = e.reshape(n, n)
        E[:, c] = (e - P.mg(P.A(e))).ravel()
    ev = np.sort(np.abs(np.linalg.eigvals(E)))[::-1]
    assert ev[0] > 1.0          # the one low-edge mode
    assert ev[8] < 0.45         # everything but a handful of edge modes contracts


def test_low_edge_mode_costs_a_few_fgmres_iterations():
    """What the even-grid alignment's low-edge mode costs: MG-preconditioned
    FGMRES(10) to 1e-8 on the omega = 0 problem at 64^2 against the same solve
    with the low-edge boundary moved onto fine index 0 (fine and coarse
    boundaries coincide, the V-cycle contracts at the two-grid LFA rate).
    Measured: 16 against 11 iterations; the Helmholtz solves need hundreds."""
    n = 64
    P = H.Problem(np.ones((n, n)), 0.0)
    b = inputs.random_complex((n, n), 3)
    _, its_even, _, rel = H.fgmres(P.A, b, P.mg, rtol=1e-8, max_iters=200)
    assert rel <= 1e-8
    k2w2 = np.zeros((n, n))
    k2w2[0, :] = -1e12
    k2w2[:, 0] = -1e12
    g = np.zeros((n, n))
    hier = H.Hierarchy(k2w2, g, 3)
    b2 = b.copy()
    b2[0, :] = 0
    b2[:, 0] = 0
    _, its_shift, _, rel2 = H.fgmres(lambda e: H.apply_op(e, k2w2, g, 1.0 / n, 0.0), b2, hier.vcycle, rtol=1e-8,
                                     max_iters=200)
    assert rel2 <= 1e-8
    assert its_shift <= 12 and its_even <= its_shift + 6, (its_even, its_shift)


# --- FGMRES -----------------------------------------------------------------

def test_fgmres_identity_preconditioner_matches_library_gmres():
    n = 32
    P = _problem(n, seed=5, omega_scale=0.3)
    b = inputs.random_complex((n, n), 1)
    res = []
    spla.gmres(P.matrix(), b.ravel(), restart=10, rtol=1e-8, atol=0, maxiter=6,
               callback=lambda r: res.append(r), callback_type="pr_norm")
    _, its, hist, _ = H.fgmres(P.A, b, lambda v: v, rtol=1e-8, max_iters=60)
    m = min(len(res), len(hist) - 1)
    assert m >= 50
    assert np.abs(np.array(res[:m]) - np.array(hist[1:m + 1])).max() <= 1e-10


def test_fgmres_exact_preconditioner_one_iteration():
    n = 24
    P = _problem(n)
    lu = spla.splu(P.matrix().tocsc())
    b = inputs.random_complex((n, n), 2)
    x, its, hist, rel = H.fgmres(P.A, b, lambda v: lu.solve(v.ravel()).reshape(n, n), rtol=1e-10)
    assert its == 1 and rel <= 1e-10


def test_fgmres_mg_matches_sparse_direct():
    n = 64
    P = _problem(n, seed=11)
    b = inputs.point_source(n, 3)
    xs = H.exact_solve(P, b)
    x, its, hist, rel = H.fgmres(P.A, b, P.mg, rtol=1e-12, max_iters=800)
    assert rel <= 1e-12
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    # the residual estimate is monotone within a cycle and ends at the true value's scale
    assert hist[-1] <= 1e-12


def test_manufactured_solution():
    n = 64
    P = _problem(n, seed=12, family="layered")
    idx = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(idx, idx, indexing="ij")
    win = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.02)
    u = win * np.exp(1j * P.omega * 0.6 * (0.8 * X + 0.6 * Y))
    b = P.A(u)
    xs = H.exact_solve(P, b)
    assert np.linalg.norm(xs - u) <= 1e-11 * np.linalg.norm(u)
    x, its, hist, rel = H.solve_mg(P, b, rtol=1e-9)
    assert rel <= 1e-9 and np.linalg.norm(x - u) <= 1e-6 * np.linalg.norm(u)


def test_mg_only_iterations_config1_magnitude():
    # 128^2 GRF model, one point source: the paper reports about 100-170 iterations
    # for its (inexact-coarse) V-cycle at 128^2; the exact coarse solve needs fewer.
    n = 128
    k = inputs.grf_slowness(n, 1000)
    P = H.Problem(k, inputs.omega_for(n, k))
    b = inputs.point_source(n, 3000)
    x, its, hist, rel = H.solve_mg(P, b)
    assert rel <= 1e-6
    assert 30 <= its <= 170
    xs = H.exact_solve(P, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-4


# ---- iterative coarsest-grid solve (GMRES with a Jacobi preconditioner, Sec. 3.4) ----

def _coarse_level(n, seed):
    k = inputs.grf_slowness(n, seed)
    prob = H.Problem(k, inputs.omega_for(n, k), coarse_iters=1)
    return prob.hier.levels[-1]


def test_coarse_gmres_jacobi_is_the_minimal_residual_krylov_iterate():
    # GMRES's defining property, by brute force: with M = diag(A_SL)^-1 on the
    # right, x_k = M y with y in span{b, (A M) b, ..., (A M)^(k-1) b} minimising
    # ||b - A M y||.  A left-preconditioned or unpreconditioned variant, a wrong
    # diagonal or a dropped Givens step gives a different iterate.
    lev = _coarse_level(32, 11)  # coarsest 8 x 8
    b = inputs.random_complex((lev.n, lev.n), 12)
    A = H.assemble(lev.k2w2, lev.gamma, lev.h, H.SL_BETA).toarray()
    dinv = 1.0 / lev.diag(H.SL_BETA).ravel()
    AM = A * dinv[None, :]
    for k in (1, 3, 6):
        K = np.empty((b.size, k), dtype=np.complex128)
        K[:, 0] = b.ravel()
        for j in range(1, k):
            K[:, j] = AM @ K[:, j - 1]
        Q, _ = np.linalg.qr(K)
        c = np.linalg.lstsq(AM @ Q, b.ravel(), rcond=None)[0]
        x_bf = (dinv * (Q @ c)).reshape(b.shape)
        x = H.gmres_jacobi(lev, b, k)
        assert np.linalg.norm(x - x_bf) / np.linalg.norm(x_bf) <= 1e-9
        # and it is not the unpreconditioned Krylov iterate
        c0 = np.linalg.lstsq(A @ Q, b.ravel(), rcond=None)[0]
        if k > 1:
            assert np.linalg.norm(x - (Q @ c0).reshape(b.shape)) / np.linalg.norm(x_bf) > 1e-3


def test_coarse_gmres_jacobi_at_full_dimension_is_the_direct_solve():
    lev = _coarse_level(16, 13)  # coarsest 4 x 4: 16 unknowns
    b = inputs.random_complex((lev.n, lev.n), 14)
    A = H.assemble(lev.k2w2, lev.gamma, lev.h, H.SL_BETA).tocsc()
    x_ref = spla.spsolve(A, b.ravel()).reshape(b.shape)
    x = H.gmres_jacobi(lev, b, 16)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-8
    assert np.array_equal(H.gmres_jacobi(lev, np.zeros_like(b), 5), np.zeros_like(b))


def test_vcycle_with_iterative_coarse_solve():
    n = 16
    k = inputs.layered_slowness(n, 15)
    om = inputs.omega_for(n, k)
    direct = H.Problem(k, om)
    it_full = H.Problem(k, om, coarse_iters=16)
    it_few = H.Problem(k, om, coarse_iters=2)
    b = inputs.random_complex((n, n), 16)
    zd = direct.mg(b)
    assert np.linalg.norm(it_full.mg(b) - zd) / np.linalg.norm(zd) <= 1e-8
    assert np.linalg.norm(it_few.mg(b) - zd) / np.linalg.norm(zd) > 1e-4


def test_out_of_distribution_media_generators():
    # inputs only: seeded, FP32-representable, normalised like the paper's
    # out-of-distribution media (largest slowness 1), values inside [0.25, 1]
    for name, f in inputs.OOD_FAMILIES.items():
        a, b = f(128, 11), f(128, 11)
        assert np.array_equal(a, b), name
        assert a.max() == 1.0 and a.min() >= 0.25, name
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64)), name
        assert len(np.unique(a)) >= 5, name
