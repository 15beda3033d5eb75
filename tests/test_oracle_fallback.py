"""The oracle's two-phase solve with the CNN+MG and MG-only preconditioners
judging each other (restart-cycle probes), pinned by three cases whose outcome
follows from the method itself:

* an exact network (the direct solve) makes CNN+MG a strong preconditioner
  (the V-cycle that follows relaxes on the shifted operator, so it is not
  exact): every CNN+MG cycle cuts the residual far below the probe ratio, the
  judge never probes and the solve needs a fraction of MG-only's iterations;
* a network that returns large noise cannot reduce the residual (FGMRES picks
  the best combination, so the cycle stalls): the judge probes once, MG-only
  wins and keeps every later cycle (its cycles reduce the residual far below
  the probe ratio on this small grid), so the solve costs at most about one
  wasted cycle more than MG-only;
* without the judge the same noisy network needs far more iterations."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import helmholtz as H
from oracle import solver as S
from paper_2306_17486_amd import inputs

N = 64


def _problem():
    k = inputs.grf_slowness(N, 5)
    return H.Problem(k, inputs.omega_for(N, k))


class _Exact:
    def __init__(self, prob):
        self.lu = spla.splu(prob.matrix(0.0).tocsc())

    def __call__(self, r):
        return self.lu.solve(r.ravel()).reshape(r.shape)


class _Noise:
    def __init__(self, seed):
        self.rng = np.random.default_rng(seed)

    def __call__(self, r):
        return 1e3 * np.abs(r).max() * (self.rng.standard_normal(r.shape) + 1j * self.rng.standard_normal(r.shape))


def test_exact_network_never_probes():
    prob = _problem()
    b = inputs.point_source(N, 3)
    _, its_mg, _, _ = H.solve_mg(prob, b)
    st = {}
    x, its, _, rel = S.solve_two_phase(prob, _Exact(prob), b, stats=st)
    assert rel <= 1e-6 and its < its_mg / 2
    assert st == {"probes": 0, "mg_cycles": 0}
    assert np.linalg.norm(b - prob.A(x)) / np.linalg.norm(b) <= 1e-6


def test_noisy_network_falls_back_to_mg_after_one_probe():
    prob = _problem()
    b = inputs.point_source(N, 4)
    _, its_mg, _, rel_mg = H.solve_mg(prob, b)
    st = {}
    _, its, _, rel = S.solve_two_phase(prob, _Noise(1), b, stats=st)
    assert rel <= 1e-6 and rel_mg <= 1e-6
    assert st["probes"] == 1 and st["mg_cycles"] >= 1
    assert st["mg_cycles"] == -(-(its - 3 - 10) // 10)  # every cycle after the stalled one
    # 3 warm + one stalled CNN+MG cycle, then MG-only from (about) where it was
    assert its <= its_mg + 2 * 10


def test_without_the_judge_the_noisy_network_costs_far_more():
    prob = _problem()
    b = inputs.point_source(N, 4)
    _, its_fb, _, _ = S.solve_two_phase(prob, _Noise(1), b)
    _, its_no, _, _ = S.solve_two_phase(prob, _Noise(1), b, fallback=False, max_iters=4 * its_fb)
    assert its_no >= 2 * its_fb


class _NaNAfter:
    """A network whose output turns non-finite from its k-th application on."""

    def __init__(self, k):
        self.k, self.calls = k, 0

    def __call__(self, r):
        self.calls += 1
        return np.full(r.shape, np.nan + 0j) if self.calls >= self.k else np.zeros_like(r)


def test_non_finite_network_output_falls_back_to_mg_from_the_last_finite_iterate():
    # the failure rule: the cycle with the non-finite application is dropped
    # (its applications still count), x keeps the cycle's starting value and
    # MG-only continues.  With a network that fails at once that is: 3 warm
    # MG-only iterations, one wasted application, then MG-only FGMRES(10) from
    # the warm iterate, counted on from 4.
    prob = _problem()
    b = inputs.point_source(N, 6)
    st = {}
    x, its, hist, rel = S.solve_two_phase(prob, _NaNAfter(1), b, stats=st)
    xw, _, _, _ = H.fgmres(prob.A, b, prob.mg, None, 10, 1e-6, 3)
    xe, its_e, _, rel_e = H.fgmres(prob.A, b, prob.mg, xw, 10, 1e-6, 2000, iters_done=4)
    assert rel <= 1e-6 and np.all(np.isfinite(x))
    assert its == its_e and np.array_equal(x, xe) and rel == rel_e
    assert st["mg_cycles"] == -(-(its - 4) // 10) and st["probes"] == 0
    # a network failing within a cycle: that cycle's earlier applications count too
    st2 = {}
    x2, its2, _, rel2 = S.solve_two_phase(prob, _NaNAfter(4), b, stats=st2)
    xe2, its_e2, _, _ = H.fgmres(prob.A, b, prob.mg, xw, 10, 1e-6, 2000, iters_done=3 + 4)
    assert its2 == its_e2 and np.array_equal(x2, xe2) and rel2 <= 1e-6
