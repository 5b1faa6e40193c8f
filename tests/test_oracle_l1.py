"""Pins of the oracle's l1 metric nearness mode: (mn1) with real
dissimilarities d (Sec. II-A: min sum w |x - d| over metric x), solved as
(qp) by Algorithm 1 exactly as correlation clustering, whose d is 0/1.
CPU only; the dense checkers in oracle_helpers share no code with the
oracle."""
import numpy as np
import pytest

import oracle
from oracle_helpers import dense_problem, lp_optimum, qp_bruteforce
from paper_1901_10084_amd import instances as I


def l1_state(inst, gamma):
    return oracle.L1Nearness(inst.n, gamma, inst.w, inst.dv)


def test_zero_one_d_is_correlation_clustering():
    """With d in {0, 1} the l1 problem is the correlation-clustering LP."""
    inst = I.workload(0)
    a = oracle.State.from_instance(inst)
    b = oracle.L1Nearness(inst.n, inst.gamma, inst.w, inst.d.astype(np.float64))
    a.sweep(7, b=8)
    b.sweep(7, b=8)
    for k in ("x", "f", "y", "y_pair"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    ra, rb = a.residuals(), b.residuals()
    assert all(ra[k] == rb[k] for k in ra)


@pytest.mark.parametrize("n,seed,gamma", [(4, 0, 1.0), (5, 1, 2.0), (6, 2, 0.8), (7, 3, 3.0)])
def test_bruteforce_qp_with_real_d(n, seed, gamma):
    """The limit equals an independent dense QP solution for real d, and the
    oracle's own (x, f, y) satisfies KKT."""
    inst = I.noisy_distances(n, seed=seed, noise=0.7)
    s = l1_state(inst, gamma)
    r = s.solve(tol=1e-13, b=3, max_sweeps=400000)
    v = qp_bruteforce(n, inst.w, inst.dv, gamma)
    npairs = len(inst.w)
    np.testing.assert_allclose(s.x, v[:npairs], atol=1e-9)
    np.testing.assert_allclose(s.f, v[npairs:], atol=1e-9)
    A, b, c, W = dense_problem(n, inst.w, inst.dv)
    yall = np.concatenate([s.y, s.y_pair])
    vv = np.concatenate([s.x, s.f])
    assert (A @ vv - b).max() < 1e-12
    assert np.abs(c + W * vv / gamma + A.T @ yall).max() < 1e-9
    assert yall.min() >= 0
    assert abs(r["gap"]) < 1e-9 * max(1.0, abs(r["primal_qp"]))


@pytest.mark.parametrize("seed", [0, 1])
def test_large_gamma_solves_the_l1_lp(seed):
    """For gamma large enough the (qp) point solves the LP (mn1) (Sec. II-B):
    its l1 cost sum w |x - d| equals the HiGHS optimum (here at gamma = 1000;
    at gamma = 200 it is still 1e-4 above, and never below it)."""
    inst = I.noisy_distances(7, seed=seed, noise=0.8)
    lp = lp_optimum(inst.n, inst.w, inst.dv)
    s = l1_state(inst, 200.0)
    r = s.solve(tol=1e-12, b=4, max_sweeps=2000000)
    assert r["lp_cost"] >= lp - 1e-9
    s = l1_state(inst, 1000.0)
    r = s.solve(tol=1e-12, b=4, max_sweeps=2000000)
    assert abs(r["lp_cost"] - lp) <= 1e-9 * max(1.0, lp)


def test_a_metric_is_the_solution_when_gamma_exceeds_it():
    """Exact Euclidean distances are already metric; with gamma above every
    d the regularised optimum is x = d, f = 0 (moving x toward 0 from d
    gains (1/gamma) d'Wd and costs w'd per unit, a net loss)."""
    inst = I.noisy_distances(9, seed=4, noise=0.0)
    s = l1_state(inst, 2.0 * float(inst.dv.max()) + 1.0)
    s.solve(tol=1e-12, b=4, max_sweeps=200000)
    np.testing.assert_allclose(s.x, inst.dv, atol=1e-9)
    np.testing.assert_allclose(s.f, 0.0, atol=1e-9)


def test_invariants_every_sweep():
    """Dual coordinate ascent: y >= 0, stationarity x = x(y), D(y) never
    falls."""
    inst = I.noisy_distances(11, seed=2, noise=0.6)
    s = l1_state(inst, 1.5)
    prev = -np.inf
    for _ in range(25):
        s.sweep(1, b=4)
        r = s.residuals()
        assert s.y.min() >= 0 and s.y_pair.min() >= 0
        assert r["stat_resid"] < 1e-12
        assert r["dual_qp"] >= prev - 1e-12 * max(1.0, abs(prev))
        prev = r["dual_qp"]
