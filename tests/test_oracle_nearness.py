"""Pins of the oracle's l2 metric nearness mode (Sec. II-A, the metric
nearness problem with p = 2, solved by Algorithm 1 from x = d): closed forms,
an independent dense solver on tiny instances, invariants of dual coordinate
ascent, and order independence of the limit."""
import numpy as np
import pytest

import oracle
from oracle_helpers import dense_metric_rows, halfspace_projection, nearness_bruteforce
from paper_1901_10084_amd import instances as I


def test_single_violated_triangle_is_the_weighted_projection():
    """n = 3 with one violated row: the optimum is the W-norm projection of d
    onto that row's halfspace (the other two rows stay satisfied)."""
    w = np.array([0.7, 1.3, 2.1])
    dv = np.array([3.0, 1.0, 1.2])          # pairs (0,1), (0,2), (1,2): x01 <= x02 + x12 fails
    s = oracle.Nearness(3, w, dv)
    s.sweep(3, b=1)
    a = np.array([1.0, -1.0, -1.0])
    np.testing.assert_allclose(s.x, halfspace_projection(dv, a, 0.0, w), rtol=0, atol=1e-14)
    r = s.residuals()
    assert r["max_viol"] <= 1e-15 and abs(r["gap"]) < 1e-14


def test_unit_weight_step_moves_delta_over_three():
    """With W = I the first visit moves the three distances by delta/3."""
    dv = np.array([3.0, 1.0, 1.0])
    s = oracle.Nearness(3, np.ones(3), dv)
    s.sweep(1, b=1)
    np.testing.assert_allclose(s.x, [3 - 1 / 3, 1 + 1 / 3, 1 + 1 / 3], rtol=0, atol=1e-15)
    assert s.y[0] == pytest.approx(1 / 3, abs=1e-15) and s.y[1] == 0.0 and s.y[2] == 0.0


def test_a_metric_is_a_fixed_point():
    """Exact Euclidean distances satisfy every row: x stays d bit for bit and
    every dual stays 0."""
    inst = I.noisy_distances(12, seed=3, noise=0.0)
    s = oracle.Nearness(inst.n, inst.w, inst.dv)
    s.sweep(2, b=4)
    assert np.array_equal(s.x, inst.dv) and not s.y.any()


@pytest.mark.parametrize("n,seed,weighted", [(4, 0, False), (5, 1, True), (6, 2, True),
                                             (7, 3, False)])
def test_bruteforce(n, seed, weighted):
    """The limit equals an independent dense QP solution; the oracle's own
    (x, y) satisfies KKT: feasibility, stationarity W(x - d) + A'y = 0,
    y >= 0, complementary slackness, zero gap."""
    inst = I.noisy_distances(n, seed=seed, noise=0.6, weighted=weighted)
    s = oracle.Nearness(inst.n, inst.w, inst.dv)
    r = s.solve(tol=1e-14, b=3, max_sweeps=200000, gap_tol=1e-14)
    np.testing.assert_allclose(s.x, nearness_bruteforce(n, inst.w, inst.dv), atol=1e-9)
    A = dense_metric_rows(n)
    assert (A @ s.x).max() < 1e-12
    assert np.abs(inst.w * (s.x - inst.dv) + A.T @ s.y).max() < 1e-12
    assert s.y.min() >= 0
    assert np.abs(s.y * (A @ s.x)).max() < 1e-12
    assert abs(r["gap"]) < 1e-10 * max(1.0, abs(r["primal"]))


def test_invariants_every_sweep():
    """Dual coordinate ascent: y >= 0, x = d - W^{-1} A'y, D(y) never falls,
    and never passes the optimum (weak duality)."""
    inst = I.noisy_distances(15, seed=5, noise=0.8)
    s = oracle.Nearness(inst.n, inst.w, inst.dv)
    last = s.residuals()["dual"]
    assert last == 0.0
    duals = []
    for _ in range(10):
        s.sweep(1, b=4)
        r = s.residuals()
        assert s.y.min() >= 0
        assert r["stat_resid"] < 1e-12
        assert r["dual"] >= last - 1e-12 * max(1.0, abs(last))
        duals.append(r["dual"])
        last = r["dual"]
    opt = s.solve(tol=1e-13, b=4, max_sweeps=200000, gap_tol=1e-13)["primal"]
    assert max(duals) <= opt + 1e-12 * max(1.0, opt)


def test_order_does_not_change_the_limit():
    """The optimum is unique: the schedule at several tile sizes and plain
    lexicographic order reach the same x."""
    inst = I.noisy_distances(11, seed=7, noise=0.7)
    xs = []
    for b, order in ((1, "schedule"), (3, "schedule"), (8, "schedule"), (8, "lex")):
        s = oracle.Nearness(inst.n, inst.w, inst.dv)
        s.solve(tol=1e-13, b=b, max_sweeps=200000, order=order, gap_tol=1e-13)
        xs.append(s.x.copy())
    for x in xs[1:]:
        np.testing.assert_allclose(x, xs[0], atol=1e-10)


# Hand-worked nearness point (every value an exact binary fraction):
# w = (1, 2, 4), d = (3, 1, 3/2), dual 1/2 on o = 0 (x_01 <= x_02 + x_12,
# a = (1, -1, -1)).  A'y = (1/2, -1/2, -1/2), so x(y) = d - W^{-1} A'y =
# (5/2, 5/4, 13/8).  Metric slacks there: o=0: 3/8, o=1: 23/8, o=2: 17/8.
# D = d'A'y - (1/2) sum (A'y)^2 / w = 1/4 - 7/32 = 1/32;
# primal (1/2) sum w (x - d)^2 = 7/32; gap 3/16.
def _near_state():
    s = oracle.Nearness(3, np.array([1.0, 2.0, 4.0]), np.array([3.0, 1.0, 1.5]))
    s.y[:] = [0.5, 0.0, 0.0]
    s.x[:] = [2.5, 1.25, 1.625]
    return s


def test_residuals_at_hand_point():
    r = _near_state().residuals()
    assert r["stat_resid"] == 0.0
    assert r["dual"] == 1 / 32 and r["primal"] == 7 / 32 and r["gap"] == 3 / 16
    assert r["cs_max"] == 0.5 * 3 / 8
    assert r["max_viol"] == 0.0


@pytest.mark.parametrize("o,slack", [(0, 0.375), (1, 2.875), (2, 2.125)])
def test_complementary_slackness_one_row(o, slack):
    s = _near_state()
    s.y[:] = 0.0
    s.y[o] = 2.0
    assert s.residuals()["cs_max"] == 2.0 * slack


@pytest.mark.parametrize("var,delta", [(0, 0.25), (1, -0.125), (2, 0.5)])
def test_stationarity_residual_is_the_perturbation(var, delta):
    s = _near_state()
    s.x[var] += delta
    assert s.residuals()["stat_resid"] == abs(delta)
