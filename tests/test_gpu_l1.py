"""l1 metric nearness on the GPU ((mn1) with real d) against the oracle's
l1 mode, through the C ABI."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from paper_1901_10084_amd import instances as I

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C


def rel_err(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(a - ref).max() / max(1.0, float(np.abs(ref).max())))


TOL64 = 1e-10


def pair(n, gamma, b, prec="f64", seed=None, noise=0.6):
    inst = I.noisy_distances(n, seed=n if seed is None else seed, noise=noise)
    g = C.L1Solver(inst.n, inst.w, inst.dv, gamma, b=b, prec=prec)
    o = oracle.L1Nearness(inst.n, gamma, inst.w, inst.dv)
    return inst, g, o


@pytest.mark.parametrize("n,b,K", [(3, 8, 2), (17, 8, 3), (40, 16, 3), (33, 16, 4), (70, 32, 2),
                                   (29, 5, 3)])
def test_l1_sweeps_match_the_oracle(n, b, K):
    """b = 5 runs on the round executor, the others on the dataflow one."""
    print(f"l1 n={n} b={b} K={K}", flush=True)
    inst, g, o = pair(n, 2.0, b)
    g.sweep(K)
    o.sweep(K, b=b)
    g.status()
    assert rel_err(g.x.cpu().numpy(), o.x) <= TOL64
    assert rel_err(g.f.cpu().numpy(), o.f) <= TOL64
    assert rel_err(g.duals_lex().cpu().numpy(), o.y) <= TOL64
    assert rel_err(g.y_pair.cpu().numpy(), o.y_pair) <= TOL64


def test_zero_one_d_reproduces_correlation_clustering():
    inst = I.workload(0)
    cc = C.Solver.from_instance(inst, b=8, prec="f64")
    l1 = C.L1Solver(inst.n, inst.w, inst.d.astype(np.float64), inst.gamma, b=8, prec="f64")
    cc.sweep(5)
    l1.sweep(5)
    for a in ("x", "f", "y", "y_pair"):
        assert torch.equal(getattr(cc, a), getattr(l1, a)), a


@pytest.mark.parametrize("n,b,prec", [(100, 16, "f64"), (130, 32, "f32")])
def test_l1_sparse_equals_dense(n, b, prec):
    inst, d, _ = pair(n, 3.0, b, prec)
    s = C.L1Solver(inst.n, inst.w, inst.dv, 3.0, b=b, prec=prec)
    d.sweep(4)
    s.sweep(4, sparse=True)
    s.status()
    for a in ("x", "f", "y", "y_pair"):
        assert torch.equal(getattr(d, a), getattr(s, a)), a


def test_l1_residuals_match_the_oracle():
    inst, g, o = pair(45, 1.5, 16)
    g.sweep(6)
    o.sweep(6, b=16)
    rg, ro = g.residuals(), o.residuals()
    for k in ("max_viol_metric", "max_viol_pair", "primal_qp", "dual_qp", "lp_cost", "cs_max"):
        assert abs(rg[k] - ro[k]) <= 1e-9 * max(1.0, abs(ro[k])), (k, rg[k], ro[k])
    assert rg["stat_resid"] < 1e-12


def test_l1_solve_reaches_the_oracle_optimum_and_the_lp():
    """Solved to 1e-10 the GPU point is the oracle's, in its sweep count (the QP optimum is
    unique); at gamma = 1000 its l1 cost is the oracle's LP-exact cost."""
    inst, g, o = pair(25, 1.0, 8, seed=9)
    r, ok, _ = g.solve(tol=1e-10, max_sweeps=20000)
    o.solve(tol=1e-10, b=8, max_sweeps=20000)
    assert ok and g.sweeps == o.sweeps
    assert rel_err(g.x.cpu().numpy(), o.x) <= 1e-8
    inst, g, o = pair(7, 1000.0, 8, seed=0, noise=0.8)
    r, ok, _ = g.solve(tol=1e-12, max_sweeps=2000000, check_every=50)
    ro = o.solve(tol=1e-12, b=8, max_sweeps=2000000)
    assert ok and abs(r["lp_cost"] - ro["lp_cost"]) <= 1e-9 * max(1.0, ro["lp_cost"])
