"""l2 metric nearness on the GPU against the oracle's nearness mode, through
the C ABI: the same metric sweep kernels, started at x = d with g = 1/w."""
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
    return float(np.abs(a - ref).max() / max(1.0, float(np.abs(ref).max())))


TOL64 = 1e-10   # FP64 GPU vs FP64 oracle, relative to max(1, |ref|_inf)


@pytest.mark.parametrize("n,b,K", [(3, 8, 2), (17, 8, 3), (40, 16, 3), (33, 16, 4), (70, 32, 2),
                                   (65, 32, 3)])
def test_sweeps_match_oracle(n, b, K):
    inst = I.noisy_distances(n, seed=n, noise=0.6)
    print(f"nearness n={n} b={b} K={K}", flush=True)
    g = C.NearnessSolver.from_instance(inst, b=b, prec="f64")
    o = oracle.Nearness(inst.n, inst.w, inst.dv)
    g.sweep(K)
    o.sweep(K, b=b)
    g.status()
    assert rel_err(g.x.cpu().numpy(), o.x) <= TOL64
    assert rel_err(g.duals_lex().cpu().numpy(), o.y) <= TOL64


def test_f32_close_to_oracle():
    """FP32 sweeps stay within single-precision drift of the FP64 oracle."""
    inst = I.noisy_distances(40, seed=11, noise=0.6)
    g = C.NearnessSolver.from_instance(inst, b=16, prec="f32")
    o = oracle.Nearness(inst.n, inst.w, inst.dv)
    g.sweep(5)
    o.sweep(5, b=16)
    assert rel_err(g.x.cpu().numpy(), o.x) <= 1e-5


@pytest.mark.parametrize("n,b,prec", [(60, 8, "f64"), (100, 16, "f64"), (130, 32, "f32")])
def test_dataflow_equals_rounds(n, b, prec):
    inst = I.noisy_distances(n, seed=3, noise=0.7)
    r = C.NearnessSolver.from_instance(inst, b=b, prec=prec)
    d = C.NearnessSolver.from_instance(inst, b=b, prec=prec)
    r.sweep(3, C.CC_EXEC_ROUNDS)
    d.sweep(3, C.CC_EXEC_DATAFLOW)
    d.status()
    assert torch.equal(r.x, d.x) and torch.equal(r.y, d.y)


def test_residuals_match_oracle():
    inst = I.noisy_distances(45, seed=5, noise=0.8)
    g = C.NearnessSolver.from_instance(inst, b=16, prec="f64")
    o = oracle.Nearness(inst.n, inst.w, inst.dv)
    g.sweep(4)
    o.sweep(4, b=16)
    rg, ro = g.residuals(), o.residuals()
    for k in ("max_viol", "primal", "dual", "cs_max"):
        assert abs(rg[k] - ro[k]) <= 1e-10 * max(1.0, abs(ro[k])), (k, rg[k], ro[k])
    assert rg["stat_resid"] < 1e-12 and ro["stat_resid"] < 1e-12
    only = g.residuals(C.CC_RESID_VIOL)
    assert only["max_viol"] == rg["max_viol"] and np.isnan(only["dual"])


def test_solve_reaches_the_oracle_optimum():
    """Solved to a small violation and gap, the GPU point is the oracle's
    optimum (unique: strongly convex objective)."""
    inst = I.noisy_distances(30, seed=9, noise=0.7)
    g = C.NearnessSolver.from_instance(inst, b=8, prec="f64")
    r, ok = g.solve(tol=1e-11, gap_tol=1e-11, max_sweeps=50000)
    assert ok and r["max_viol"] <= 1e-11
    o = oracle.Nearness(inst.n, inst.w, inst.dv)
    o.solve(tol=1e-12, b=8, max_sweeps=200000, gap_tol=1e-12)
    assert rel_err(g.x.cpu().numpy(), o.x) <= 1e-8


def test_metric_is_a_fixed_point():
    inst = I.noisy_distances(50, seed=2, noise=0.0)
    g = C.NearnessSolver.from_instance(inst, b=16, prec="f64")
    g.sweep(2)
    g.status()
    assert np.array_equal(g.x.cpu().numpy(), inst.dv) and not g.y.any()
