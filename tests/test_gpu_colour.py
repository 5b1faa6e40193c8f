"""The sum-mod-n colouring order on the GPU (cc_sweep_colour) against the
oracle's colour order, through the C ABI."""
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


@pytest.mark.parametrize("n,K", [(3, 2), (4, 3), (10, 3), (33, 4), (60, 3), (97, 2)])
def test_colour_sweeps_match_the_oracle(n, K):
    inst = I.random_signed(n, seed=n, gamma=2.0)
    print(f"colour n={n} K={K}", flush=True)
    g = C.ColourSolver.from_instance(inst, prec="f64")
    o = oracle.State.from_instance(inst)
    g.sweep(K)
    o.sweep(K, order="colour")
    torch.cuda.synchronize()
    for a in ("x", "f", "y", "y_pair"):
        err = rel_err(getattr(g, a).cpu().numpy(), getattr(o, a))
        assert err <= 1e-10, (a, err)


def test_colour_f32_close_to_the_oracle():
    inst = I.random_signed(40, seed=2, gamma=3.0)
    g = C.ColourSolver.from_instance(inst, prec="f32")
    o = oracle.State.from_instance(inst)
    g.sweep(4)
    o.sweep(4, order="colour")
    assert rel_err(g.x.cpu().numpy(), o.x) <= 1e-5
    assert rel_err(g.y.cpu().numpy(), o.y) <= 1e-4


def test_colour_solve_takes_the_oracles_sweep_count():
    """The n = 60 workload solved to 1e-6 in the colour order: the same
    number of sweeps as the oracle's colour order, and the same point."""
    inst = I.workload(0)
    g = C.ColourSolver.from_instance(inst, prec="f64")
    r, ok, _ = g.solve(tol=1e-6, max_sweeps=5000, check_every=1)
    o = oracle.State.from_instance(inst)
    o.solve(tol=1e-6, max_sweeps=5000, order="colour")
    assert ok and g.sweeps == o.sweeps
    assert rel_err(g.x.cpu().numpy(), o.x) <= 1e-10


def test_colour_and_schedule_orders_reach_the_same_optimum():
    inst = I.random_signed(30, seed=4, gamma=2.0)
    a = C.ColourSolver.from_instance(inst, prec="f64")
    a.solve(tol=1e-11, max_sweeps=20000)
    b = C.Solver.from_instance(inst, b=8, prec="f64")
    b.solve(tol=1e-11, max_sweeps=20000)
    assert rel_err(a.x.cpu().numpy(), b.x.cpu().numpy()) <= 1e-8
