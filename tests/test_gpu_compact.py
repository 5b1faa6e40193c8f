"""Compacted dual lists (the memory form of Sec. III-D) on the GPU: sweeps
without a dense dual array must equal the dense sweeps bit for bit, also
when a pool overflows and the sweep is repeated into a larger one, and the
exported nonzero duals must equal the oracle's."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from paper_1901_10084_amd import instances as I

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C


@pytest.mark.parametrize("n,b,prec,K", [(40, 8, "f64", 3), (33, 16, "f64", 4), (70, 16, "f64", 3),
                                        (100, 16, "f32", 3), (300, 16, "f64", 3), (61, 8, "f32", 4)])
def test_compact_sweeps_equal_dense(n, b, prec, K):
    inst = I.random_signed(n, seed=n, gamma=3.0)
    print(f"compact n={n} b={b} {prec} K={K}", flush=True)
    dense = C.Solver.from_instance(inst, b=b, prec=prec)
    comp = C.CompactSolver.from_instance(inst, b=b, prec=prec, capacity=1 << 16)
    for _ in range(K):
        dense.sweep(1)
        comp.sweep(1)
        assert torch.equal(dense.x, comp.x) and torch.equal(dense.f, comp.f)
        assert torch.equal(dense.y_pair, comp.y_pair)
        y = comp.to_slots()
        assert torch.equal(dense.y.view(torch.uint8), y.view(torch.uint8))
        nz = int(torch.count_nonzero(dense.y))
        assert comp.info()["nnz"] == nz


def test_pool_overflow_repeats_the_sweep():
    """A pool of 1 entry overflows at the first nonzero dual: the sweep is
    repeated from the saved x into a grown pool, with the dense result."""
    inst = I.workload(0)
    dense = C.Solver.from_instance(inst, b=8, prec="f64")
    comp = C.CompactSolver.from_instance(inst, b=8, prec="f64", capacity=1)
    dense.sweep(6)
    comp.sweep(6)
    info = comp.info()
    assert info["regrows"] >= 1 and info["nnz"] > 1
    assert torch.equal(dense.x, comp.x) and torch.equal(dense.f, comp.f)
    assert torch.equal(dense.y, comp.to_slots())


def test_export_matches_the_oracle():
    inst = I.planted_partition(45, 3, 0.4, 0.05, seed=7, gamma=2.0)
    comp = C.CompactSolver.from_instance(inst, b=16, prec="f64")
    o = oracle.State.from_instance(inst)
    comp.sweep(5)
    o.sweep(5, b=16)
    lex, val = comp.export()
    lex, val = lex.cpu().numpy(), val.cpu().numpy()
    assert len(np.unique(lex)) == len(lex)
    got = np.zeros_like(o.y)
    got[lex] = val
    assert np.abs(got - o.y).max() <= 1e-10 * max(1.0, np.abs(o.y).max())
    assert np.abs(comp.x.cpu().numpy() - o.x).max() <= 1e-10


def test_solve_with_compacted_lists_takes_the_dense_sweeps():
    inst = I.workload(0)
    comp = C.CompactSolver.from_instance(inst, b=8, prec="f64")
    r, ok, _ = comp.solve(tol=1e-6, max_sweeps=5000, check_every=1)
    o = oracle.State.from_instance(inst)
    o.solve(tol=1e-6, b=8, max_sweeps=5000)
    assert ok and comp.sweeps == o.sweeps


def test_compacted_lists_reject_b32():
    inst = I.workload(0)
    with pytest.raises(C.CCError):
        C.CompactSolver.from_instance(inst, b=32, prec="f64")
