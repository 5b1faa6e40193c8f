"""The largest workloads at full size, in the launch configuration the
benchmark times, checked through properties that hold at any size (the
oracle cannot run whole sweeps here: one FP64 sweep at n = 4000 would take
about ten minutes on one core).  Smaller sizes are compared with the oracle
element by element in the other GPU tests."""
import pytest

from conftest import gpu_available
from paper_1901_10084_amd import instances as I

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C

CHUNK = 1 << 28


def chunked_min(t):
    return min(float(t[i:i + CHUNK].min()) for i in range(0, t.numel(), CHUNK))


def chunked_equal(a, b):
    return all(torch.equal(a[i:i + CHUNK], b[i:i + CHUNK]) for i in range(0, a.numel(), CHUNK))


def test_n4000_f32_dataflow_sweeps_keep_the_invariants():
    """n = 4000 Chung-Lu, FP32 duals (128 GB), b = 32, dataflow executor.
    Hildreth's method is exact dual coordinate ascent (Sec. II-B): the dual
    objective never falls, the duals stay nonnegative, and x stays x(y),
    here to FP32 rounding (stat_resid is max |x - x(y)| with x(y) rebuilt
    from the duals in FP64)."""
    inst = I.workload(4)
    print(f"full size n={inst.n} b=32 f32", flush=True)
    g = C.Solver.from_instance(inst, b=32, prec="f32")
    duals = []
    for k in range(3):
        g.sweep(1)
        r = g.residuals()
        duals.append(r["dual_qp"])
        print(f"sweep {k + 1}: dual {r['dual_qp']:.6f} max violation "
              f"{max(r['max_viol_metric'], r['max_viol_pair']):.3e} stat {r['stat_resid']:.2e}",
              flush=True)
        assert r["stat_resid"] <= 1e-4
    g.status()
    for a, b_ in zip(duals, duals[1:]):
        assert b_ >= a - 1e-6 * abs(a)
    assert chunked_min(g.y) >= 0.0 and float(g.y_pair.min()) >= 0.0
    del g
    torch.cuda.empty_cache()  # hand the 128 GB back before the next test


def test_n2000_f32_sparse_equals_dense():
    """The sparse sweep at the size and tile of its benchmark (n = 2000,
    FP32, b = 16) equals the dense one bit for bit, and its mask stays the
    nonzero pattern of the duals (counted)."""
    inst = I.workload(3)
    dense = C.Solver.from_instance(inst, b=16, prec="f32")
    sparse = C.Solver.from_instance(inst, b=16, prec="f32")
    for _ in range(3):
        dense.sweep(1)
        sparse.sweep(1, sparse=True)
    sparse.status()
    assert torch.equal(dense.x, sparse.x) and torch.equal(dense.f, sparse.f)
    assert torch.equal(dense.y_pair, sparse.y_pair)
    assert chunked_equal(dense.y.view(torch.int32), sparse.y.view(torch.int32))
    bits = sum(int(torch.bitwise_and(sparse.mask[i:i + CHUNK].unsqueeze(1) >>
                                     torch.arange(8, device="cuda", dtype=torch.uint8), 1).sum())
               for i in range(0, sparse.mask.numel(), CHUNK))
    nonzero = sum(int(torch.count_nonzero(sparse.y[i:i + CHUNK].view(torch.int32)))
                  for i in range(0, sparse.y.numel(), CHUNK))
    assert bits == nonzero > 0
    del dense, sparse
    torch.cuda.empty_cache()
