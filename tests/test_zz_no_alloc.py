"""cc_sweep_noalloc (the allocation-free dataflow sweep, scratch in a static
device array) against cc_sweep with the dataflow executor, bit for bit,
through the C ABI: two calls in a row, the second on a smaller input."""
import pytest

from conftest import gpu_available
from paper_1901_10084_amd import instances as I

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C


def _pair(inst, b, prec):
    ref = C.Solver.from_instance(inst, b=b, prec=prec)
    new = C.Solver.from_instance(inst, b=b, prec=prec)
    return ref, new


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_sweeps_equal_dataflow_sweeps(prec):
    cases = [(I.random_signed(300, seed=21, gamma=3.0, weighted=True), 16, 4),
             (I.random_signed(70, seed=22, gamma=1.5, weighted=True), 32, 3)]  # smaller, ragged
    for inst, b, K in cases:
        print(f"noalloc n={inst.n} b={b} {prec} K={K}", flush=True)
        ref, new = _pair(inst, b, prec)
        ref.ctx.sweep(ref.x, ref.f, ref.y, ref.y_pair, ref.g, ref.d, K, C.CC_EXEC_DATAFLOW)
        ref.status()
        new.ctx.sweep_noalloc(new.x, new.f, new.y, new.y_pair, new.g, new.d, K)
        for a in ("x", "f", "y", "y_pair"):
            assert torch.equal(getattr(ref, a), getattr(new, a)), (inst.n, a)
        # calls continue from any state: one more sweep each, again equal
        ref.ctx.sweep(ref.x, ref.f, ref.y, ref.y_pair, ref.g, ref.d, 1, C.CC_EXEC_DATAFLOW)
        ref.status()
        new.ctx.sweep_noalloc(new.x, new.f, new.y, new.y_pair, new.g, new.d, 1)
        for a in ("x", "f", "y", "y_pair"):
            assert torch.equal(getattr(ref, a), getattr(new, a)), (inst.n, a, "second")


def test_noalloc_rejects_sizes_beyond_its_scratch():
    # ceil(n/b) = 256 blocks per side: 32,896 blocks of x, above the 32,766
    # the 4 MiB array holds; rejected before any work (the pointers are
    # never read)
    ctx = C.Context(2048, 8, "f32")
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    d8 = torch.zeros(16, dtype=torch.uint8, device="cuda")
    args = [dummy.data_ptr()] * 5 + [d8.data_ptr()]
    rc = C._L.cc_sweep_noalloc(ctx.handle, *args, 1)
    assert rc == C.CC_EINVAL
    assert "static scratch" in C.last_error()
    small = C.Context(64, 8, "f32")
    assert C._L.cc_sweep_noalloc(small.handle, *args, -1) == C.CC_EINVAL


def test_noalloc_at_its_largest_size():
    """ceil(n/b) = 255 blocks per side (n = 2040, b = 8: 32,640 blocks of x,
    the most the 4 MiB array holds): equal to cc_sweep bit for bit."""
    inst = I.random_signed(2040, seed=23, gamma=2.0, weighted=True)
    ref, new = _pair(inst, 8, "f32")
    ref.ctx.sweep(ref.x, ref.f, ref.y, ref.y_pair, ref.g, ref.d, 1, C.CC_EXEC_DATAFLOW)
    ref.status()
    new.ctx.sweep_noalloc(new.x, new.f, new.y, new.y_pair, new.g, new.d, 1)
    for a in ("x", "f", "y", "y_pair"):
        assert torch.equal(getattr(ref, a), getattr(new, a)), a
    del ref, new
    torch.cuda.empty_cache()
