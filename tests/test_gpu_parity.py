"""GPU path against the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from paper_1901_10084_amd import instances as I
from parity_helpers import U64, one_sided_bound, rel_err, tol_f32, union_duals

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C


TOL64 = 1e-10   # FP64 GPU vs FP64 oracle, relative to max(1, |ref|_inf)


def compare_state(gs, os_, tol, what=""):
    x, f = gs.x.cpu().numpy(), gs.f.cpu().numpy()
    yp = gs.y_pair.cpu().numpy()
    ylex = gs.duals_lex().cpu().numpy()
    errs = dict(x=rel_err(x, os_.x), f=rel_err(f, os_.f), y_pair=rel_err(yp, os_.y_pair),
                y=rel_err(ylex, os_.y))
    print(what, errs, flush=True)
    for k, e in errs.items():
        assert e <= tol, (what, k, e)
    return errs


CASES = [
    # (instance, b, sweeps)
    (lambda: I.random_signed(13, seed=1, gamma=1.5, weighted=True), 4, 3),
    (lambda: I.random_signed(20, seed=2, gamma=0.8, weighted=True), 3, 5),
    (lambda: I.random_signed(37, seed=3, gamma=2.0, weighted=True), 8, 4),
    (lambda: I.random_signed(45, seed=4, gamma=1.0, weighted=False), 5, 3),
    (lambda: I.random_signed(70, seed=5, gamma=3.0, weighted=True), 32, 2),
    (lambda: I.random_signed(50, seed=9, gamma=2.0, weighted=True), 24, 3),  # b = 24, ragged tail of 2
    (lambda: I.random_signed(5, seed=6, gamma=1.0, weighted=True), 8, 6),    # one tile
    (lambda: I.random_signed(3, seed=7, gamma=1.0, weighted=True), 1, 10),   # one triplet
    (lambda: I.random_signed(17, seed=8, gamma=1.0, weighted=True), 1, 3),   # b = 1: Fig. 2
    (lambda: I.workload(0), 8, 20),
    (lambda: I.workload(0), 16, 3),
    (lambda: I.workload(0), 4, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sweep_parity_f64(case):
    mk, b, K = CASES[case]
    inst = mk()
    print(f"case {case}: n={inst.n} b={b} K={K}", flush=True)
    g = C.Solver.from_instance(inst, b=b, prec="f64")
    o = oracle.State.from_instance(inst)
    for k in range(K):
        g.sweep(1)
        o.sweep(1, b=b)
    compare_state(g, o, TOL64, f"n={inst.n} b={b} K={K}")


def test_parity_workload0_to_tolerance():
    """n = 60 Erdos-Renyi, gamma = 1: both reach max violation <= 1e-6 at the
    same sweep and agree there."""
    inst = I.workload(0)
    g = C.Solver.from_instance(inst, b=8)
    r, conv, _ = g.solve(tol=1e-6, max_sweeps=5000)
    assert conv
    o = oracle.State.from_instance(inst)
    ro = o.solve(tol=1e-6, b=8, max_sweeps=5000)
    assert o.sweeps == g.sweeps
    compare_state(g, o, TOL64, "workload0 converged")
    for key in ("max_viol_metric", "max_viol_pair", "primal_qp", "dual_qp", "lp_cost",
                "stat_resid"):
        assert abs(r[key] - ro[key]) <= 1e-9 * max(1.0, abs(ro[key])), key


def test_parity_workload1_three_sweeps():
    """n = 500 planted partition (62M metric rows), b = 16, full state after 3
    sweeps."""
    inst = I.workload(1)
    g = C.Solver.from_instance(inst, b=16)
    o = oracle.State.from_instance(inst)
    g.sweep(3)
    o.sweep(3, b=16)
    compare_state(g, o, TOL64, "workload1 K=3")


@pytest.mark.parametrize("n,b,rounds,executor", [(1500, 16, 3, "rounds"), (2000, 16, 2, "dataflow")])
def test_prefix_parity_large(n, b, rounds, executor):
    """Large instances: sweep 1, then the first rounds of sweep 2 (round by
    round, or on the dataflow executor in its full-sweep launch shape),
    against the oracle's sparse-dual prefix.  Duals are compared as dense
    vectors over the union of both sides' nonzero positions, so a dual
    nonzero on one side only must itself be within 1e-10; it must also be
    within the clipping bound of one_sided_bound (a value within rounding of
    zero)."""
    inst = I.workload(2) if n == 1500 else I.workload(3)
    g = C.Solver.from_instance(inst, b=b)
    g.sweep(1)
    if executor == "rounds":
        g.sweep_rounds(0, rounds)
    else:
        g.sweep_metric_prefix(rounds)
    x, f, yp, t, o, y = oracle.second_sweep_prefix(n, b, inst.gamma, inst.w, inst.d, rounds)
    gx = g.x.cpu().numpy()
    assert rel_err(gx, x) <= TOL64
    assert rel_err(g.f.cpu().numpy(), f) <= TOL64
    assert rel_err(g.y_pair.cpu().numpy(), yp) <= TOL64
    gpos, gval = g.nonzero_duals()
    assert (gpos >= 0).all()
    union, gv, ov, only = union_duals(gpos, gval, 3 * t + o.astype(np.int64), y)
    assert rel_err(gv, ov) <= TOL64
    bound = one_sided_bound(U64, float(np.abs(gx - x).max()), float(np.abs(y).max()),
                            float(np.abs(x).max()), float(inst.w.max()) / (3.0 * inst.gamma))
    worst = float(np.abs(gv - ov)[np.searchsorted(union, only)].max()) if only.size else 0.0
    print(f"prefix n={n}: {len(t)} nonzero duals, {only.size} on one side only, largest "
          f"{worst:.3e} (bound {bound:.3e})", flush=True)
    assert worst <= bound


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_residuals_and_x_from_y(prec):
    inst = I.random_signed(31, seed=9, gamma=2.5, weighted=True)
    g = C.Solver.from_instance(inst, b=8, prec=prec)
    o = oracle.State.from_instance(inst)
    g.sweep(7)
    o.sweep(7, b=8)
    r = g.residuals()
    ro = o.residuals()
    tol = 1e-9 if prec == "f64" else 2e-4
    for key in ro:
        assert abs(r[key] - ro[key]) <= tol * max(1.0, abs(ro[key])), (key, r[key], ro[key])
    x, f = g.x_from_y()
    xo, fo = o.x_from_y()
    assert rel_err(x.cpu().numpy(), xo) <= (1e-12 if prec == "f64" else 1e-5)
    assert rel_err(f.cpu().numpy(), fo) <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("n,b,prec", [(3, 1, "f64"), (5, 8, "f64"), (13, 4, "f64"), (37, 8, "f32"),
                                      (50, 24, "f64"), (70, 32, "f64"), (130, 16, "f32"),
                                      (100, 16, "f64"), (300, 32, "f32")])
def test_violation_check_matches_the_full_residuals(n, b, prec):
    """The violation-only check (cc_residuals with CC_RESID_VIOL, the solve's
    stop test) walks each lane's triplets in order rather than the
    conflict-free order; its maximum is the full residual pass's, bit for
    bit, and the oracle's.  A non-finite x is reported by both."""
    inst = I.random_signed(n, seed=n + 3 * b, gamma=2.0, weighted=True)
    g = C.Solver.from_instance(inst, b=b, prec=prec)
    o = oracle.State.from_instance(inst)
    g.sweep(2)
    o.sweep(2, b=b)
    rv = g.residuals(C.CC_RESID_VIOL)
    ra = g.residuals(C.CC_RESID_ALL)
    ro = o.residuals()
    print(n, b, prec, rv["max_viol_metric"], ra["max_viol_metric"], ro["max_viol_metric"], flush=True)
    assert rv["max_viol_metric"] == ra["max_viol_metric"]
    assert rv["max_viol_pair"] == ra["max_viol_pair"]
    tol = 1e-12 if prec == "f64" else 1e-5
    assert abs(rv["max_viol_metric"] - ro["max_viol_metric"]) <= tol * max(1.0, ro["max_viol_metric"])
    for bad in (float("nan"), float("inf")):
        h = C.Solver.from_instance(inst, b=b, prec=prec)
        h.sweep(1)
        h.x[h.x.numel() // 2] = bad
        assert h.residuals(C.CC_RESID_VIOL, raise_nonfinite=False).get("nonfinite")
        assert h.residuals(C.CC_RESID_ALL, raise_nonfinite=False).get("nonfinite")


@pytest.mark.parametrize("n,b,prec", [(45, 8, "f64"), (70, 16, "f64"), (100, 32, "f64"),
                                      (70, 16, "f32"), (73, 24, "f64")])
def test_x_from_y_dataflow(n, b, prec):
    """A'y runs on the dataflow schedule for b = 8, 16, 24, 32: equal to the
    oracle's x(y), and the same bits on every call (fixed summation order)."""
    inst = I.random_signed(n, seed=n + b, gamma=1.5, weighted=True)
    g = C.Solver.from_instance(inst, b=b, prec=prec)
    o = oracle.State.from_instance(inst)
    g.sweep(3)
    o.sweep(3, b=b)
    x1, f1 = g.x_from_y()
    x2, f2 = g.x_from_y()
    assert torch.equal(x1, x2) and torch.equal(f1, f2)
    xo, fo = o.x_from_y()
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel_err(x1.cpu().numpy(), xo) <= tol
    assert rel_err(f1.cpu().numpy(), fo) <= tol


F32_CASES = [
    # (instance, b, sweeps): the FP32 tile sizes of the larger workloads
    (lambda: I.random_signed(130, seed=11, gamma=5.0, weighted=False), 16, 3),  # ragged tail of 2
    (lambda: I.random_signed(300, seed=12, gamma=10.0, weighted=True), 32, 3),  # weighted, ragged
    (lambda: I.workload(1), 16, 3),                                             # n = 500
    (lambda: I.random_signed(200, seed=13, gamma=10.0, weighted=True), 32, 3),
    (lambda: I.random_signed(75, seed=14, gamma=3.0, weighted=True), 24, 3),   # b = 24, tail of 3
]


@pytest.mark.parametrize("case", range(len(F32_CASES)))
def test_sweep_parity_f32(case):
    """FP32 sweeps (the arithmetic of the n = 1500..4000 workloads: b = 16
    and 32, dataflow executor, W = diag(w)) against the FP64 oracle, element
    by element, to the FP32 rounding model of tol_f32 with the visits a
    variable gets (3 (n - 2) per sweep)."""
    mk, b, K = F32_CASES[case]
    inst = mk()
    g = C.Solver.from_instance(inst, b=b, prec="f32")
    o = oracle.State.from_instance(inst)
    g.sweep(K, C.CC_EXEC_DATAFLOW)
    o.sweep(K, b=b)
    tol = tol_f32(3 * (inst.n - 2) * K)
    print(f"f32 n={inst.n} b={b} K={K} tol {tol:.2e}", flush=True)
    compare_state(g, o, tol, f"f32 n={inst.n} b={b} K={K}")


def test_f32_close_to_oracle():
    """FP32 sweeps against the FP64 oracle: the error stays at FP32 level."""
    inst = I.workload(0)
    g = C.Solver.from_instance(inst, b=8, prec="f32")
    o = oracle.State.from_instance(inst)
    g.sweep(20)
    o.sweep(20, b=8)
    compare_state(g, o, 5e-5, "f32 workload0 K=20")


def test_padding_slots_stay_zero():
    inst = I.random_signed(19, seed=3, gamma=1.0, weighted=True)
    g = C.Solver.from_instance(inst, b=8)
    g.sweep(5)
    idx = torch.arange(g.ctx.slots, device="cuda", dtype=torch.int64)
    lex = torch.empty_like(idx)
    g.ctx.slots_to_lex(idx, lex)
    pad = lex < 0
    assert int((~pad).sum()) == C.num_metric_duals(19)
    assert not g.y[pad].any()
    # every colex index appears exactly once
    assert torch.equal(torch.sort(lex[~pad]).values,
                       torch.arange(C.num_metric_duals(19), device="cuda"))


def test_nonfinite_detected():
    inst = I.random_signed(12, seed=1)
    g = C.Solver.from_instance(inst, b=4)
    g.sweep(2)
    g.x[5] = float("nan")
    r = g.residuals(C.CC_RESID_VIOL, raise_nonfinite=False)
    assert r.get("nonfinite")
    with pytest.raises(C.CCError) as e:
        g.residuals(C.CC_RESID_VIOL)
    assert e.value.code == C.CC_ENONFINITE


def test_bad_weights_rejected():
    inst = I.random_signed(10, seed=1)
    w = inst.w.copy()
    w[3] = 0.0
    with pytest.raises(C.CCError) as e:
        C.Solver(inst.n, w, inst.d, 1.0, b=4)
    assert e.value.code == C.CC_EINVAL
    w[3] = np.inf
    with pytest.raises(C.CCError):
        C.Solver(inst.n, w, inst.d, 1.0, b=4)


def test_duals_nonnegative_and_stationary():
    inst = I.workload(0)
    g = C.Solver.from_instance(inst, b=8)
    g.sweep(50)
    assert float(g.y.min()) >= 0.0 and float(g.y_pair.min()) >= 0.0
    r = g.residuals()
    assert r["stat_resid"] < 1e-12


# --------------------------------------------------------------------------
# Dataflow executor: same updates in the same order per variable, so the
# result must equal the round-by-round executor bit for bit.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,b,prec,K", [(60, 8, "f64", 3), (61, 8, "f64", 2), (100, 16, "f64", 3),
                                        (130, 32, "f64", 2), (200, 16, "f32", 3),
                                        (150, 32, "f32", 2), (3, 8, "f64", 2), (5, 8, "f64", 2),
                                        (16, 16, "f64", 2), (17, 16, "f32", 2), (33, 32, "f64", 2),
                                        (500, 16, "f64", 2), (300, 8, "f32", 2),
                                        (1000, 32, "f32", 1), (200, 8, "f64", 10),
                                        (600, 16, "f32", 5), (50, 24, "f64", 3), (97, 24, "f32", 2),
                                        (24, 24, "f64", 2), (500, 24, "f64", 2)])
def test_dataflow_equals_rounds(n, b, prec, K):
    inst = I.workload(1) if n == 500 else I.random_signed(n, seed=n, gamma=2.0, weighted=True)
    print(f"dataflow n={n} b={b} {prec} K={K}", flush=True)
    r = C.Solver.from_instance(inst, b=b, prec=prec)
    d = C.Solver.from_instance(inst, b=b, prec=prec)
    r.sweep(K, C.CC_EXEC_ROUNDS)
    d.sweep(K, C.CC_EXEC_DATAFLOW)
    d.status()
    for name in ("x", "f", "y", "y_pair"):
        a, bb = getattr(r, name), getattr(d, name)
        assert torch.equal(a, bb), (name, float((a - bb).abs().max()))


@pytest.mark.parametrize("n,b,prec", [(100, 16, "f64"), (130, 24, "f32"), (70, 8, "f64")])
def test_dataflow_workgroup_count_leaves_results_unchanged(n, b, prec):
    """Any number of workgroups gives the default sweep's bits: one
    workgroup runs the tiles one after another in schedule order; a request
    above what the GPU holds at once is capped."""
    inst = I.random_signed(n, seed=n + b, gamma=2.0, weighted=True)
    ref = C.Solver.from_instance(inst, b=b, prec=prec)
    ref.sweep(3, C.CC_EXEC_DATAFLOW)
    ref.status()
    default = ref.ctx.set_dataflow_workgroups(0)
    assert default >= 1
    for wg in (1, 2, 7, 1 << 20):
        s = C.Solver.from_instance(inst, b=b, prec=prec)
        eff = s.ctx.set_dataflow_workgroups(wg)
        assert eff == wg if wg < default else 1 <= eff <= max(wg, default)
        print(f"workgroups n={n} b={b} {prec}: asked {wg}, ran {eff}", flush=True)
        s.sweep(3, C.CC_EXEC_DATAFLOW)
        s.status()
        for name in ("x", "f", "y", "y_pair"):
            assert torch.equal(getattr(ref, name), getattr(s, name)), (wg, name)
    with pytest.raises(C.CCError):
        ref.ctx.set_dataflow_workgroups(-1)


def test_dataflow_breakdown_counts_every_step():
    """The diagnostic sweep runs the same updates (same bits as a plain
    dataflow sweep) and counts every tile step once."""
    n, b = 100, 16
    inst = I.random_signed(n, seed=3, gamma=1.0, weighted=True)
    a = C.Solver.from_instance(inst, b=b)
    c = C.Solver.from_instance(inst, b=b)
    a.sweep_metric(C.CC_EXEC_DATAFLOW)
    a.status()
    br = c.ctx.dataflow_breakdown(c.x, c.y, c.g)
    nb = (n + b - 1) // b
    assert br["tile_steps"] == nb * (nb + 1) * (nb + 2) // 6
    assert br["workgroups"] >= 1
    assert all(br[k] >= 0 for k in ("wait_us", "load_us", "substeps_us", "publish_us"))
    assert torch.equal(a.x, c.x) and torch.equal(a.y, c.y)


def test_dataflow_parity_oracle():
    inst = I.random_signed(70, seed=4, gamma=1.5, weighted=True)
    g = C.Solver.from_instance(inst, b=8)
    o = oracle.State.from_instance(inst)
    g.sweep(6, C.CC_EXEC_DATAFLOW)
    g.status()
    o.sweep(6, b=8)
    compare_state(g, o, TOL64, "dataflow n=70 K=6")


# --------------------------------------------------------------------------
# One-shot solve: FP64, FP32, and FP32 sweeps followed by FP64 polish.
# --------------------------------------------------------------------------
def test_solve_modes():
    inst = I.workload(0)
    rc64, x64, y64, i64 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=8,
                                        mode=C.CC_MODE_F64, want_duals=True)
    assert rc64 == C.CC_OK
    o = oracle.State.from_instance(inst)
    ro = o.solve(tol=1e-6, b=8, max_sweeps=5000)
    assert i64["sweeps"] == o.sweeps
    assert rel_err(x64, o.x) <= TOL64 and rel_err(y64, o.y) <= TOL64
    rc32, x32, _, i32 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-4, b=8,
                                      mode=C.CC_MODE_F32)
    assert rc32 == C.CC_OK and i32["sweeps_f32"] == i32["sweeps"]
    assert max(i32["resid"]["max_viol_metric"], i32["resid"]["max_viol_pair"]) <= 1e-4
    rcp, xp, _, ip = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=8,
                                   mode=C.CC_MODE_F32_POLISH)
    assert rcp == C.CC_OK and 0 < ip["sweeps_f32"] < ip["sweeps"]
    r = ip["resid"]
    assert max(r["max_viol_metric"], r["max_viol_pair"]) <= 1e-6
    # the polished solution is the FP64 one (unique primal optimum of the QP)
    assert abs(r["primal_qp"] - ro["primal_qp"]) <= 1e-5 * abs(ro["primal_qp"])
    assert rel_err(xp, o.x) <= 1e-4
    print("sweeps f64", i64["sweeps"], "f32", i32["sweeps"], "polish", ip["sweeps_f32"],
          ip["sweeps"], flush=True)


def test_solve_gap_tolerance():
    """Stop on max violation and the relative duality gap: the one-shot solve
    and the Solver take the oracle's sweep count under the same test, and
    the gap they stop at meets the bound."""
    inst = I.workload(0)
    o = oracle.State.from_instance(inst)
    ro = o.solve(tol=1e-6, b=8, max_sweeps=5000, gap_tol=1e-10)
    _, _, _, iv = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=8)
    rc, x, _, ig = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=8, gap_tol=1e-10)
    assert rc == C.CC_OK and ig["sweeps"] == o.sweeps >= iv["sweeps"]
    r = ig["resid"]
    assert abs(r["gap"]) <= 1e-10 * max(1.0, abs(r["primal_qp"]))
    assert rel_err(x, o.x) <= TOL64
    g = C.Solver.from_instance(inst, b=8)
    rg, ok, _ = g.solve(tol=1e-6, gap_tol=1e-10, max_sweeps=5000)
    assert ok and g.sweeps == o.sweeps
    with pytest.raises(C.CCError):
        C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=8, gap_tol=float("nan"))
    print("sweeps: violation only", iv["sweeps"], "with the gap", ig["sweeps"], flush=True)


def test_solve_not_converged_reports():
    inst = I.workload(0)
    rc, x, _, info = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-12, b=8,
                                   max_sweeps=5, mode=C.CC_MODE_F64)
    assert rc == C.CC_ENOTCONV and info["sweeps"] == 5
    assert info["resid"]["max_viol_metric"] > 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_prepare_and_cold_start_are_exact(prec):
    """a1: g = gamma / w, rounded once to the working precision; a2: the
    starting point of Algorithm 1, x = 0, f = -gamma, every dual 0, equal
    to the oracle's."""
    inst = I.random_signed(23, seed=3, gamma=2.5, weighted=True)
    g = C.Solver.from_instance(inst, b=8, prec=prec)
    dt = np.float64 if prec == "f64" else np.float32
    assert np.array_equal(g.g.cpu().numpy(), (inst.gamma / inst.w).astype(dt))
    o = oracle.State.from_instance(inst)
    assert np.array_equal(g.x.cpu().numpy().astype(np.float64), o.x)
    assert np.array_equal(g.f.cpu().numpy().astype(np.float64), o.f)
    assert np.array_equal(g.y_pair.cpu().numpy().astype(np.float64), o.y_pair)
    assert not g.y.any()
