"""GPU warm-start network against its float64 reference, and the warm start
itself (valid start, same optimum, what it gains)."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from oracle import mlp_ref as M
from paper_1901_10084_amd import instances as I

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1901_10084_amd import ccproj as C
    from paper_1901_10084_amd import warmstart as W


def test_param_count_and_init():
    assert W.NPARAM == M.NPARAM == 1249
    p0, p1 = W.init_params(7), W.init_params(7)
    assert np.array_equal(p0, p1) and np.isfinite(p0).all()


@pytest.mark.parametrize("count", [1, 16, 17, 1000, 4099])
def test_forward_matches_reference(count):
    rng = np.random.default_rng(count)
    p = M.init_params(11)
    phi = rng.normal(0, 1, (count, 4)).astype(np.float32)
    net = W.Network(params=p)
    y = net.forward(torch.as_tensor(phi).cuda()).cpu().numpy()
    yr, _ = M.forward(p, phi)
    assert np.abs(y - yr).max() <= 1e-3 * max(1.0, np.abs(yr).max()), np.abs(y - yr).max()
    assert (y >= 0).all()


@pytest.mark.parametrize("count", [32, 100, 5000])
def test_gradient_matches_reference(count):
    rng = np.random.default_rng(count + 1)
    p = M.init_params(12)
    phi = rng.normal(0, 1, (count, 4)).astype(np.float32)
    t = np.maximum(rng.normal(0.5, 0.5, count), 0).astype(np.float32)
    net = W.Network(params=p)
    g = torch.zeros(W.NPARAM, dtype=torch.float32, device="cuda")
    loss = net.train_step(torch.as_tensor(phi).cuda(), torch.as_tensor(t).cuda(), lr=0.0,
                          grad_out=g)
    lr_, gr = M.loss_and_grad(p, phi, t)
    g = g.cpu().numpy()
    assert abs(float(loss) - lr_) <= 1e-4 * abs(lr_)
    err = np.abs(g - gr).max() / np.abs(gr).max()
    print("grad rel err", err, flush=True)
    # Every block of parameters against its own largest reference gradient:
    # the reference takes the GPU's bf16 roundings, so what remains is the
    # fp32 accumulation order of the MFMA products and reductions, a few
    # fp32 ulps of a block's sums (measured below 1e-6).
    for name, lo, hi in (("W1", 0, 128), ("b1", 128, 160), ("W2", 160, 1184),
                         ("b2", 1184, 1216), ("W3", 1216, 1248), ("b3", 1248, 1249)):
        ref = gr[lo:hi]
        scale = np.abs(ref).max()
        if scale == 0.0:
            assert not g[lo:hi].any(), name
            continue
        e = np.abs(g[lo:hi] - ref).max() / scale
        gb = g[lo:hi].astype(np.float64)
        cos = float(gb @ ref / (np.linalg.norm(gb) * np.linalg.norm(ref)))
        print(f"  {name}: rel err {e:.2e} cosine {cos:.9f}", flush=True)
        assert e <= 1e-5, (name, e)
        assert cos >= 1.0 - 1e-9, (name, cos)


def test_slot_features_match_reference():
    inst = I.random_signed(23, seed=2, gamma=1.0, weighted=True)
    s = C.Solver.from_instance(inst, b=8)
    deg = W.degrees(inst)
    slots = torch.arange(s.ctx.slots, device="cuda", dtype=torch.int64)
    lex = torch.empty_like(slots)
    s.ctx.slots_to_lex(slots, lex)
    phi = W.slot_features(s, deg, slots).cpu().numpy()
    lex = lex.cpu().numpy()
    valid = lex >= 0
    assert not phi[~valid].any()
    t, o = lex[valid] // 3, lex[valid] % 3
    # colex triplet index -> (i, j, k)
    k = np.floor(np.cbrt(6.0 * t)).astype(np.int64) + 2
    while True:
        over = k * (k - 1) * (k - 2) // 6 > t
        if not over.any():
            break
        k[over] -= 1
    r = t - k * (k - 1) * (k - 2) // 6
    j = np.floor(np.sqrt(2.0 * r)).astype(np.int64) + 1
    while True:
        over = j * (j - 1) // 2 > r
        if not over.any():
            break
        j[over] -= 1
    i = r - j * (j - 1) // 2
    ref = M.bf16(M.features(inst.d, inst.w, inst.deg, i, j, k, o))
    assert np.allclose(phi[valid], ref, rtol=0, atol=1e-6)


def colex_triplets(t):
    """(i, j, k) of colex triplet indices t (numpy int64 arrays)."""
    k = np.floor(np.cbrt(6.0 * t)).astype(np.int64) + 2
    while True:
        over = k * (k - 1) * (k - 2) // 6 > t
        if not over.any():
            break
        k[over] -= 1
    r = t - k * (k - 1) * (k - 2) // 6
    j = np.floor(np.sqrt(2.0 * r)).astype(np.int64) + 1
    while True:
        over = j * (j - 1) // 2 > r
        if not over.any():
            break
        j[over] -= 1
    return r - j * (j - 1) // 2, j, k


@pytest.mark.parametrize("n,b,prec", [(23, 8, "f32"), (40, 16, "f32"), (70, 32, "f32"),
                                      (37, 16, "f64"), (19, 5, "f32")])
def test_inference_matches_reference(n, b, prec):
    """cc_mlp_infer on every schedule slot against the float64 reference
    network on the reference features, divided by n - 2; padding gets 0."""
    inst = I.random_signed(n, seed=n, gamma=1.0, weighted=True)
    s = C.Solver.from_instance(inst, b=b, prec=prec)
    deg = W.degrees(inst)
    p = M.init_params(5)
    net = W.Network(params=p)
    yv = torch.full_like(s.y, -1.0)
    W.infer(s, net, deg, yv)
    slots = torch.arange(s.ctx.slots, device="cuda", dtype=torch.int64)
    lex = torch.empty_like(slots)
    s.ctx.slots_to_lex(slots, lex)
    yv, lex = yv.cpu().numpy().astype(np.float64), lex.cpu().numpy()
    valid = lex >= 0
    assert not yv[~valid].any()
    t, o = lex[valid] // 3, lex[valid] % 3
    i, j, k = colex_triplets(t)
    phi = M.features(inst.d, inst.w, inst.deg, i, j, k, o)
    yr, _ = M.forward(p, phi)
    yr = yr / (n - 2)
    e = np.abs(yv[valid] - yr) / max(1e-30, np.abs(yr).max())
    q999 = np.quantile(e, 0.999)
    print("inference rel err: max %.3g, 99.9%% %.3g, median %.3g, rows %d"
          % (e.max(), q999, np.median(e), e.size), flush=True)
    # The kernel accumulates in fp32 (MFMA) before each bf16 rounding of the
    # hidden layers, the reference in float64: a hidden value on a bf16
    # rounding boundary can land one bf16 step apart, which moves that row's
    # output by up to a few 1e-3.  A wrong feature, orientation or slot moves
    # a large share of rows.
    assert q999 <= 1e-3
    assert e.max() <= 2e-2


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    phi = rng.normal(0, 1, (8192, 4)).astype(np.float32)
    t = np.maximum(0.5 * phi[:, 0] - 0.3 * phi[:, 1] * phi[:, 2] + 0.2, 0).astype(np.float32)
    net = W.Network(seed=1)
    P, T = torch.as_tensor(phi).cuda(), torch.as_tensor(t).cuda()
    first = float(net.train_step(P, T, lr=3e-3))
    for _ in range(400):
        last = float(net.train_step(P, T, lr=3e-3))
    print("loss", first, "->", last, flush=True)
    assert last < 0.2 * first


def small_trained_network(n_graphs=8):
    net, hist = W.train(seeds=range(1000, 1000 + n_graphs), tol=1e-5, steps_per_graph=60,
                        batch=8192, lr=3e-3)
    return net, hist


def test_warm_start_is_valid_and_reaches_the_same_optimum():
    net, hist = small_trained_network(4)
    inst = I.training_graph(2000)                     # held out
    deg = W.degrees(inst)
    cold = C.Solver.from_instance(inst, b=16)
    rc, conv_c, _ = cold.solve(tol=1e-6, executor=C.CC_EXEC_DATAFLOW)
    warm = C.Solver.from_instance(inst, b=16)
    info = W.warm_start(warm, net, deg)
    print("warm start", info, flush=True)
    assert float(warm.y.min()) >= 0.0
    rw, conv_w, _ = warm.solve(tol=1e-6, executor=C.CC_EXEC_DATAFLOW)
    assert conv_c and conv_w
    assert rw["stat_resid"] < 1e-9
    # unique primal optimum of the QP
    assert abs(rw["primal_qp"] - rc["primal_qp"]) <= 1e-6 * abs(rc["primal_qp"])
    assert float((warm.x - cold.x).abs().max()) <= 1e-4
    print("sweeps to 1e-6: cold", cold.sweeps, "warm", warm.sweeps, flush=True)


def test_warm_start_gain_report():
    """What the trained network gains: sweeps and time to max violation
    <= 1e-4 in FP32 on held-out planted partitions (n = 300, the training
    family), learned start vs cold start.  The shipped network (trained by
    warmstart.train on 200 graphs with the library's own kernels) must save
    at least a quarter of the sweeps and reach the same objective; a network
    trained here on 16 graphs is reported beside it."""
    import time
    nets = {"shipped": W.load(), "16 graphs": small_trained_network(16)[0]}
    for seed in (2001, 2002, 2003):
        inst = I.training_graph(seed)
        deg = W.degrees(inst)
        cold = C.Solver.from_instance(inst, b=16, prec="f32")
        rc, cc, tc = cold.solve(tol=1e-4, executor=C.CC_EXEC_DATAFLOW)
        assert cc
        for name, net in nets.items():
            warm = C.Solver.from_instance(inst, b=16, prec="f32")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = W.warm_start(warm, net, deg)
            rw, cw, _ = warm.solve(tol=1e-4, executor=C.CC_EXEC_DATAFLOW)
            tw = time.perf_counter() - t0
            print(f"seed {seed} {name}: accepted {info['accepted']} sweeps cold {cold.sweeps} "
                  f"warm {warm.sweeps} time cold {tc:.4f} warm {tw:.4f} objective "
                  f"{rc['primal_qp']:.6f} {rw['primal_qp']:.6f}", flush=True)
            assert cw
            assert abs(rw["primal_qp"] - rc["primal_qp"]) <= 1e-3 * abs(rc["primal_qp"])
            if name == "shipped":
                assert info["accepted"]
                assert warm.sweeps <= 0.75 * cold.sweeps, (warm.sweeps, cold.sweeps)


def test_gate_rejects_a_bad_prediction():
    """A network whose output bias is huge predicts every dual far too
    large: the dual objective falls, the gate rejects the prediction and the
    state is the cold start, bit for bit, in both precisions."""
    p = M.init_params(3)
    p[1248] = 1.0e3                       # output bias: every prediction is huge
    net = W.Network(params=p)
    inst = I.training_graph(2001)
    deg = W.degrees(inst)
    for prec in ("f32", "f64"):
        warm = C.Solver.from_instance(inst, b=16, prec=prec)
        warm.sweep(2)                     # start from a state that is not the cold one
        info = W.warm_start(warm, net, deg)
        cold = C.Solver.from_instance(inst, b=16, prec=prec)
        print(prec, info, flush=True)
        assert not info["accepted"]
        assert info["dual_warm"] < info["dual_cold"]
        for a in ("x", "f", "y", "y_pair"):
            assert torch.equal(getattr(warm, a), getattr(cold, a)), a


def test_gate_bound_and_share():
    """The gate's bound U is the objective of (qp) at the best constant point
    x = c, f = |c - d| (every row holds there), found here by brute force
    over c; it lies above the optimum the solve reaches, and the kept start
    closes at least 5% of the gap U - D_cold."""
    inst = I.training_graph(2002)
    w, d, gam = inst.w.astype(np.float64), inst.d.astype(np.float64), inst.gamma
    cs = np.linspace(0.0, 1.0, 20001)
    P = [float(np.sum(w * np.abs(c - d)) + np.sum(w * (c * c + (c - d) ** 2)) / (2 * gam)) for c in cs]
    s = C.Solver.from_instance(inst, b=16, prec="f64")
    info = W.warm_start(s, W.load(), W.degrees(inst))
    print(info, min(P), flush=True)
    assert abs(info["dual_bound"] - min(P)) <= 1e-9 * min(P)
    r, conv, _ = s.solve(tol=1e-8)
    assert conv and r["primal_qp"] <= info["dual_bound"]
    assert info["dual_cold"] <= info["dual_warm"] <= r["primal_qp"]
    assert info["accepted"] and info["gap_share"] >= 0.05


@pytest.mark.parametrize("b,prec", [(8, "f32"), (16, "f32"), (32, "f32"), (16, "f64"), (24, "f32")])
def test_fused_warm_start_equals_the_separate_passes(b, prec):
    """For b = 8, 16, 24, 32 the warm start runs the network fused with A'y
    on the dataflow executor.  Its duals equal cc_mlp_infer's bit for bit
    (b = 8, 16, 32; b = 24 against the reference network), and its x, f and
    pair duals equal those of cc_x_from_y on the same duals followed by one
    pair pass, bit for bit: the fused sums are A'y's."""
    inst = I.training_graph(2001)
    net, deg = W.load(), W.degrees(inst)
    s = C.Solver.from_instance(inst, b=b, prec=prec)
    info = W.warm_start(s, net, deg)
    assert info["accepted"]
    r = C.Solver.from_instance(inst, b=b, prec=prec)
    if b != 24:
        W.infer(r, net, deg, r.y)
        assert torch.equal(r.y, s.y)
    else:
        slots = torch.arange(s.ctx.slots, device="cuda", dtype=torch.int64)
        lex = torch.empty_like(slots)
        s.ctx.slots_to_lex(slots, lex)
        yv, lex = s.y.cpu().numpy().astype(np.float64), lex.cpu().numpy()
        valid = lex >= 0
        assert not yv[~valid].any()
        i, j, k = colex_triplets(lex[valid] // 3)
        yr, _ = M.forward(net.host_params(), M.features(inst.d, inst.w, inst.deg, i, j, k, lex[valid] % 3))
        e = np.abs(yv[valid] - yr / (inst.n - 2)) / np.abs(yr / (inst.n - 2)).max()
        assert np.quantile(e, 0.999) <= 1e-3 and e.max() <= 2e-2
    r.y.copy_(s.y)
    r.y_pair.zero_()
    x, f = r.x_from_y()
    r.x.copy_(x)
    r.f.copy_(f)
    r.pair_pass()
    for a in ("x", "f", "y_pair"):
        assert torch.equal(getattr(r, a), getattr(s, a)), a


# --------------------------------------------------------------------------
# The sampled gate: per-pair terms of D_warm - D_cold (cc_warm_gate_terms)
# and the early rejection it allows (cc_set_gate_sample).
# --------------------------------------------------------------------------
def _oracle_predictions(inst, params):
    """The reference network's dual for every metric row, colex order."""
    i, j, k = oracle.colex_triplets(inst.n)
    y = np.zeros((i.size, 3))
    for o in range(3):
        phi = M.features(inst.d, inst.w, inst.deg, i, j, k, np.full(i.size, o))
        y[:, o] = M.forward(params, phi)[0] / (inst.n - 2)
    return y.ravel()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gate_terms_match_the_oracle(prec):
    """Every pair's metric A'y at the predicted duals and its term of
    D_warm - D_cold, against the oracle's on its own reference predictions.
    The network differs from the reference only where a hidden value sits
    on a bf16 rounding boundary (see test_inference_matches_reference); a
    wrong coefficient, side or row moves a pair's sum by whole predictions."""
    inst = I.planted_partition(60, 3, 0.25, 0.05, seed=3, gamma=5.0)
    net, deg = W.load(), W.degrees(inst)
    ref = oracle.gate_pair_terms(inst.n, inst.gamma, inst.w, inst.d,
                                 _oracle_predictions(inst, net.host_params()))
    s = C.Solver.from_instance(inst, b=16, prec=prec)
    npairs = inst.n * (inst.n - 1) // 2
    rng = np.random.default_rng(0)
    pairs = np.concatenate([np.arange(npairs), rng.integers(0, npairs, 200)])
    aty, delta = W.gate_terms(s, net, deg, torch.as_tensor(pairs))
    aty, delta = aty.cpu().numpy(), delta.cpu().numpy()
    ra, rd = ref["aty"][pairs], (ref["term_warm"] - ref["term_cold"])[pairs]
    ea = np.abs(aty - ra) / np.abs(ra).max()
    ed = np.abs(delta - rd) / np.abs(rd).max()
    print(f"{prec}: A'y rel err max {ea.max():.3g} median {np.median(ea):.3g}; "
          f"delta rel err max {ed.max():.3g} median {np.median(ed):.3g}", flush=True)
    assert ea.max() <= 1e-2 and np.median(ea) <= 1e-4
    assert ed.max() <= 1e-2 and np.median(ed) <= 1e-4
    # repeats of a pair give the same bits
    for e in range(npairs, pairs.size):
        assert aty[e] == aty[pairs[e]] and delta[e] == delta[pairs[e]]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gate_terms_sum_to_the_exact_gate(prec):
    """Over all pairs the terms add up to the exact gate's D_warm - D_cold,
    and each pair's A'y is the full inference's (x(y) of the predicted duals
    with zero pair duals is -gamma A'y / w).  Only the FP64 summation order of
    A'y differs, and in FP32 the rounding of x = x(y) that follows it."""
    inst = I.training_graph(2001)
    net, deg = W.load(), W.degrees(inst)
    s = C.Solver.from_instance(inst, b=16, prec=prec)
    s.ctx.set_gate_sample(0)
    info = W.warm_start(s, net, deg)
    assert info["sample_drawn"] == 0 and info["accepted"]
    npairs = inst.n * (inst.n - 1) // 2
    r = C.Solver.from_instance(inst, b=16, prec=prec)
    aty, delta = W.gate_terms(r, net, deg, torch.arange(npairs))
    gap = info["dual_bound"] - info["dual_cold"]
    got, want = float(delta.sum()), info["dual_warm"] - info["dual_cold"]
    print(f"{prec}: sum of terms {got:.9g}, exact gain {want:.9g}, gap {gap:.6g}", flush=True)
    assert abs(got - want) <= (1e-10 if prec == "f64" else 1e-6) * gap
    if prec == "f64":
        W.infer(r, net, deg, r.y)
        r.y_pair.zero_()
        x, _ = r.x_from_y()
        full = -x.double() * r.w / inst.gamma
        assert float((aty - full).abs().max()) <= 1e-13 * float(full.abs().max())


def test_sampled_gate_rejects_a_bad_start_early():
    """A network that predicts every dual far too large: the sample alone
    rejects it, the state is the cold start bit for bit, and the estimate
    lies within a few standard errors of the exact gain."""
    p = M.init_params(3)
    p[1248] = 1.0e3
    net = W.Network(params=p)
    inst = I.planted_partition(600, 4, 0.1, 0.005, seed=11, gamma=5.0)
    deg = W.degrees(inst)
    edges = int((inst.d == 0).sum())
    assert 24 * (edges + 1024) <= inst.n * (inst.n - 1) // 2   # the estimate runs
    for prec in ("f32", "f64"):
        s = C.Solver.from_instance(inst, b=16, prec=prec)
        s.sweep(2)
        s.ctx.set_gate_sample(1024)
        info = W.warm_start(s, net, deg)
        print(prec, info, flush=True)
        assert info["sample_drawn"] == edges + 1024
        assert info["sample_rejected"] and not info["accepted"]
        cold = C.Solver.from_instance(inst, b=16, prec=prec)
        for a in ("x", "f", "y", "y_pair"):
            assert torch.equal(getattr(s, a), getattr(cold, a)), a
        e = C.Solver.from_instance(inst, b=16, prec=prec)
        e.ctx.set_gate_sample(0)
        exact = W.warm_start(e, net, deg)
        assert exact["sample_drawn"] == 0 and not exact["accepted"]
        assert exact["dual_cold"] == info["dual_cold"] and exact["dual_bound"] == info["dual_bound"]
        est, se = info["sample_gain"], info["sample_std_error"]
        true_gain = exact["dual_warm"] - exact["dual_cold"]
        assert info["dual_warm"] == info["dual_cold"] + est
        assert abs(est - true_gain) <= 5.0 * se, (est, se, true_gain)


def test_sampled_gate_keeps_a_good_start():
    """The trained network on a graph of its family (100-node blocks, the
    training graphs' densities): the estimate does not reject, and the exact
    gate's start is the same, bit for bit, as with the estimate turned off."""
    inst = I.planted_partition(1000, 10, 0.25, 0.01, seed=12, gamma=5.0)
    net, deg = W.load(), W.degrees(inst)
    edges = int((inst.d == 0).sum())
    assert 24 * (edges + 1024) <= inst.n * (inst.n - 1) // 2
    states = []
    for count in (1024, 0):
        s = C.Solver.from_instance(inst, b=16, prec="f32")
        s.ctx.set_gate_sample(count)
        info = W.warm_start(s, net, deg)
        print(count, info, flush=True)
        assert info["accepted"] and not info["sample_rejected"]
        assert info["sample_drawn"] == (edges + count if count else 0)
        states.append(s)
    for a in ("x", "f", "y", "y_pair"):
        assert torch.equal(getattr(states[0], a), getattr(states[1], a)), a


def test_gate_terms_edge_cases():
    """An index outside [0, N_p) gives NaN and leaves its neighbours' values
    alone; no pairs is a no-op; n = 3 has one pair per side of its triplet."""
    inst = I.random_signed(3, seed=2, gamma=2.0)
    net, deg = W.load(), W.degrees(inst)
    s = C.Solver.from_instance(inst, b=8, prec="f64")
    aty, delta = W.gate_terms(s, net, deg, torch.tensor([-1, 3, 0, 1, 2]))
    aty, delta = aty.cpu().numpy(), delta.cpu().numpy()
    assert np.isnan(aty[:2]).all() and np.isnan(delta[:2]).all()
    assert np.isfinite(aty[2:]).all() and np.isfinite(delta[2:]).all()
    ref = oracle.gate_pair_terms(3, inst.gamma, inst.w, inst.d, _oracle_predictions(inst, net.host_params()))
    scale = max(1e-30, np.abs(ref["aty"]).max())
    assert np.abs(aty[2:] - ref["aty"]).max() <= 1e-2 * scale
    e, _ = W.gate_terms(s, net, deg, torch.zeros(0, dtype=torch.int64))
    assert e.numel() == 0


def test_one_shot_solve_with_the_warm_start():
    """cc_solve_cc_lp with CC_WARM_MLP, both branches of the gate.
    The shipped network on a held-out graph of its family is kept (FP32):
    fewer sweeps to 1e-4 than the cold start and the same objective.  A
    network with a huge output bias at n = 1200 is rejected by the estimate
    (FP64; at the default 16,384 draws the estimate runs from n of about 1100
    on a graph this sparse): the solve is the cold one, bit for bit."""
    inst = I.training_graph(2002)
    net = W.load()
    params, deg = net.host_params().astype(np.float32), inst.deg.astype(np.float32)
    rc0, x0, _, i0 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-4, b=16,
                                   mode=C.CC_MODE_F32)
    rc1, x1, _, i1 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-4, b=16,
                                   mode=C.CC_MODE_F32, mlp_weights=params, deg=deg)
    print("kept:", i0["sweeps"], i1["sweeps"], i1["warm_accepted"], i1["warm_sampled"], flush=True)
    assert rc0 == C.CC_OK and rc1 == C.CC_OK
    assert i1["warm_accepted"] == 1 and i1["warm_sampled"] == 0
    assert i1["sweeps"] < i0["sweeps"]
    p0, p1 = i0["resid"]["primal_qp"], i1["resid"]["primal_qp"]
    assert abs(p1 - p0) <= 1e-3 * abs(p0)

    bad = M.init_params(3)
    bad[1248] = 1.0e3
    inst = I.planted_partition(1200, 12, 0.1, 0.002, seed=11, gamma=5.0)
    assert 24 * (int((inst.d == 0).sum()) + 16384) <= inst.n * (inst.n - 1) // 2
    deg = inst.deg.astype(np.float32)
    rc0, x0, _, i0 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-3, b=16,
                                   mode=C.CC_MODE_F64)
    rc1, x1, _, i1 = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-3, b=16,
                                   mode=C.CC_MODE_F64, mlp_weights=bad.astype(np.float32), deg=deg)
    print("rejected:", i0["sweeps"], i1["sweeps"], i1["warm_accepted"], i1["warm_sampled"], flush=True)
    assert rc0 == C.CC_OK and rc1 == C.CC_OK
    assert i1["warm_accepted"] == 0 and i1["warm_sampled"] == 1
    assert i1["sweeps"] == i0["sweeps"]
    assert np.array_equal(x0, x1)


def test_one_shot_warm_start_with_sparse_dual_access():
    """CC_WARM_MLP with CC_MODE_SPARSE: the mask is built from the kept
    start, and the solve is the dense one's, bit for bit (FP32 sweeps to
    1e-5, then FP64 polish to 1e-6)."""
    inst = I.training_graph(2003)
    params = W.load().host_params().astype(np.float32)
    deg = inst.deg.astype(np.float32)
    out = {}
    for flag in (0, C.CC_MODE_SPARSE):
        rc, x, y, info = C.solve_cc_lp(inst.n, inst.w, inst.d, inst.gamma, tol=1e-6, b=16,
                                       mode=C.CC_MODE_F32_POLISH | flag, mlp_weights=params, deg=deg,
                                       want_duals=True)
        assert rc == C.CC_OK and info["warm_accepted"] == 1
        out[flag] = (x, y, info["sweeps"], info["sweeps_f32"])
    print("sweeps", out[0][2:], out[C.CC_MODE_SPARSE][2:], flush=True)
    assert out[0][2:] == out[C.CC_MODE_SPARSE][2:]
    assert np.array_equal(out[0][0], out[C.CC_MODE_SPARSE][0])
    assert np.array_equal(out[0][1], out[C.CC_MODE_SPARSE][1])
