"""Pins of the float64 reference of the warm-start network (CPU)."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M


def test_bf16_rounding_matches_torch_and_ties():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 1000), rng.normal(0, 1e-3, 100), rng.normal(0, 1e4, 100),
                        [0.0, -0.0, 1.0, np.pi, 1e-40]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(v), ref)
    # ties go to the even mantissa
    assert M.bf16(1 + 2.0 ** -8) == 1.0
    assert M.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert M.bf16(1 + 2.0 ** -9) == 1.0


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(3).astype(np.float64)
    phi = rng.normal(0, 1, (40, 4))
    t = np.maximum(rng.normal(0.3, 0.5, 40), 0)
    _, g = M.loss_and_grad(p, phi, t, round=False)
    h = 1e-6
    for idx in rng.choice(M.NPARAM, 60, replace=False).tolist() + [M.NPARAM - 1, 0, 160]:
        e = np.zeros(M.NPARAM)
        e[idx] = h
        fd = (M.loss_and_grad(p + e, phi, t, round=False)[0]
              - M.loss_and_grad(p - e, phi, t, round=False)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_rounded_gradient_close_to_exact():
    rng = np.random.default_rng(2)
    p = M.init_params(4).astype(np.float64)
    phi = rng.normal(0, 1, (200, 4))
    t = np.maximum(rng.normal(0.3, 0.5, 200), 0)
    l0, g0 = M.loss_and_grad(p, phi, t, round=False)
    l1, g1 = M.loss_and_grad(p, phi, t, round=True)
    assert abs(l1 - l0) < 0.05 * abs(l0)
    assert np.abs(g1 - g0).max() < 0.05 * np.abs(g0).max()


def test_features_hand_example():
    # pairs (0,1), (0,2), (1,2): positive, positive, negative; weights 1, 2, 3
    d = np.array([0, 0, 1], np.uint8)
    w = np.array([1.0, 2.0, 3.0])
    deg = np.array([1.0, 1.0, 0.0])                      # mean 2/3
    f = M.features(d, w, deg, [0, 0, 0], [1, 1, 1], [2, 2, 2], [0, 1, 2])
    # o=0: long (0,1), sides (0,2), (1,2); o=1: long (0,2), sides (0,1), (1,2);
    # o=2: long (1,2), sides (0,1), (0,2)
    np.testing.assert_allclose(f[0], [1, 2, -3, (1 + 1) / (2 * 2 / 3)])
    np.testing.assert_allclose(f[1], [2, 1, -3, (1 + 0) / (2 * 2 / 3)])
    np.testing.assert_allclose(f[2], [-3, 1, 2, (1 + 0) / (2 * 2 / 3)])


def test_clamped_output_learns_positive_targets_only():
    p = M.init_params(5).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    p2 = M.pack(W1, b1, W2, b2, W3, -1e3)                 # output always clamped at 0
    phi = np.random.default_rng(0).normal(0, 1, (30, 4))
    y, _ = M.forward(p2, phi)
    assert (y == 0).all()
    # zero targets are already fitted: no loss, no gradient
    l0, g0 = M.loss_and_grad(p2, phi, np.zeros(30))
    assert l0 == 0 and not g0.any()
    # positive targets pull the output bias up
    _, g1 = M.loss_and_grad(p2, phi, np.ones(30))
    assert g1[-1] < 0
