"""Pins of the oracle's other visiting orders (Sec. IV-E: the order changes
the iteration count, not the limit), in particular the sum-mod-n colouring
of the triplets (the colouring view in the related-work section: triplets
that share a pair conflict).  CPU only."""
import itertools

import numpy as np
import pytest

import oracle
from oracle_helpers import qp_bruteforce
from paper_1901_10084_amd import instances as I


def brute_colour_order(n):
    """Every triplet i<j<k<n, ordered by colour (i+j+k) mod n and then by
    (i, j): written from the definition, independently of the oracle."""
    rows = [(i, j, k, (i + j + k) % n) for i, j, k in itertools.combinations(range(n), 3)]
    rows.sort(key=lambda r: (r[3], r[0], r[1]))
    return np.array(rows, dtype=np.int64).reshape(-1, 4)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 11, 16])
def test_colour_order_is_the_definition(n):
    assert np.array_equal(oracle.colour_order(n), brute_colour_order(n))


@pytest.mark.parametrize("n", [3, 6, 9, 14, 23])
def test_colour_classes_are_conflict_free_and_cover_once(n):
    o = oracle.colour_order(n)
    assert len({tuple(r[:3]) for r in o}) == len(o) == n * (n - 1) * (n - 2) // 6
    for t in range(n):
        pairs = []
        for i, j, k, _ in o[o[:, 3] == t]:
            pairs += [(i, j), (i, k), (j, k)]
        assert len(pairs) == len(set(pairs)), f"colour {t} has triplets sharing a pair"


def test_shuffling_inside_colours_changes_nothing_and_across_colours_does():
    """Triplets of one colour share no pair, so their order inside the colour
    cannot change a single bit; a shuffle across colours reorders conflicting
    triplets and changes the iterate (the test can tell the two apart)."""
    inst = I.random_signed(13, seed=5, gamma=2.0)
    rng = np.random.default_rng(0)
    order = oracle.colour_order(inst.n)
    inside = np.concatenate([rng.permutation(order[order[:, 3] == t]) for t in range(inst.n)])
    across = rng.permutation(order)

    def run(rows, how):
        s = oracle.State.from_instance(inst)
        if how == "colour":
            s.sweep(4, order="colour")
        else:
            s.sweep_list(rows[:, :3], 4)
        return s

    ref = run(None, "colour")
    same = run(inside, "list")
    other = run(across, "list")
    for a in ("x", "f", "y", "y_pair"):
        assert np.array_equal(getattr(ref, a), getattr(same, a)), a
    assert not np.array_equal(ref.x, other.x)


@pytest.mark.parametrize("n,seed,gamma", [(5, 1, 2.0), (6, 2, 0.7), (7, 3, 5.0)])
def test_colour_order_reaches_the_qp_optimum(n, seed, gamma):
    inst = I.random_signed(n, seed=seed, gamma=gamma, weighted=True)
    s = oracle.State.from_instance(inst)
    s.solve(tol=1e-13, max_sweeps=200000, order="colour")
    v = qp_bruteforce(n, inst.w, inst.d, gamma)
    np.testing.assert_allclose(s.x, v[:len(inst.w)], atol=1e-9)
    np.testing.assert_allclose(s.f, v[len(inst.w):], atol=1e-9)


def test_orders_share_the_limit_but_not_the_path():
    """Schedule, lexicographic and colour orders converge to the same point
    (the QP optimum is unique) along different iterates."""
    inst = I.workload(0)
    xs = {}
    after3 = {}
    for order in ("schedule", "lex", "colour"):
        s = oracle.State.from_instance(inst)
        s.sweep(3, b=8, order=order)
        after3[order] = s.x.copy()
        s.solve(tol=1e-11, b=8, max_sweeps=20000, order=order)
        xs[order] = s.x
    for order in ("lex", "colour"):
        np.testing.assert_allclose(xs[order], xs["schedule"], atol=1e-8)
        assert not np.array_equal(after3[order], after3["schedule"])


def test_nearness_colour_order_matches_the_other_orders():
    inst = I.noisy_distances(12, seed=3, noise=0.6)
    ref = oracle.Nearness(inst.n, inst.w, inst.dv)
    ref.solve(tol=1e-12, b=4, max_sweeps=200000, gap_tol=1e-12)
    s = oracle.Nearness(inst.n, inst.w, inst.dv)
    s.solve(tol=1e-12, max_sweeps=200000, order="colour", gap_tol=1e-12)
    np.testing.assert_allclose(s.x, ref.x, atol=1e-9)


def test_unknown_order_is_rejected():
    inst = I.workload(0)
    s = oracle.State.from_instance(inst)
    with pytest.raises(ValueError):
        s.sweep(1, order="random")
