"""Seeded synthetic correlation-clustering instances.

This module only draws random graphs and turns them into the arrays both
solvers consume; it holds none of the projection method's arithmetic.

An instance is a signed, weighted complete graph on n nodes (Sec. II-A):
every pair p = (i, j), i < j, carries a label d_p in {0, 1} (1 for a negative
edge, 0 for a positive one, as in the metric-nearness form (mn1)) and a weight
w_p > 0.  Pairs are stored in packed upper-triangular column-major order,
p(i, j) = j (j - 1) / 2 + i for 0-based i < j, so column j of the distance
matrix is contiguous.

The paper builds its instances from five public graphs with a Jaccard-index
transform (Sec. IV-B); neither the graphs nor the transform constants are
available, so sparse unsigned random graphs stand in: an edge of the unsigned
graph becomes a positive pair, a non-edge a negative pair, which gives every
pair a nonzero weight and a sign, as the paper's construction does.

Randomness: numpy PCG64 ``default_rng(seed)``; one uniform per pair in packed
order decides the edge; weights (when not unit) come from
``default_rng(seed + 1)``, one uniform per pair in packed order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def num_pairs(n: int) -> int:
    return n * (n - 1) // 2


def num_triplets(n: int) -> int:
    return n * (n - 1) * (n - 2) // 6


def pair_index(i, j):
    """Packed column-major upper-triangular index of pair (i, j), i < j."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return j * (j - 1) // 2 + i


def pair_coords(n: int):
    """(i, j) arrays for every pair in packed order."""
    j = np.repeat(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64))
    start = np.repeat(np.cumsum(np.arange(n, dtype=np.int64)) - np.arange(n, dtype=np.int64),
                      np.arange(n, dtype=np.int64))
    i = np.arange(num_pairs(n), dtype=np.int64) - start
    return i, j


@dataclass
class Instance:
    """A signed weighted complete graph in packed pair order."""
    name: str
    n: int
    d: np.ndarray            # uint8 [N_p], 1 = negative pair, 0 = positive pair
    w: np.ndarray            # float64 [N_p], > 0
    deg: np.ndarray          # float64 [n], degree in the unsigned source graph
    gamma: float
    meta: dict = field(default_factory=dict)

    @property
    def num_pairs(self) -> int:
        return num_pairs(self.n)

    @property
    def num_constraints(self) -> int:
        return 3 * num_triplets(self.n)


def _from_edge_prob(name, n, prob_fn, seed, gamma, weights="unit", meta=None):
    rng = np.random.default_rng(seed)
    u = rng.random(num_pairs(n))
    i, j = pair_coords(n)
    pij = prob_fn(i, j)
    edge = u < pij
    d = np.where(edge, 0, 1).astype(np.uint8)
    if weights == "unit":
        w = np.ones(num_pairs(n), dtype=np.float64)
    elif weights == "uniform_0.5_1.5":
        w = np.random.default_rng(seed + 1).uniform(0.5, 1.5, num_pairs(n))
    else:
        raise ValueError(f"unknown weights {weights!r}")
    deg = np.zeros(n, dtype=np.float64)
    np.add.at(deg, i[edge], 1.0)
    np.add.at(deg, j[edge], 1.0)
    m = dict(meta or {})
    m.update(seed=seed, weights=weights, edges=int(edge.sum()),
             mean_degree=float(deg.mean()) if n else 0.0)
    return Instance(name, n, d, w, deg, float(gamma), m)


def erdos_renyi(n: int, p: float, seed: int = 0, gamma: float = 1.0) -> Instance:
    """G(n, p): each pair is an edge independently with probability p."""
    return _from_edge_prob(f"er_n{n}_p{p}", n, lambda i, j: np.full(i.shape, p),
                           seed, gamma, meta=dict(model="er", p=p))


def planted_partition(n: int, blocks: int, p_in: float, p_out: float, seed: int = 0,
                      gamma: float = 5.0) -> Instance:
    """Stochastic block model with `blocks` equal blocks of consecutive nodes."""
    size = n // blocks
    if size * blocks != n:
        raise ValueError("n must be a multiple of blocks")
    lab = np.arange(n) // size
    return _from_edge_prob(f"sbm_n{n}_k{blocks}", n,
                           lambda i, j: np.where(lab[i] == lab[j], p_in, p_out),
                           seed, gamma,
                           meta=dict(model="sbm", blocks=blocks, p_in=p_in, p_out=p_out))


def chung_lu(n: int, exponent: float, mean_degree: float, seed: int = 0,
             gamma: float = 5.0, weights: str = "unit", i0: float = 1.0) -> Instance:
    """Chung-Lu graph with power-law expected degrees.

    Expected weight of node v is proportional to (v + i0)^(-1/(exponent-1)),
    scaled so the weights sum to n * mean_degree; p_ij = min(1, w_i w_j / sum w).
    """
    v = np.arange(n, dtype=np.float64)
    ew = (v + i0) ** (-1.0 / (exponent - 1.0))
    ew *= n * mean_degree / ew.sum()
    tot = ew.sum()
    return _from_edge_prob(f"chunglu_n{n}_b{exponent}", n,
                           lambda i, j: np.minimum(1.0, ew[i] * ew[j] / tot),
                           seed, gamma, weights=weights,
                           meta=dict(model="chung_lu", exponent=exponent,
                                     target_mean_degree=mean_degree, i0=i0))


def disjoint_cliques(sizes, gamma: float = 1.0) -> Instance:
    """Positive pairs inside cliques, negative pairs between them, unit weights."""
    lab = np.repeat(np.arange(len(sizes)), sizes)
    n = int(lab.size)
    i, j = pair_coords(n)
    d = np.where(lab[i] == lab[j], 0, 1).astype(np.uint8)
    deg = np.array([sizes[c] - 1 for c in lab], dtype=np.float64)
    return Instance(f"cliques_{'_'.join(map(str, sizes))}", n, d,
                    np.ones(num_pairs(n)), deg, float(gamma), dict(model="cliques"))


def random_signed(n: int, seed: int = 0, gamma: float = 1.0, weighted: bool = True,
                  p_neg: float = 0.5) -> Instance:
    """Small test instance: random signs, optionally random weights in [0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    d = (rng.random(num_pairs(n)) < p_neg).astype(np.uint8)
    w = rng.uniform(0.5, 1.5, num_pairs(n)) if weighted else np.ones(num_pairs(n))
    i, j = pair_coords(n)
    deg = np.zeros(n)
    np.add.at(deg, i[d == 0], 1.0)
    np.add.at(deg, j[d == 0], 1.0)
    return Instance(f"rand_n{n}_s{seed}", n, d, w, deg, float(gamma), dict(model="random"))


@dataclass
class NearnessInstance:
    """Dissimilarities for the l2 metric nearness problem, in packed pair order."""
    name: str
    n: int
    dv: np.ndarray           # float64 [N_p], dissimilarity d_p
    w: np.ndarray            # float64 [N_p], > 0
    meta: dict = field(default_factory=dict)


def noisy_distances(n: int, seed: int = 0, dim: int = 2, noise: float = 0.5,
                    weighted: bool = True) -> NearnessInstance:
    """Euclidean distances of n uniform points in the unit cube of dimension
    `dim`, each multiplied by an independent factor U[1 - noise, 1 + noise]
    (which breaks triangle inequalities), weights U[0.5, 1.5] or 1.
    noise = 0 gives a metric."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, dim))
    i, j = pair_coords(n)
    base = np.sqrt(((pts[i] - pts[j]) ** 2).sum(axis=1))
    dv = base * rng.uniform(1.0 - noise, 1.0 + noise, base.shape)
    w = rng.uniform(0.5, 1.5, base.shape) if weighted else np.ones(base.shape)
    return NearnessInstance(f"noisy_euclid_n{n}_d{dim}_s{seed}", n, dv, w,
                            dict(model="noisy_euclidean", dim=dim, noise=noise, seed=seed))


# The five benchmark workloads: sizes, models and parameters of the headline runs.
def workload(idx: int) -> Instance:
    if idx == 0:
        return erdos_renyi(60, 0.1, seed=0, gamma=1.0)
    if idx == 1:
        return planted_partition(500, 10, 0.3, 0.02, seed=0, gamma=5.0)
    if idx == 2:
        return chung_lu(1500, 2.5, 10.0, seed=0, gamma=5.0)
    if idx == 3:
        return planted_partition(2000, 20, 0.25, 0.01, seed=0, gamma=5.0)
    if idx == 4:
        return chung_lu(4000, 2.2, 20.0, seed=0, gamma=10.0, weights="uniform_0.5_1.5")
    raise ValueError(idx)


TRAINING_FAMILIES = ("sbm300", "chunglu300")


def training_graph(seed: int, family: str = "sbm300") -> Instance:
    """Warm-start training instance.

    sbm300: n=300, 3 blocks of 100, p_in=0.25, p_out=0.01, unit weights,
    gamma=5 (the n=2000 planted partition's densities).
    chunglu300: n=300 Chung-Lu, exponent 2.2, mean degree 20, weights
    U[0.5, 1.5], gamma=10 (the n=4000 Chung-Lu workload's shape)."""
    if family == "sbm300":
        return planted_partition(300, 3, 0.25, 0.01, seed=seed, gamma=5.0)
    if family == "chunglu300":
        return chung_lu(300, 2.2, 20.0, seed=seed, gamma=10.0, weights="uniform_0.5_1.5")
    raise ValueError(family)
