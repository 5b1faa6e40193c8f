"""Serial FP64 CPU oracle for the regularised correlation-clustering LP.

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check and time the GPU library; the GPU library
never loads it and it never loads the GPU library.  The arithmetic lives in
``ccoracle.c`` (Algorithm 1 of Sec. II-B, one row at a time as dual
coordinate ascent, in the tiled schedule order of Sec. III); this file only
marshals numpy arrays, plus a float64 reference of the warm-start network in
``mlp_ref``.

Layouts: pairs packed column-major, p(i, j) = j (j - 1) / 2 + i; metric duals
in colex triplet order y[3 t + o], t = C(k,3) + C(j,2) + i; pair duals
y_pair[2 p + c].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccoracle.c")
_LIB = os.environ.get("CCORACLE_LIB") or os.path.join(_HERE, "libccoracle.so")

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Resid(ctypes.Structure):
    _fields_ = [(k, _dbl) for k in ("max_viol_metric", "max_viol_pair", "primal_qp",
                                     "dual_qp", "gap", "lp_cost", "cs_max", "stat_resid")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NResid(ctypes.Structure):
    _fields_ = [(k, _dbl) for k in ("max_viol", "primal", "dual", "gap", "cs_max", "stat_resid")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("CCORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_schedule.argtypes = [_i64, _i64, _p, _i64]
        L.orc_schedule.restype = _i64
        L.orc_colour_order.argtypes = [_i64, _p, _i64]
        L.orc_colour_order.restype = _i64
        L.orc_sweeps_list.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p, _p, _i32, _p, _i64]
        L.orc_sweeps_list.restype = ctypes.c_int
        L.orc_init_cold.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p]
        L.orc_init_cold.restype = None
        L.orc_sweeps.argtypes = [_i64, _i64, _dbl, _p, _p, _p, _p, _p, _p, _i32, _i32]
        L.orc_sweeps.restype = ctypes.c_int
        L.orc_pair_pass.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p]
        L.orc_pair_pass.restype = ctypes.c_int
        L.orc_round_prefix.argtypes = [_i64, _i64, _dbl, _p, _p, _i64, _p, _p, _p, _i64]
        L.orc_round_prefix.restype = _i64
        L.orc_x_from_y.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p]
        L.orc_x_from_y.restype = ctypes.c_int
        L.orc_residuals.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p, _p, ctypes.POINTER(Resid)]
        L.orc_residuals.restype = ctypes.c_int
        L.orc_l1_sweeps.argtypes = [_i64, _i64, _dbl, _p, _p, _p, _p, _p, _p, _i32, _i32]
        L.orc_l1_sweeps.restype = ctypes.c_int
        L.orc_l1_residuals.argtypes = [_i64, _dbl, _p, _p, _p, _p, _p, _p, ctypes.POINTER(Resid)]
        L.orc_l1_residuals.restype = ctypes.c_int
        L.orc_dual_objective.argtypes = [_i64, _dbl, _p, _p, _p, _p]
        L.orc_dual_objective.restype = _dbl
        L.orc_nearness_init.argtypes = [_i64, _p, _p, _p]
        L.orc_nearness_init.restype = None
        L.orc_nearness_sweeps.argtypes = [_i64, _i64, _p, _p, _p, _i32, _i32]
        L.orc_nearness_sweeps.restype = ctypes.c_int
        L.orc_nearness_residuals.argtypes = [_i64, _p, _p, _p, _p, ctypes.POINTER(NResid)]
        L.orc_nearness_residuals.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# visiting orders of the metric rows: the tiled schedule (Sec. III-B/C),
# plain lexicographic order, the sum-mod-n colouring
ORDERS = {"schedule": 0, "lex": 1, "colour": 2}


def _order(order):
    if order not in ORDERS:
        raise ValueError(f"unknown order {order!r}")
    return ORDERS[order]


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def num_pairs(n):
    return n * (n - 1) // 2


def num_triplets(n):
    return n * (n - 1) * (n - 2) // 6


class State:
    """Oracle iterate: x, f (per pair), y (colex metric duals), y_pair."""

    def __init__(self, n, gamma, w, d, dense_duals=True):
        self.n = int(n)
        self.gamma = float(gamma)
        self.w = _f64(w)
        self.d = np.ascontiguousarray(d, dtype=np.uint8)
        npairs = num_pairs(self.n)
        assert self.w.shape == (npairs,) and self.d.shape == (npairs,)
        self.x = np.zeros(npairs)
        self.f = np.zeros(npairs)
        self.y = np.zeros(3 * num_triplets(self.n)) if dense_duals else None
        self.y_pair = np.zeros(2 * npairs)
        self.sweeps = 0
        self.init_cold()

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.n, inst.gamma, inst.w, inst.d, **kw)

    def init_cold(self):
        lib().orc_init_cold(self.n, self.gamma, _ptr(self.w), _ptr(self.x), _ptr(self.f),
                            _ptr(self.y), _ptr(self.y_pair))
        self.sweeps = 0

    def sweep(self, nsweeps=1, b=8, order="schedule"):
        assert self.y is not None
        rc = lib().orc_sweeps(self.n, int(b), self.gamma, _ptr(self.w), _ptr(self.d),
                              _ptr(self.x), _ptr(self.f), _ptr(self.y), _ptr(self.y_pair),
                              int(nsweeps), _order(order))
        if rc != 0:
            raise ValueError("oracle sweep rejected its input")
        self.sweeps += nsweeps

    def sweep_list(self, triplets, nsweeps=1):
        """Sweeps that visit the given (i, j, k) rows in the given order."""
        tr = np.ascontiguousarray(triplets, dtype=np.int64).reshape(-1, 3)
        rc = lib().orc_sweeps_list(self.n, self.gamma, _ptr(self.w), _ptr(self.d), _ptr(self.x),
                                   _ptr(self.f), _ptr(self.y), _ptr(self.y_pair), int(nsweeps),
                                   _ptr(tr), tr.shape[0])
        if rc != 0:
            raise ValueError("oracle sweep rejected its input")
        self.sweeps += nsweeps

    def residuals(self) -> dict:
        out = Resid()
        rc = lib().orc_residuals(self.n, self.gamma, _ptr(self.w), _ptr(self.d),
                                 _ptr(self.x), _ptr(self.f), _ptr(self.y),
                                 _ptr(self.y_pair), ctypes.byref(out))
        if rc != 0:
            raise MemoryError
        return out.as_dict()

    def dual_objective(self) -> float:
        return lib().orc_dual_objective(self.n, self.gamma, _ptr(self.w), _ptr(self.d),
                                        _ptr(self.y), _ptr(self.y_pair))

    def x_from_y(self):
        x = np.zeros_like(self.x)
        f = np.zeros_like(self.f)
        lib().orc_x_from_y(self.n, self.gamma, _ptr(self.w), _ptr(self.y),
                           _ptr(self.y_pair), _ptr(x), _ptr(f))
        return x, f

    def solve(self, tol=1e-6, b=8, max_sweeps=100000, check_every=1, order="schedule",
              gap_tol=None):
        """Sweep until the max constraint violation is at most tol and, with
        gap_tol, the duality gap is at most gap_tol * max(1, |primal|)
        (Sec. IV-D stops on constraint satisfaction and the gap)."""
        while self.sweeps < max_sweeps:
            self.sweep(check_every, b=b, order=order)
            r = self.residuals()
            if max(r["max_viol_metric"], r["max_viol_pair"]) <= tol and (
                    gap_tol is None or abs(r["gap"]) <= gap_tol * max(1.0, abs(r["primal_qp"]))):
                return r
        return self.residuals()


def schedule(n: int, b: int) -> np.ndarray:
    """Visiting order as rows (i, j, k, round, P, J, t)."""
    cnt = num_triplets(n)
    out = np.zeros((max(cnt, 1), 7), dtype=np.int64)
    got = lib().orc_schedule(n, b, _ptr(out), cnt)
    assert got == cnt, (got, cnt)
    return out[:cnt]


class L1Nearness(State):
    """Oracle iterate of the l1 metric nearness problem: (mn1) with real
    dissimilarities dv (Sec. II-A: min sum w |x - d| over metric x), solved
    as (qp) by Algorithm 1 exactly as correlation clustering, whose d is
    0/1.  x, f per pair; y colex metric duals; y_pair per pair row."""

    def __init__(self, n, gamma, w, dv):
        self.dv = _f64(dv)
        super().__init__(n, gamma, w, np.zeros(num_pairs(int(n)), dtype=np.uint8))
        assert self.dv.shape == self.w.shape

    def sweep(self, nsweeps=1, b=8, order="schedule"):
        rc = lib().orc_l1_sweeps(self.n, int(b), self.gamma, _ptr(self.w), _ptr(self.dv),
                                 _ptr(self.x), _ptr(self.f), _ptr(self.y), _ptr(self.y_pair),
                                 int(nsweeps), _order(order))
        if rc != 0:
            raise ValueError("oracle sweep rejected its input")
        self.sweeps += nsweeps

    def residuals(self) -> dict:
        out = Resid()
        rc = lib().orc_l1_residuals(self.n, self.gamma, _ptr(self.w), _ptr(self.dv), _ptr(self.x),
                                    _ptr(self.f), _ptr(self.y), _ptr(self.y_pair),
                                    ctypes.byref(out))
        if rc != 0:
            raise MemoryError
        return out.as_dict()

    def sweep_list(self, triplets, nsweeps=1):
        raise NotImplementedError("explicit visit lists are offered for 0/1 d only")

    def dual_objective(self) -> float:
        return self.residuals()["dual_qp"]


def colour_order(n: int) -> np.ndarray:
    """The sum-mod-n colouring's visiting order as rows (i, j, k, colour)."""
    cnt = num_triplets(n)
    out = np.zeros((max(cnt, 1), 7), dtype=np.int64)
    got = lib().orc_colour_order(n, _ptr(out), cnt)
    assert got == cnt, (got, cnt)
    return out[:cnt, :4]


def pair_pass(n, gamma, w, d, x, f, y_pair):
    """One pass over the pair constraints, in place."""
    w, d = _f64(w), np.ascontiguousarray(d, dtype=np.uint8)   # alive through the call
    rc = lib().orc_pair_pass(int(n), float(gamma), _ptr(w), _ptr(d),
                             _ptr(x), _ptr(f), _ptr(y_pair))
    if rc != 0:
        raise MemoryError


def colex_triplets(n):
    """(i, j, k) of every triplet i < j < k in colex order (arrays)."""
    n = int(n)
    parts = [(np.arange(j), np.full(j, j), np.full(j, k)) for k in range(2, n) for j in range(1, k)]
    if not parts:
        z = np.zeros(0, dtype=np.int64)
        return z, z, z
    return tuple(np.concatenate([q[e] for q in parts]).astype(np.int64) for e in range(3))


def gate_pair_terms(n, gamma, w, d, y):
    """Per-pair terms of the warm-start gate for the metric duals y (colex
    order, three rows per triplet: long side ij, ik, jk).

    A start takes x = x(y) with zero pair duals (Algorithm 1's primal point
    of a dual vector, Sec. II-B), then one pass over the pair rows.  With
    b = 0 on every metric row and W diagonal, the dual of (qp) is then a sum
    of one term per pair p:
        -d_p (y1 - y2) - (gamma / 2) ((A'y)_p + y1 - y2)^2 + (w_p - y1 - y2)^2) / w_p,
    (A'y)_p being the metric rows' part: +1 for a row whose long side is p,
    -1 for a row where p is one of the two short sides.  Returns per-pair
    arrays: aty (that part, from its definition), term_warm (the start from
    y), term_cold (the start from y = 0), and the pair duals of both starts
    after their pass."""
    n = int(n)
    w = _f64(w)
    d = np.ascontiguousarray(d, dtype=np.uint8)
    npairs = num_pairs(n)
    yv = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    assert yv.shape[0] == num_triplets(n)
    i, j, k = colex_triplets(n)
    pij, pik, pjk = j * (j - 1) // 2 + i, k * (k - 1) // 2 + i, k * (k - 1) // 2 + j
    aty = np.zeros(npairs)
    np.add.at(aty, pij, yv[:, 0] - yv[:, 1] - yv[:, 2])
    np.add.at(aty, pik, yv[:, 1] - yv[:, 0] - yv[:, 2])
    np.add.at(aty, pjk, yv[:, 2] - yv[:, 0] - yv[:, 1])
    dv = d.astype(np.float64)
    out = {"aty": aty}
    for name, ax in (("warm", aty), ("cold", np.zeros(npairs))):
        s = State(n, gamma, w, d, dense_duals=False)   # the cold start
        if name == "warm":
            s.y = np.ascontiguousarray(yv.ravel())
            s.x, s.f = s.x_from_y()
        pair_pass(n, gamma, w, d, s.x, s.f, s.y_pair)
        y1, y2 = s.y_pair[0::2], s.y_pair[1::2]
        out["term_" + name] = -(dv * y1 - dv * y2) - 0.5 * float(gamma) * (
            (ax + y1 - y2) ** 2 + (w - y1 - y2) ** 2) / w
        out["y_pair_" + name] = s.y_pair.copy()
    return out


def second_sweep_prefix(n, b, gamma, w, d, rounds, cap=None):
    """Cold start, one pair pass, then the first `rounds` metric rounds.

    This is the state after sweep 1 plus a prefix of sweep 2 (a cold-start
    sweep changes no metric dual), without dense dual storage.  Returns
    (x, f, y_pair, t, o, y) with the nonzero metric duals in visit order.
    """
    w = _f64(w)
    npairs = num_pairs(n)
    x0 = np.zeros(npairs)
    f = np.full(npairs, -float(gamma))
    y_pair = np.zeros(2 * npairs)
    pair_pass(n, gamma, w, d, x0, f, y_pair)
    if cap is None:
        cap = 1 << 20
    while True:
        x = x0.copy()
        t = np.zeros(cap, dtype=np.int64)
        o = np.zeros(cap, dtype=np.int8)
        y = np.zeros(cap)
        cnt = lib().orc_round_prefix(n, b, float(gamma), _ptr(w), _ptr(x), int(rounds),
                                     _ptr(t), _ptr(o), _ptr(y), cap)
        if cnt < 0:
            raise MemoryError
        if cnt <= cap:
            return x, f, y_pair, t[:cnt], o[:cnt], y[:cnt]
        cap = int(cnt)


class Nearness:
    """Oracle iterate of the l2 metric nearness problem (Sec. II-A, p = 2):
    min (1/2) sum_p w_p (x_p - d_p)^2 over metric x, for real dissimilarities
    d.  x per pair, y colex metric duals; Algorithm 1 from x = d, y = 0."""

    def __init__(self, n, w, dv):
        self.n = int(n)
        self.w = _f64(w)
        self.dv = _f64(dv)
        npairs = num_pairs(self.n)
        assert self.w.shape == (npairs,) and self.dv.shape == (npairs,)
        self.x = np.zeros(npairs)
        self.y = np.zeros(3 * num_triplets(self.n))
        self.sweeps = 0
        self.init()

    def init(self):
        lib().orc_nearness_init(self.n, _ptr(self.dv), _ptr(self.x), _ptr(self.y))
        self.sweeps = 0

    def sweep(self, nsweeps=1, b=8, order="schedule"):
        rc = lib().orc_nearness_sweeps(self.n, int(b), _ptr(self.w), _ptr(self.x), _ptr(self.y),
                                       int(nsweeps), _order(order))
        if rc != 0:
            raise ValueError("oracle sweep rejected its input")
        self.sweeps += nsweeps

    def residuals(self) -> dict:
        out = NResid()
        rc = lib().orc_nearness_residuals(self.n, _ptr(self.w), _ptr(self.dv), _ptr(self.x),
                                          _ptr(self.y), ctypes.byref(out))
        if rc != 0:
            raise MemoryError
        return out.as_dict()

    def solve(self, tol=1e-6, b=8, max_sweeps=100000, order="schedule", gap_tol=None):
        """Sweep until the max metric violation is at most tol and, with
        gap_tol, the primal-dual gap is at most gap_tol * max(1, |primal|).
        (The iterate can be feasible well before it is optimal.)"""
        while self.sweeps < max_sweeps:
            self.sweep(1, b=b, order=order)
            r = self.residuals()
            if r["max_viol"] <= tol and (gap_tol is None or
                                         abs(r["gap"]) <= gap_tol * max(1.0, abs(r["primal"]))):
                return r
        return self.residuals()
