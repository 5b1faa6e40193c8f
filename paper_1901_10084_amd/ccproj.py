"""ctypes binding of ``libccproj.so`` (the C ABI in ``include/ccproj.h``).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the
library is missing this module raises at import time; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CCPROJ_LIB") or os.path.join(_HERE, "libccproj.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1901_10084_amd/build.py")

_L = ctypes.CDLL(LIB_PATH)

CC_OK, CC_ENOTCONV = 0, 1
CC_EINVAL, CC_ENOMEM, CC_EHIP, CC_ENONFINITE = -1, -2, -3, -4
CC_F64, CC_F32 = 0, 1
CC_MODE_F64, CC_MODE_F32, CC_MODE_F32_POLISH = 0, 1, 2
CC_MODE_SPARSE = 16  # flag or-ed into a mode: sparse dual access
CC_WARM_NONE, CC_WARM_MLP = 0, 1
CC_EXEC_ROUNDS, CC_EXEC_DATAFLOW = 0, 1
CC_RESID_VIOL, CC_RESID_CS, CC_RESID_DUAL, CC_RESID_ALL = 1, 2, 4, 7

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


class Resid(ctypes.Structure):
    _fields_ = [(k, _dbl) for k in ("max_viol_metric", "max_viol_pair", "primal_qp",
                                     "dual_qp", "gap", "lp_cost", "cs_max", "stat_resid")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NResid(ctypes.Structure):
    _fields_ = [(k, _dbl) for k in ("max_viol", "primal", "dual", "gap", "cs_max", "stat_resid")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("sweeps", _i32), ("sweeps_f32", _i32), ("warm_accepted", _i32),
                ("warm_sampled", _i32), ("wall_s", _dbl), ("resid", Resid)]


def _sig(name, res, *args):
    fn = getattr(_L, name)
    fn.restype = res
    fn.argtypes = list(args)
    return fn


_sig("cc_last_error", ctypes.c_char_p)
_sig("cc_num_metric_duals", _i64, _i64)
_sig("cc_create", ctypes.c_int, ctypes.POINTER(_p), _i64, _i32, _i32, _p)
_sig("cc_destroy", ctypes.c_int, _p)
_sig("cc_dual_slots", _i64, _p)
_sig("cc_num_rounds", _i32, _p)
_sig("cc_prepare", ctypes.c_int, _p, _p, _dbl, _p)
_sig("cc_init_cold", ctypes.c_int, _p, _p, _p, _p, _p, _dbl)
_sig("cc_sweep", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _i32, _i32)
_sig("cc_sweep_rounds", ctypes.c_int, _p, _p, _p, _p, _i32, _i32)
_sig("cc_sweep_metric_prefix", ctypes.c_int, _p, _p, _p, _p, _i32)
_sig("cc_sweep_noalloc", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _i32)
_sig("cc_sweep_metric", ctypes.c_int, _p, _p, _p, _p, _i32)
_sig("cc_status", ctypes.c_int, _p)
_sig("cc_dataflow_breakdown", ctypes.c_int, _p, _p, _p, _p, ctypes.POINTER(_dbl))
_sig("cc_set_dataflow_workgroups", ctypes.c_int, _p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32))
_sig("cc_pair_pass", ctypes.c_int, _p, _p, _p, _p, _p, _p)
_sig("cc_residuals", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _dbl, _i32,
     ctypes.POINTER(Resid))
_sig("cc_x_from_y", ctypes.c_int, _p, _p, _p, _p, _dbl, _p, _p)
_sig("cc_duals_to_lex", ctypes.c_int, _p, _p, _p)
_sig("cc_slots_to_lex", ctypes.c_int, _p, _p, _i64, _p)
_sig("cc_dataflow_tables", ctypes.c_int, _i64, _i32, _p, _p, _p, _p, _p, _p, _p, _p)
_sig("cc_widen", ctypes.c_int, _p, _p, _i64, _p)
_sig("cc_solve_cc_lp", ctypes.c_int, _i64, _p, _p, _dbl, _dbl, _dbl, _i32, _i32, _i32, _i32, _p, _p,
     _p, _p, ctypes.POINTER(Info))
_sig("cc_narrow", ctypes.c_int, _p, _p, _i64, _p)
_sig("cc_nearness_init", ctypes.c_int, _p, _p, _p, _p)
_sig("cc_dual_mask_bytes", _i64, _p)
_sig("cc_dual_mask_build", ctypes.c_int, _p, _p, _p)
_sig("cc_sweep_sparse", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _p, _i32)
_sig("cc_sweep_metric_sparse", ctypes.c_int, _p, _p, _p, _p, _p)
_sig("cc_sweep_colour", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _i32)
_sig("cc_l1_sweep", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _p, _i32)
_sig("cc_compact_init", ctypes.c_int, _p, _i64)
_sig("cc_sweep_compact", ctypes.c_int, _p, _p, _p, _p, _p, _p, _i32)
_sig("cc_compact_to_slots", ctypes.c_int, _p, _p)
_sig("cc_compact_export", ctypes.c_int, _p, _p, _p, _i64, ctypes.POINTER(_i64))
_sig("cc_compact_info", ctypes.c_int, _p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32))
_sig("cc_compact_release", ctypes.c_int, _p)
_sig("cc_l1_residuals", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, _dbl, _i32, ctypes.POINTER(Resid))
_sig("cc_init_cold_lex", ctypes.c_int, _p, _p, _p, _p, _p, _dbl)
_sig("cc_nearness_residuals", ctypes.c_int, _p, _p, _p, _p, _p, _i32, ctypes.POINTER(NResid))

_sig("cc_mlp_num_params", _i32)
_sig("cc_mlp_workspace_bytes", _i64, _i64)
_sig("cc_mlp_init", ctypes.c_int, _p, ctypes.c_uint64)
_sig("cc_mlp_forward", ctypes.c_int, _p, _p, _i64, _p, _p)
_sig("cc_mlp_train_step", ctypes.c_int, _p, _p, _i64, _p, _p, _p, _i32, ctypes.c_float, _p, _p,
     _p, _p)
_sig("cc_mlp_train_graph", ctypes.c_int, _p, _p, _p, _p, _p, _i64, ctypes.c_uint64, _p, _p, _p,
     _i32, ctypes.c_float, _p, _p)
_sig("cc_mlp_slot_features", ctypes.c_int, _p, _p, _p, _p, _p, _i64, _p)
_sig("cc_mlp_infer", ctypes.c_int, _p, _p, _p, _p, _p, _p)
_sig("cc_warm_start_mlp", ctypes.c_int, _p, _p, _p, _p, _p, _dbl, _p, _p, _p, _p, _p,
     ctypes.POINTER(_i32), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl))
_sig("cc_warm_gate_terms", ctypes.c_int, _p, _p, _p, _p, _p, _dbl, _p, _p, _i64, _p, _p)
_sig("cc_set_gate_sample", ctypes.c_int, _p, _i64)
_sig("cc_last_gate_sample", ctypes.c_int, _p, ctypes.POINTER(_i64), ctypes.POINTER(_dbl),
     ctypes.POINTER(_dbl), ctypes.POINTER(_i32))

EXPORTS = ["cc_last_error", "cc_num_metric_duals", "cc_create", "cc_destroy", "cc_dual_slots",
           "cc_num_rounds", "cc_prepare", "cc_init_cold", "cc_sweep", "cc_sweep_rounds",
           "cc_sweep_metric_prefix", "cc_sweep_metric", "cc_sweep_noalloc", "cc_status",
           "cc_pair_pass", "cc_residuals", "cc_x_from_y", "cc_duals_to_lex", "cc_slots_to_lex",
           "cc_dataflow_tables", "cc_widen", "cc_narrow", "cc_solve_cc_lp",
           "cc_nearness_init", "cc_nearness_residuals", "cc_dual_mask_bytes",
           "cc_dual_mask_build", "cc_sweep_sparse", "cc_sweep_metric_sparse", "cc_sweep_colour",
           "cc_init_cold_lex", "cc_l1_sweep", "cc_l1_residuals", "cc_compact_init",
           "cc_sweep_compact", "cc_compact_to_slots", "cc_compact_export", "cc_compact_info",
           "cc_compact_release", "cc_set_dataflow_workgroups", "cc_dataflow_breakdown"]


class CCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccproj error {code}: {msg}")
        self.code = code


def last_error() -> str:
    m = _L.cc_last_error()
    return m.decode() if m else ""


def check(rc: int, allow_notconv: bool = False) -> int:
    if rc < 0 or (rc == CC_ENOTCONV and not allow_notconv):
        raise CCError(rc, last_error())
    return rc


def num_metric_duals(n: int) -> int:
    return int(_L.cc_num_metric_duals(n))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return t.data_ptr()
    return int(t)


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """A schedule context: n nodes, tile size b, precision, stream."""

    def __init__(self, n: int, b: int, prec: str = "f64", stream=None):
        self.n, self.b = int(n), int(b)
        self.prec = prec
        self.dtype = {"f64": torch.float64, "f32": torch.float32}[prec]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _p()
        check(_L.cc_create(ctypes.byref(h), self.n, self.b,
                           CC_F64 if prec == "f64" else CC_F32, _stream_handle(self.stream)))
        self._h = h
        self.slots = int(_L.cc_dual_slots(h))
        self.rounds = int(_L.cc_num_rounds(h))

    @property
    def handle(self):
        return self._h

    def executor(self, executor=None):
        """The given executor, or by default the dataflow executor where it
        exists (b = 8, 16, 24, 32) and the round-by-round one elsewhere."""
        if executor is not None:
            return int(executor)
        return CC_EXEC_DATAFLOW if self.b in (8, 16, 24, 32) else CC_EXEC_ROUNDS

    def close(self):
        if getattr(self, "_h", None):
            _L.cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, w, gamma, g):
        check(_L.cc_prepare(self._h, _ptr(w), float(gamma), _ptr(g)))

    def init_cold(self, x, f, y, y_pair, gamma):
        check(_L.cc_init_cold(self._h, _ptr(x), _ptr(f), _ptr(y), _ptr(y_pair), float(gamma)))

    def sweep(self, x, f, y, y_pair, g, d, nsweeps=1, executor=None):
        check(_L.cc_sweep(self._h, _ptr(x), _ptr(f), _ptr(y), _ptr(y_pair), _ptr(g), _ptr(d),
                          int(nsweeps), self.executor(executor)))

    def sweep_rounds(self, x, y, g, first, count):
        check(_L.cc_sweep_rounds(self._h, _ptr(x), _ptr(y), _ptr(g), int(first), int(count)))

    def sweep_metric_prefix(self, x, y, g, rounds):
        check(_L.cc_sweep_metric_prefix(self._h, _ptr(x), _ptr(y), _ptr(g), int(rounds)))

    def sweep_noalloc(self, x, f, y, y_pair, g, d, nsweeps=1):
        """cc_sweep_noalloc: dataflow sweeps with the library's static
        scratch (no device allocation); synchronises."""
        check(_L.cc_sweep_noalloc(self._h, _ptr(x), _ptr(f), _ptr(y), _ptr(y_pair), _ptr(g),
                                  _ptr(d), int(nsweeps)))

    def sweep_metric(self, x, y, g, executor=None):
        check(_L.cc_sweep_metric(self._h, _ptr(x), _ptr(y), _ptr(g), self.executor(executor)))

    def mask_bytes(self) -> int:
        nbytes = _L.cc_dual_mask_bytes(self._h)
        if nbytes < 0:
            raise CCError(CC_EINVAL, "sparse dual access needs b = 8, 16, 24 or 32")
        return nbytes

    def mask_build(self, y, mask):
        check(_L.cc_dual_mask_build(self._h, _ptr(y), _ptr(mask)))

    def sweep_sparse(self, x, f, y, y_pair, g, d, mask, nsweeps=1):
        check(_L.cc_sweep_sparse(self._h, _ptr(x), _ptr(f), _ptr(y), _ptr(y_pair), _ptr(g),
                                 _ptr(d), _ptr(mask), int(nsweeps)))

    def sweep_metric_sparse(self, x, y, g, mask):
        check(_L.cc_sweep_metric_sparse(self._h, _ptr(x), _ptr(y), _ptr(g), _ptr(mask)))

    def status(self):
        check(_L.cc_status(self._h))

    def set_dataflow_workgroups(self, workgroups=0):
        """Workgroups of the dataflow sweeps (0: the default); returns the
        count used."""
        eff = ctypes.c_int32(0)
        check(_L.cc_set_dataflow_workgroups(self._h, int(workgroups), ctypes.byref(eff)))
        return int(eff.value)

    def set_gate_sample(self, count):
        """Pairs the sampled warm-start gate draws (0: off)."""
        check(_L.cc_set_gate_sample(self._h, int(count)))

    def last_gate_sample(self):
        drawn, rej = _i64(0), _i32(0)
        gain, se = _dbl(0.0), _dbl(0.0)
        check(_L.cc_last_gate_sample(self._h, ctypes.byref(drawn), ctypes.byref(gain),
                                     ctypes.byref(se), ctypes.byref(rej)))
        return {"drawn": int(drawn.value), "gain": gain.value, "std_error": se.value,
                "rejected": bool(rej.value)}

    def dataflow_breakdown(self, x, y, g):
        out = (_dbl * 8)()
        check(_L.cc_dataflow_breakdown(self._h, _ptr(x), _ptr(y), _ptr(g), out))
        keys = ("wait_us", "load_us", "substeps_us", "publish_us", "tile_steps", "workgroups")
        return {k: out[e] for e, k in enumerate(keys)}

    def pair_pass(self, x, f, y_pair, g, d):
        check(_L.cc_pair_pass(self._h, _ptr(x), _ptr(f), _ptr(y_pair), _ptr(g), _ptr(d)))

    def residuals(self, x, f, y, y_pair, w, d, gamma, what=CC_RESID_ALL, raise_nonfinite=True):
        out = Resid()
        rc = _L.cc_residuals(self._h, _ptr(x), _ptr(f), _ptr(y), _ptr(y_pair), _ptr(w), _ptr(d),
                             float(gamma), int(what), ctypes.byref(out))
        if rc == CC_ENONFINITE and not raise_nonfinite:
            r = out.as_dict()
            r["nonfinite"] = True
            return r
        check(rc)
        return out.as_dict()

    def x_from_y(self, y, y_pair, w, gamma, x_out, f_out):
        check(_L.cc_x_from_y(self._h, _ptr(y), _ptr(y_pair), _ptr(w), float(gamma),
                             _ptr(x_out), _ptr(f_out)))

    def duals_to_lex(self, y, y_lex):
        check(_L.cc_duals_to_lex(self._h, _ptr(y), _ptr(y_lex)))

    def slots_to_lex(self, slots, out):
        check(_L.cc_slots_to_lex(self._h, _ptr(slots), int(slots.numel()), _ptr(out)))


def dataflow_tables(n: int, b: int) -> dict:
    """Dependency tables of the dataflow executor (host only, no GPU)."""
    nt, ns, nbk = _i64(), _i64(), _i64()
    check(_L.cc_dataflow_tables(n, b, ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(nbk),
                                None, None, None, None, None))
    pq = np.zeros(2 * nt.value, dtype=np.int32)
    needc = np.zeros(nt.value, dtype=np.uint32)
    jsb = np.zeros(nt.value, dtype=np.int32)
    needs = np.zeros(2 * ns.value, dtype=np.uint32)
    K = np.zeros(nbk.value, dtype=np.uint32)
    check(_L.cc_dataflow_tables(n, b, None, None, None, pq.ctypes.data, needc.ctypes.data,
                                jsb.ctypes.data, needs.ctypes.data, K.ctypes.data))
    return dict(tile_pq=pq.reshape(-1, 2), need_c=needc, jsbase=jsb, needs=needs.reshape(-1, 2),
                K=K)


def solve_cc_lp(n, w, d, gamma, tol=1e-6, max_sweeps=100000, b=16, mode=CC_MODE_F64,
                mlp_weights=None, deg=None, want_duals=False, gap_tol=0.0):
    """One-shot solve from host arrays (cc_solve_cc_lp).  Returns
    (status, x, y_lex or None, info dict)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.uint8)
    x = np.zeros(n * (n - 1) // 2)
    ylex = np.zeros(num_metric_duals(n)) if want_duals else None
    warm = CC_WARM_MLP if mlp_weights is not None else CC_WARM_NONE
    mw = None if mlp_weights is None else np.ascontiguousarray(mlp_weights, dtype=np.float32)
    dg = None if deg is None else np.ascontiguousarray(deg, dtype=np.float32)
    info = Info()
    rc = _L.cc_solve_cc_lp(int(n), w.ctypes.data, d.ctypes.data, float(gamma), float(tol),
                           float(gap_tol), int(max_sweeps), int(b), int(mode), int(warm),
                           None if mw is None else mw.ctypes.data,
                           None if dg is None else dg.ctypes.data, x.ctypes.data,
                           None if ylex is None else ylex.ctypes.data, ctypes.byref(info))
    check(rc, allow_notconv=True)
    out = dict(sweeps=info.sweeps, sweeps_f32=info.sweeps_f32, wall_s=info.wall_s,
               warm_accepted=info.warm_accepted, warm_sampled=info.warm_sampled,
               resid=info.resid.as_dict())
    return rc, x, ylex, out


def widen(src, dst, stream=None):
    check(_L.cc_widen(_ptr(src), _ptr(dst), int(src.numel()), _stream_handle(stream)))


def narrow(src, dst, stream=None):
    check(_L.cc_narrow(_ptr(src), _ptr(dst), int(src.numel()), _stream_handle(stream)))


class Solver:
    """Device state of one instance: w, d, g, x, f, y (schedule order), y_pair."""

    def __init__(self, n, w, d, gamma, b=16, prec="f64", device="cuda", stream=None,
                 cold=True):
        if not torch.cuda.is_available():
            raise RuntimeError("ccproj needs a ROCm GPU; none is visible")
        self.n, self.gamma, self.b, self.prec = int(n), float(gamma), int(b), prec
        self.ctx = Context(n, b, prec, stream)
        dt = self.ctx.dtype
        npairs = self.n * (self.n - 1) // 2
        self.npairs = npairs
        self.w = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
        self.d = torch.as_tensor(np.ascontiguousarray(d, dtype=np.uint8)).to(device)
        self.g = torch.empty(npairs, dtype=dt, device=device)
        self.x = torch.empty(npairs, dtype=dt, device=device)
        self.f = torch.empty(npairs, dtype=dt, device=device)
        self.y = torch.empty(self.ctx.slots, dtype=dt, device=device)
        self.y_pair = torch.empty(2 * npairs, dtype=dt, device=device)
        self.ctx.prepare(self.w, self.gamma, self.g)
        self.sweeps = 0
        # sparse dual access (Sec. III-D): the nonzero pattern of y, valid
        # only while no dense writer has touched y since it was built
        self.mask = None
        self.mask_valid = False
        if cold:
            self.init_cold()

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.n, inst.w, inst.d, inst.gamma, **kw)

    def invalidate_mask(self):
        """Call after writing y by any means other than sparse sweeps."""
        self.mask_valid = False

    def ensure_mask(self):
        if self.mask is None:
            self.mask = torch.empty(self.ctx.mask_bytes(), dtype=torch.uint8, device=self.y.device)
        if not self.mask_valid:
            self.ctx.mask_build(self.y, self.mask)
            self.mask_valid = True
        return self.mask

    def init_cold(self):
        self.ctx.init_cold(self.x, self.f, self.y, self.y_pair, self.gamma)
        self.invalidate_mask()
        self.sweeps = 0

    def sweep(self, nsweeps=1, executor=None, sparse=False):
        """nsweeps sweeps; sparse=True reads only the duals the mask marks
        (dataflow executor, b = 8, 16, 24, 32; the same results bit for
        bit)."""
        if sparse:
            self.ctx.sweep_sparse(self.x, self.f, self.y, self.y_pair, self.g, self.d,
                                  self.ensure_mask(), nsweeps)
        else:
            self.ctx.sweep(self.x, self.f, self.y, self.y_pair, self.g, self.d, nsweeps, executor)
            self.invalidate_mask()
        self.sweeps += nsweeps

    def sweep_rounds(self, first, count):
        self.ctx.sweep_rounds(self.x, self.y, self.g, first, count)
        self.invalidate_mask()

    def sweep_metric_prefix(self, rounds):
        """The first `rounds` metric rounds of a sweep on the dataflow
        executor (the full sweep's kernel and launch shape)."""
        self.ctx.sweep_metric_prefix(self.x, self.y, self.g, rounds)
        self.invalidate_mask()

    def sweep_metric(self, executor=None, sparse=False):
        if sparse:
            self.ctx.sweep_metric_sparse(self.x, self.y, self.g, self.ensure_mask())
        else:
            self.ctx.sweep_metric(self.x, self.y, self.g, executor)
            self.invalidate_mask()

    def status(self):
        self.ctx.status()

    def pair_pass(self):
        self.ctx.pair_pass(self.x, self.f, self.y_pair, self.g, self.d)

    def residuals(self, what=CC_RESID_ALL, raise_nonfinite=True):
        return self.ctx.residuals(self.x, self.f, self.y, self.y_pair, self.w, self.d,
                                  self.gamma, what, raise_nonfinite)

    def x_from_y(self):
        x = torch.empty_like(self.x)
        f = torch.empty_like(self.f)
        self.ctx.x_from_y(self.y, self.y_pair, self.w, self.gamma, x, f)
        return x, f

    def duals_lex(self):
        y_lex = torch.empty(num_metric_duals(self.n), dtype=self.y.dtype, device=self.y.device)
        self.ctx.duals_to_lex(self.y, y_lex)
        return y_lex

    def nonzero_duals(self, chunk=1 << 28):
        """The nonzero metric duals as host arrays (colex row index 3t + o,
        value as float64), in slot order.  Scans y in chunks (torch.nonzero
        takes at most 2^32 elements)."""
        parts = [torch.nonzero(self.y[s:s + chunk]).flatten() + s
                 for s in range(0, self.y.numel(), chunk)]
        nz = torch.cat(parts)
        lex = torch.empty_like(nz)
        if nz.numel():
            self.ctx.slots_to_lex(nz, lex)
        return lex.cpu().numpy(), self.y[nz].double().cpu().numpy()

    def solve(self, tol=1e-6, max_sweeps=100000, check_every=None, executor=None, sparse=False,
              gap_tol=None):
        """Sweep until both max violations are <= tol (and, with gap_tol,
        the relative duality gap is <= gap_tol), checked every `check_every`
        sweeps (default as in cc_solve_cc_lp: every sweep up to n = 1000,
        every 5 above; a check reads every triplet).  Returns (residuals,
        converged, seconds)."""
        if check_every is None:
            check_every = 1 if self.n <= 1000 else 5
        t0 = time.perf_counter()
        r = None
        while self.sweeps < max_sweeps:
            k = min(check_every, max_sweeps - self.sweeps)
            self.sweep(k, executor, sparse)
            r = self.residuals(CC_RESID_VIOL)
            if max(r["max_viol_metric"], r["max_viol_pair"]) <= tol:
                full = self.residuals()
                if gap_tol is None or abs(full["gap"]) <= gap_tol * max(1.0, abs(full["primal_qp"])):
                    return full, True, time.perf_counter() - t0
        return self.residuals(), False, time.perf_counter() - t0


class CompactSolver:
    """Correlation-clustering state with compacted dual lists (the memory
    form of Sec. III-D): w, d, g, x, f, y_pair on the device, and only the
    nonzero metric duals, in per-tile-step lists the context owns.  b = 8 or
    16.  No dense dual array is allocated."""

    def __init__(self, n, w, d, gamma, b=16, prec="f64", capacity=1 << 20, device="cuda",
                 stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("ccproj needs a ROCm GPU; none is visible")
        self.n, self.gamma, self.b, self.prec = int(n), float(gamma), int(b), prec
        self.ctx = Context(self.n, self.b, prec, stream)
        dt = self.ctx.dtype
        npairs = self.n * (self.n - 1) // 2
        self.w = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
        self.d = torch.as_tensor(np.ascontiguousarray(d, dtype=np.uint8)).to(device)
        self.g = torch.empty(npairs, dtype=dt, device=device)
        self.x = torch.empty(npairs, dtype=dt, device=device)
        self.f = torch.empty(npairs, dtype=dt, device=device)
        self.y_pair = torch.empty(2 * npairs, dtype=dt, device=device)
        self.capacity = int(capacity)
        self.ctx.prepare(self.w, self.gamma, self.g)
        self.init_cold()

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.n, inst.w, inst.d, inst.gamma, **kw)

    def init_cold(self):
        self.ctx.init_cold(self.x, self.f, None, self.y_pair, self.gamma)
        check(_L.cc_compact_init(self.ctx.handle, self.capacity))
        self.sweeps = 0

    def sweep(self, nsweeps=1):
        check(_L.cc_sweep_compact(self.ctx.handle, _ptr(self.x), _ptr(self.f), _ptr(self.y_pair),
                                  _ptr(self.g), _ptr(self.d), int(nsweeps)))
        self.sweeps += nsweeps

    def info(self) -> dict:
        nnz, by, rg = _i64(), _i64(), _i32()
        check(_L.cc_compact_info(self.ctx.handle, ctypes.byref(nnz), ctypes.byref(by),
                                 ctypes.byref(rg)))
        return {"nnz": nnz.value, "bytes": by.value, "regrows": rg.value}

    def to_slots(self):
        """The current duals as a dense schedule-ordered array (tests)."""
        y = torch.empty(self.ctx.slots, dtype=self.x.dtype, device=self.x.device)
        check(_L.cc_compact_to_slots(self.ctx.handle, _ptr(y)))
        return y

    def export(self):
        """(colex row indices, duals) of the nonzero duals, on the device."""
        cnt = _i64()
        check(_L.cc_compact_export(self.ctx.handle, None, None, 0, ctypes.byref(cnt)))
        lex = torch.empty(max(cnt.value, 1), dtype=torch.int64, device=self.x.device)
        val = torch.empty(max(cnt.value, 1), dtype=self.x.dtype, device=self.x.device)
        check(_L.cc_compact_export(self.ctx.handle, _ptr(lex), _ptr(val), lex.numel(),
                                   ctypes.byref(cnt)))
        return lex[:cnt.value], val[:cnt.value]

    def residuals(self):
        """Max violations and the primal objective (x and f only)."""
        return self.ctx.residuals(self.x, self.f, None, None, self.w, self.d, self.gamma,
                                  CC_RESID_VIOL)

    def solve(self, tol=1e-6, max_sweeps=100000, check_every=None):
        if check_every is None:
            check_every = 1 if self.n <= 1000 else 5
        t0 = time.perf_counter()
        r = None
        while self.sweeps < max_sweeps:
            self.sweep(min(check_every, max_sweeps - self.sweeps))
            r = self.residuals()
            if max(r["max_viol_metric"], r["max_viol_pair"]) <= tol:
                return r, True, time.perf_counter() - t0
        return r, False, time.perf_counter() - t0


class L1Solver(Solver):
    """l1 metric nearness (Sec. II-A): min sum w |x - d| over metric x for
    real dissimilarities dv, i.e. (mn1) with real d, on the same device
    state and kernels as Solver; only the pair rows read dv."""

    def __init__(self, n, w, dv, gamma, b=16, prec="f64", device="cuda", stream=None):
        npairs = int(n) * (int(n) - 1) // 2
        super().__init__(n, w, np.zeros(npairs, dtype=np.uint8), gamma, b=b, prec=prec,
                         device=device, stream=stream)
        self.dv = torch.as_tensor(np.ascontiguousarray(dv, dtype=np.float64)).to(device)
        assert self.dv.numel() == npairs

    @classmethod
    def from_instance(cls, inst, gamma=None, **kw):
        return cls(inst.n, inst.w, inst.dv, inst.meta.get("gamma", 1.0) if gamma is None else gamma,
                   **kw)

    def sweep(self, nsweeps=1, executor=None, sparse=False):
        mask = self.ensure_mask() if sparse else None
        check(_L.cc_l1_sweep(self.ctx.handle, _ptr(self.x), _ptr(self.f), _ptr(self.y),
                             _ptr(self.y_pair), _ptr(self.g), _ptr(self.dv), _ptr(mask),
                             int(nsweeps)))
        if not sparse:
            self.invalidate_mask()
        self.sweeps += nsweeps

    def pair_pass(self):
        raise NotImplementedError("the l1 pair rows run inside cc_l1_sweep")

    def residuals(self, what=CC_RESID_ALL, raise_nonfinite=True):
        out = Resid()
        rc = _L.cc_l1_residuals(self.ctx.handle, _ptr(self.x), _ptr(self.f), _ptr(self.y),
                                _ptr(self.y_pair), _ptr(self.w), _ptr(self.dv), self.gamma,
                                int(what), ctypes.byref(out))
        if rc == CC_ENONFINITE and not raise_nonfinite:
            r = out.as_dict()
            r["nonfinite"] = True
            return r
        check(rc)
        return out.as_dict()


class ColourSolver:
    """Device state for the sum-mod-n colouring order (cc_sweep_colour): w,
    d, g, x, f, y_pair as in Solver, the metric duals y in colex order."""

    def __init__(self, n, w, d, gamma, prec="f64", device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("ccproj needs a ROCm GPU; none is visible")
        self.n, self.gamma, self.prec = int(n), float(gamma), prec
        self.ctx = Context(self.n, 16, prec, stream)
        dt = self.ctx.dtype
        npairs = self.n * (self.n - 1) // 2
        self.w = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
        self.d = torch.as_tensor(np.ascontiguousarray(d, dtype=np.uint8)).to(device)
        self.g = torch.empty(npairs, dtype=dt, device=device)
        self.x = torch.empty(npairs, dtype=dt, device=device)
        self.f = torch.empty(npairs, dtype=dt, device=device)
        self.y = torch.empty(num_metric_duals(self.n), dtype=dt, device=device)
        self.y_pair = torch.empty(2 * npairs, dtype=dt, device=device)
        self.ctx.prepare(self.w, self.gamma, self.g)
        self.init_cold()

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.n, inst.w, inst.d, inst.gamma, **kw)

    def init_cold(self):
        check(_L.cc_init_cold_lex(self.ctx.handle, _ptr(self.x), _ptr(self.f), _ptr(self.y),
                                  _ptr(self.y_pair), self.gamma))
        self.sweeps = 0

    def sweep(self, nsweeps=1):
        check(_L.cc_sweep_colour(self.ctx.handle, _ptr(self.x), _ptr(self.f), _ptr(self.y),
                                 _ptr(self.y_pair), _ptr(self.g), _ptr(self.d), int(nsweeps)))
        self.sweeps += nsweeps

    def residuals(self):
        """Max violations and the primal objective (the dual terms need the
        schedule-ordered duals and are not offered here)."""
        return self.ctx.residuals(self.x, self.f, None, None, self.w, self.d, self.gamma,
                                  CC_RESID_VIOL)

    def solve(self, tol=1e-6, max_sweeps=100000, check_every=None):
        if check_every is None:
            check_every = 1 if self.n <= 1000 else 5
        t0 = time.perf_counter()
        r = None
        while self.sweeps < max_sweeps:
            self.sweep(min(check_every, max_sweeps - self.sweeps))
            r = self.residuals()
            if max(r["max_viol_metric"], r["max_viol_pair"]) <= tol:
                return r, True, time.perf_counter() - t0
        return r, False, time.perf_counter() - t0


class NearnessSolver:
    """Device state of an l2 metric nearness instance (Sec. II-A, p = 2):
    min (1/2) sum w (x - d)^2 over metric x.  w, d (float64, device), g =
    1/w, x and y (schedule order) in the chosen precision.  Algorithm 1 from
    x = d, y = 0; a sweep is the metric rounds only."""

    def __init__(self, n, w, dv, b=16, prec="f64", device="cuda", stream=None):
        self.n, self.b, self.prec = int(n), int(b), prec
        self.ctx = Context(self.n, self.b, prec, stream)
        dt = torch.float64 if prec == "f64" else torch.float32
        self.w = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
        self.dv = torch.as_tensor(np.ascontiguousarray(dv, dtype=np.float64)).to(device)
        npairs = self.n * (self.n - 1) // 2
        assert self.w.numel() == npairs and self.dv.numel() == npairs
        self.g = torch.empty(npairs, dtype=dt, device=device)
        self.x = torch.empty(npairs, dtype=dt, device=device)
        self.y = torch.empty(self.ctx.slots, dtype=dt, device=device)
        self.ctx.prepare(self.w, 1.0, self.g)
        self.mask = None  # nonzero pattern of y for sparse sweeps
        self.init()

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.n, inst.w, inst.dv, **kw)

    def init(self):
        check(_L.cc_nearness_init(self.ctx.handle, _ptr(self.dv), _ptr(self.x), _ptr(self.y)))
        self.mask_valid = False
        self.sweeps = 0

    def ensure_mask(self):
        if self.mask is None:
            self.mask = torch.empty(self.ctx.mask_bytes(), dtype=torch.uint8, device=self.y.device)
        if not self.mask_valid:
            self.ctx.mask_build(self.y, self.mask)
            self.mask_valid = True
        return self.mask

    def sweep(self, nsweeps=1, executor=None, sparse=False):
        for _ in range(nsweeps):
            if sparse:
                self.ctx.sweep_metric_sparse(self.x, self.y, self.g, self.ensure_mask())
            else:
                self.ctx.sweep_metric(self.x, self.y, self.g, executor)
                self.mask_valid = False
        self.sweeps += nsweeps

    def status(self):
        self.ctx.status()

    def residuals(self, what=CC_RESID_ALL, raise_nonfinite=True):
        out = NResid()
        rc = _L.cc_nearness_residuals(self.ctx.handle, _ptr(self.x), _ptr(self.y), _ptr(self.w),
                                      _ptr(self.dv), int(what), ctypes.byref(out))
        if rc == CC_ENONFINITE and not raise_nonfinite:
            return out.as_dict()
        check(rc)
        return out.as_dict()

    def duals_lex(self):
        y_lex = torch.empty(num_metric_duals(self.n), dtype=self.y.dtype, device=self.y.device)
        self.ctx.duals_to_lex(self.y, y_lex)
        return y_lex

    def solve(self, tol=1e-6, gap_tol=None, max_sweeps=100000, check_every=None, executor=None,
              sparse=False):
        """Sweep until the max metric violation is at most tol and, with
        gap_tol, the relative primal-dual gap is at most gap_tol.  Returns
        (residuals, converged)."""
        every = check_every or (1 if self.n <= 1000 else 5)
        what = CC_RESID_VIOL | (CC_RESID_DUAL if gap_tol is not None else 0)
        r = self.residuals(what)
        while self.sweeps < max_sweeps:
            self.sweep(min(every, max_sweeps - self.sweeps), executor, sparse)
            r = self.residuals(what)
            if r["max_viol"] <= tol and (gap_tol is None or
                                         abs(r["gap"]) <= gap_tol * max(1.0, abs(r["primal"]))):
                return r, True
        return r, False
