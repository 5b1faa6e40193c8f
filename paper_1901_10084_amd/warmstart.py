"""Learned warm start: a 4-32-32-1 network predicting the converged dual of
every metric row from local features, trained on duals the solver itself
produces (binding of the cc_mlp_* / cc_warm_start_mlp entry points).

Every step runs in the library's kernels; this module holds the loops.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

from . import ccproj as C
from . import instances as I

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "warm_start_sbm300.npy")


def weights_path(family: str = "sbm300") -> str:
    return os.path.join(WEIGHTS_DIR, f"warm_start_{family}.npy")
NPARAM = int(C._L.cc_mlp_num_params())


def init_params(seed: int) -> np.ndarray:
    p = np.zeros(NPARAM, dtype=np.float32)
    C.check(C._L.cc_mlp_init(p.ctypes.data, int(seed)))
    return p


class Network:
    """Parameters and Adam state on the device."""

    def __init__(self, params=None, seed=0, device="cuda"):
        if params is None:
            params = init_params(seed)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._ws = None

    def host_params(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()

    def _workspace(self, count):
        nbytes = int(C._L.cc_mlp_workspace_bytes(int(count)))
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.params.device)
        return self._ws

    def forward(self, phi: torch.Tensor) -> torch.Tensor:
        phi = phi.contiguous()
        y = torch.empty(phi.shape[0], dtype=torch.float32, device=phi.device)
        C.check(C._L.cc_mlp_forward(self.params.data_ptr(), phi.data_ptr(), phi.shape[0],
                                    y.data_ptr(), C._stream_handle(None)))
        return y

    def train_step(self, phi, target, lr=1e-3, grad_out=None):
        """One step on explicit samples; returns the loss before the step."""
        phi, target = phi.contiguous(), target.contiguous()
        n = phi.shape[0]
        if lr > 0:
            self.step += 1
        C.check(C._L.cc_mlp_train_step(phi.data_ptr(), target.data_ptr(), n,
                                       self.params.data_ptr(), self.m.data_ptr(),
                                       self.v.data_ptr(), max(self.step, 1), float(lr),
                                       None if grad_out is None else grad_out.data_ptr(),
                                       self._workspace(n).data_ptr(), self.loss.data_ptr(),
                                       C._stream_handle(None)))
        return self.loss

    def train_on_graph(self, solver, y_star, deg, batch, steps, lr, seed):
        """`steps` Adam steps on rows sampled from a solved instance."""
        ws = self._workspace(batch)
        losses = []
        for s in range(steps):
            self.step += 1
            C.check(C._L.cc_mlp_train_graph(solver.ctx.handle, y_star.data_ptr(),
                                            solver.w.data_ptr(), solver.d.data_ptr(),
                                            deg.data_ptr(), int(batch),
                                            int(seed * 1000003 + s), self.params.data_ptr(),
                                            self.m.data_ptr(), self.v.data_ptr(), self.step,
                                            float(lr), ws.data_ptr(), self.loss.data_ptr()))
            if s % 50 == 0 or s == steps - 1:
                losses.append(float(self.loss))
        return losses


def slot_features(solver, deg, slots):
    phi = torch.empty((slots.numel(), 4), dtype=torch.float32, device=slots.device)
    C.check(C._L.cc_mlp_slot_features(solver.ctx.handle, solver.w.data_ptr(), solver.d.data_ptr(),
                                      deg.data_ptr(), slots.data_ptr(), slots.numel(),
                                      phi.data_ptr()))
    return phi


def infer(solver, net: Network, deg, y_out):
    """Network prediction of every metric dual into y_out (schedule order)."""
    C.check(C._L.cc_mlp_infer(solver.ctx.handle, net.params.data_ptr(), deg.data_ptr(),
                              solver.w.data_ptr(), solver.d.data_ptr(), y_out.data_ptr()))


def warm_start(solver, net: Network, deg) -> dict:
    """Gated learned warm start of a Solver in place (see cc_warm_start_mlp)."""
    acc = ctypes.c_int32()
    dw, dc, ub = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    C.check(C._L.cc_warm_start_mlp(solver.ctx.handle, net.params.data_ptr(), deg.data_ptr(),
                                   solver.w.data_ptr(), solver.d.data_ptr(), solver.gamma,
                                   solver.x.data_ptr(), solver.f.data_ptr(), solver.y.data_ptr(),
                                   solver.y_pair.data_ptr(), solver.g.data_ptr(),
                                   ctypes.byref(acc), ctypes.byref(dw), ctypes.byref(dc),
                                   ctypes.byref(ub)))
    solver.invalidate_mask()
    solver.sweeps = 0
    smp = solver.ctx.last_gate_sample()
    return {"accepted": bool(acc.value), "dual_warm": dw.value, "dual_cold": dc.value,
            "dual_bound": ub.value,
            "gap_share": (dw.value - dc.value) / (ub.value - dc.value),
            "sample_drawn": smp["drawn"], "sample_gain": smp["gain"],
            "sample_std_error": smp["std_error"], "sample_rejected": smp["rejected"]}


def gate_terms(solver, net: Network, deg, pairs, want_delta=True):
    """Terms of the warm-start gate for the given pairs (packed indices, a
    device int64 tensor): their metric A'y at the predicted duals and their
    terms of D_warm - D_cold (cc_warm_gate_terms)."""
    pairs = pairs.to(device="cuda", dtype=torch.int64).contiguous()
    aty = torch.empty(pairs.numel(), device="cuda", dtype=torch.float64)
    delta = torch.empty_like(aty) if want_delta else None
    C.check(C._L.cc_warm_gate_terms(solver.ctx.handle, net.params.data_ptr(), deg.data_ptr(),
                                    solver.w.data_ptr(), solver.d.data_ptr(), solver.gamma,
                                    solver.g.data_ptr(), pairs.data_ptr(), pairs.numel(),
                                    aty.data_ptr(), None if delta is None else delta.data_ptr()))
    return aty, delta


def degrees(inst, device="cuda"):
    return torch.as_tensor(inst.deg.astype(np.float32)).to(device)


def train(seeds=range(1000, 1200), tol=1e-6, b=16, batch=8192, steps_per_graph=40, lr=2e-3,
          net_seed=0, log=None, family="sbm300"):
    """Train on the converged FP64 duals of the warm-start training graphs
    (n = 300, see instances.training_graph), one graph at a time."""
    net = Network(seed=net_seed)
    t0 = time.perf_counter()
    hist = []
    for e, seed in enumerate(seeds):
        inst = I.training_graph(seed, family)
        s = C.Solver.from_instance(inst, b=b, prec="f64")
        r, conv, _ = s.solve(tol=tol, max_sweeps=20000, executor=C.CC_EXEC_DATAFLOW)
        losses = net.train_on_graph(s, s.y, degrees(inst), batch, steps_per_graph, lr, seed)
        hist.append((seed, s.sweeps, losses[0], losses[-1]))
        if log and (e % 20 == 0 or e == len(seeds) - 1):
            log(f"graph {seed}: {s.sweeps} sweeps, loss {losses[0]:.4g} -> {losses[-1]:.4g}, "
                f"{time.perf_counter() - t0:.1f} s")
        del s
    return net, hist


def save(net: Network, path=DEFAULT_WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, net.host_params())


def load(path=DEFAULT_WEIGHTS) -> Network:
    return Network(params=np.load(path))


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="train the warm-start network on solved graphs")
    ap.add_argument("--family", default="sbm300", choices=I.TRAINING_FAMILIES)
    ap.add_argument("--out", default=None, help="weights file (default: weights/warm_start_<family>.npy)")
    args = ap.parse_args()
    net, hist = train(log=lambda m: print(m, flush=True), family=args.family)
    out = args.out or weights_path(args.family)
    save(net, out)
    print("saved", out, flush=True)
