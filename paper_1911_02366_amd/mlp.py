"""Binding of the learned-initial-guess network (scdg_mlp_* / scdg_guess_* in
the C ABI): a per-element multilayer perceptron with forward, backward, Adam
and loss kernels, and the maps between DG vectors and network features.
Argument marshalling only; every kernel runs in libscdg.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .plan import _ptr, _stream


def _f32(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float32 or t.numel() < n:
        raise ValueError(f"{name}: expected at least {n} float32 values")


class Mlp:
    """One scdg_mlp object; parameters and Adam moments are caller tensors."""

    def __init__(self, n_in: int, n_hidden: int, n_layers: int, n_out: int, max_batch: int,
                 stream=None):
        self.lib = L.load()
        shape = L.MlpShape(n_in, n_hidden, n_layers, n_out, max_batch)
        handle = C.c_void_p()
        st = self.lib.scdg_mlp_create(C.byref(handle), C.byref(shape), _stream(stream))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_mlp_create")
        self.handle = handle
        self.n_in, self.n_hidden, self.n_layers, self.n_out = n_in, n_hidden, n_layers, n_out
        self.max_batch = max_batch
        self.compute = "fp32"
        n = C.c_int64()
        self.lib.scdg_mlp_param_count(handle, C.byref(n))
        self.n_params = n.value

    def set_compute(self, mode: str):
        """'fp32' (FP32 operands) or 'bf16' (operands rounded to bfloat16), both
        with FP32 accumulation."""
        self._ok(self.lib.scdg_mlp_set_compute(self.handle, {"fp32": 0, "bf16": 1}[mode]), "scdg_mlp_set_compute")
        self.compute = mode

    # ---------------------------------------------------------------- layout
    def layer_slices(self):
        """[(w_offset, fan_in, fan_out, b_offset)] of the flat parameter vector."""
        out, off = [], 0
        for layer in range(self.n_layers + 1):
            fi = self.n_in if layer == 0 else self.n_hidden
            fo = self.n_out if layer == self.n_layers else self.n_hidden
            out.append((off, fi, fo, off + fi * fo))
            off += fi * fo + fo
        return out

    def init_params(self, seed: int, device="cuda", zero_output: bool = False) -> torch.Tensor:
        """Glorot-uniform weights, zero biases, from numpy's seeded PCG64 (host);
        zero_output leaves the output layer at zero, so the untrained network
        predicts a zero correction."""
        rng = np.random.default_rng(seed)
        w = np.zeros(self.n_params, dtype=np.float32)
        lay = self.layer_slices()
        for i, (off, fi, fo, _) in enumerate(lay):
            a = np.sqrt(6.0 / (fi + fo))
            vals = rng.uniform(-a, a, fi * fo).astype(np.float32)
            if not (zero_output and i == len(lay) - 1):
                w[off:off + fi * fo] = vals
        return torch.tensor(w, device=device)

    def _ok(self, st, where):
        if st != L.SCDG_OK:
            raise L.ScdgError(st, where)

    # ---------------------------------------------------------------- network
    def forward(self, w, x, batch: int, y=None):
        _f32(w, self.n_params, "w")
        _f32(x, batch * self.n_in, "x")
        if y is None:
            y = torch.empty(batch * self.n_out, dtype=torch.float32, device=x.device)
        _f32(y, batch * self.n_out, "y")
        self._ok(self.lib.scdg_mlp_forward(self.handle, _ptr(w), _ptr(x), batch, _ptr(y)),
                 "scdg_mlp_forward")
        return y

    def backward(self, w, x, dy, batch: int, dw=None, dx=None):
        _f32(dy, batch * self.n_out, "dy")
        if dw is None:
            dw = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        _f32(dw, self.n_params, "dw")
        if dx is not None:
            _f32(dx, batch * self.n_in, "dx")
        self._ok(self.lib.scdg_mlp_backward(self.handle, _ptr(w), _ptr(x), _ptr(dy), batch, _ptr(dw),
                                            _ptr(dx)), "scdg_mlp_backward")
        return dw

    def adam(self, w, dw, m1, m2, lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-8):
        for t, name in ((w, "w"), (dw, "dw"), (m1, "m1"), (m2, "m2")):
            _f32(t, self.n_params, name)
        self._ok(self.lib.scdg_mlp_adam(self.handle, _ptr(w), _ptr(dw), _ptr(m1), _ptr(m2), lr, beta1,
                                        beta2, eps, step), "scdg_mlp_adam")

    def mse(self, y, t, n: int, dy=None, loss=None):
        _f32(y, n, "y")
        _f32(t, n, "t")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=y.device)
        self._ok(self.lib.scdg_mlp_mse(self.handle, _ptr(y), _ptr(t), n, _ptr(dy), _ptr(loss)),
                 "scdg_mlp_mse")
        return loss

    def gather(self, src, width: int, idx, count: int, dst=None):
        if idx.dtype != torch.int32:
            raise ValueError("idx must be int32")
        if dst is None:
            dst = torch.empty(count * width, dtype=torch.float32, device=src.device)
        self._ok(self.lib.scdg_mlp_gather(self.handle, _ptr(src), width, _ptr(idx), count, _ptr(dst)),
                 "scdg_mlp_gather")
        return dst

    # ---------------------------------------------------------------- DG maps
    def guess_stats(self, q, dq_prev, dq=None, r=None, stats=None):
        """25 field statistics [mean, std, rms_prev, rms_corr, rms_res] x 5 variables."""
        if stats is None:
            stats = torch.empty(25, dtype=torch.float64, device=q.device)
        self._ok(self.lib.scdg_guess_stats(self.handle, _ptr(q), _ptr(dq_prev), _ptr(dq), _ptr(r), q.numel(),
                                           _ptr(stats)), "scdg_guess_stats")
        return stats

    def features(self, q, dq_prev, stats, n_elem: int, x=None, r=None):
        if x is None:
            x = torch.empty(n_elem * self.n_in, dtype=torch.float32, device=q.device)
        self._ok(self.lib.scdg_guess_features(self.handle, _ptr(q), _ptr(dq_prev), _ptr(r), _ptr(stats), n_elem,
                                              _ptr(x)), "scdg_guess_features")
        return x

    def target(self, dq, dq_prev, stats, n_elem: int, t=None):
        if t is None:
            t = torch.empty(n_elem * self.n_out, dtype=torch.float32, device=dq.device)
        self._ok(self.lib.scdg_guess_target(self.handle, _ptr(dq), _ptr(dq_prev), _ptr(stats), n_elem,
                                            _ptr(t)), "scdg_guess_target")
        return t

    def apply(self, dq_prev, y, stats, n_elem: int, dq=None):
        if dq is None:
            dq = torch.empty(n_elem * self.n_out, dtype=torch.float64, device=dq_prev.device)
        self._ok(self.lib.scdg_guess_apply(self.handle, _ptr(dq_prev), _ptr(y), _ptr(stats), n_elem,
                                           _ptr(dq)), "scdg_guess_apply")
        return dq

    def close(self):
        if getattr(self, "handle", None):
            self.lib.scdg_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
