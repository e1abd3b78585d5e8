"""Binding of the device nonlinear residual (scdg_dg_* in the C ABI).

R(Q) = M (Q - Q_s) / dt + H(Q) for the GL-DGSEM compressible Navier-Stokes
operator on a periodic Cartesian mesh (paper, eq. ImplicitDisc, eq. DiscretNS,
eq. DGSEMsystem).  Argument marshalling only: both kernels run in libscdg.so.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L
from .plan import _ptr, _stream


class DgResidual:
    """Owns one scdg_dg object (parameters + lifted-gradient workspace)."""

    def __init__(self, k_elem: int, order: int, mach: float, reynolds: float,
                 length: float = 2.0 * math.pi, gamma: float = 1.4, prandtl: float = 0.72,
                 sutherland_ratio: float = 110.4 / 288.15, stream=None, viscous: str = "br1",
                 sipg_eta: float = 1.0):
        """viscous: face viscous flux, "br1" (Bassi-Rebay 1) or "sipg" (symmetric
        interior penalty with sigma = sipg_eta (N + 1)^2 / h; Cartesian cubes only)."""
        self.lib = L.load()
        vf = {"br1": 0, "sipg": 1}[viscous]
        prm = L.DgParams(k_elem, order, length, mach, reynolds, gamma, prandtl, sutherland_ratio, vf, sipg_eta)
        handle = C.c_void_p()
        st = self.lib.scdg_dg_create(C.byref(handle), C.byref(prm), _stream(stream))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_create")
        self.handle = handle
        self.k_elem, self.order = k_elem, order
        self.n_dof = k_elem ** 3 * (order + 1) ** 3 * 5

    def _check(self, t: torch.Tensor, name: str):
        if t.dtype != torch.float64 or t.numel() != self.n_dof:
            raise ValueError(f"{name}: expected {self.n_dof} float64 values")

    def residual(self, q: torch.Tensor, q_s: torch.Tensor | None = None, inv_dt: float = 0.0,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(q, "q")
        if q_s is not None:
            self._check(q_s, "q_s")
        if out is None:
            out = torch.empty(self.n_dof, dtype=torch.float64, device=q.device)
        self._check(out, "out")
        st = self.lib.scdg_dg_residual(self.handle, _ptr(q), _ptr(q_s), float(inv_dt), _ptr(out))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_residual")
        return out

    def jacobian_blocks(self, plan, q: torch.Tensor, inv_dt: float) -> dict:
        """Element blocks of A = M inv_dt + dH/dQ(q) in the plan's format (aii,
        aib, abi, bb_val), formed on the device (scdg_dg_jacobian_blocks)."""
        self._check(q, "q")
        h = plan._host
        n_i = 5 * (h["order"].astype(np.int64) - 1) ** 3
        n_c = 5 * np.diff(h["c_ptr"])
        dev = q.device
        out = dict(aii=torch.empty(int((n_i * n_i).sum()), dtype=torch.float64, device=dev),
                   aib=torch.empty(int((n_i * n_c).sum()), dtype=torch.float64, device=dev),
                   abi=torch.empty(int((n_i * n_c).sum()), dtype=torch.float64, device=dev),
                   bb_val=torch.empty(max(1, 25 * len(h["bb_col"])), dtype=torch.float64, device=dev))
        st = self.lib.scdg_dg_jacobian_blocks(self.handle, plan.handle, _ptr(q), float(inv_dt), _ptr(out["aii"]),
                                              _ptr(out["aib"]), _ptr(out["abi"]), _ptr(out["bb_val"]))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_jacobian_blocks", L.last_error(plan.handle))
        out["bb_val"] = out["bb_val"][:25 * len(h["bb_col"])]
        return out

    def jacobian_apply(self, q: torch.Tensor, v: torch.Tensor, inv_dt: float = 0.0,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """A v = M v inv_dt + dH/dQ(q) v, the Newton matrix at q applied to v
        (scdg_dg_jacobian_apply)."""
        self._check(q, "q")
        self._check(v, "v")
        if out is None:
            out = torch.empty(self.n_dof, dtype=torch.float64, device=q.device)
        self._check(out, "out")
        if out.data_ptr() in (q.data_ptr(), v.data_ptr()):
            raise ValueError("out must not alias q or v")
        st = self.lib.scdg_dg_jacobian_apply(self.handle, _ptr(q), _ptr(v), float(inv_dt), _ptr(out))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_jacobian_apply")
        return out

    def set_geometry(self, xyz=None):
        """Curved elements from the node positions (numpy, 3 per node in the natural
        node order, e.g. [K, K, K, P, P, P, 3]); None returns to Cartesian cubes."""
        if xyz is None:
            st = self.lib.scdg_dg_set_geometry(self.handle, None)
        else:
            arr = np.ascontiguousarray(xyz, dtype=np.float64)
            if arr.size != 3 * (self.n_dof // 5):
                raise ValueError(f"xyz: expected {3 * (self.n_dof // 5)} values")
            st = self.lib.scdg_dg_set_geometry(self.handle, arr.ctypes.data)
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_set_geometry")

    def gradient(self, out: torch.Tensor | None = None) -> torch.Tensor:
        n_nodes = self.n_dof // 5
        if out is None:
            out = torch.empty(n_nodes * 15, dtype=torch.float64, device="cuda")
        st = self.lib.scdg_dg_gradient(self.handle, _ptr(out))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_dg_gradient")
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.scdg_dg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
