"""Python binding of the scdg C ABI with the same call names.

Device memory and streams come from PyTorch (tensors on a HIP device); the
binding only passes their pointers.  Host structure arrays are numpy.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from . import tuning


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("scdg works on device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Plan:
    """Owns one scdg_plan.  Call order: assemble -> factor -> condense -> solve*."""

    def __init__(self, order, c_ptr, c_node, bb_rowptr, bb_col, stream=None, phys_faces=None, device: int = -1):
        self.lib = L.load()
        self._host = dict(
            order=np.ascontiguousarray(order, dtype=np.int32),
            c_ptr=np.ascontiguousarray(c_ptr, dtype=np.int64),
            c_node=np.ascontiguousarray(c_node, dtype=np.int32),
            bb_rowptr=np.ascontiguousarray(bb_rowptr, dtype=np.int64),
            bb_col=np.ascontiguousarray(bb_col, dtype=np.int32),
        )
        h = self._host
        if phys_faces is not None:
            h["phys_faces"] = np.ascontiguousarray(phys_faces, dtype=np.uint8)
            if h["phys_faces"].shape != h["order"].shape:
                raise ValueError("phys_faces: one mask per element")
        s = L.Structure(len(h["order"]), h["order"].ctypes.data, h["c_ptr"].ctypes.data,
                        h["c_node"].ctypes.data, h["bb_rowptr"].ctypes.data,
                        h["bb_col"].ctypes.data if len(h["bb_col"]) else None,
                        h["phys_faces"].ctypes.data if phys_faces is not None else None)
        handle = C.c_void_p()
        st = self.lib.scdg_plan_create(C.byref(handle), C.byref(s), _stream(stream), int(device))
        if st != L.SCDG_OK:
            raise L.ScdgError(st, "scdg_plan_create", L.last_error(None))
        self.handle = handle
        self._keep = ()
        n_dof, n1, n2, nb = (C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64())
        self.lib.scdg_plan_sizes(handle, C.byref(n_dof), C.byref(n1), C.byref(n2), C.byref(nb))
        self.n_dof, self.n1, self.n2, self.n_bnodes = n_dof.value, n1.value, n2.value, nb.value
        nf, nr = C.c_int64(), C.c_int64()
        self.lib.scdg_plan_fold_counts(handle, C.byref(nf), C.byref(nr))
        self.n_folded, self.n_remainder = nf.value, nr.value

    @classmethod
    def from_structure(cls, st: dict, stream=None, device: int = -1) -> "Plan":
        return cls(st["order"], st["c_ptr"], st["c_node"], st["bb_rowptr"], st["bb_col"], stream,
                   st.get("phys_faces"), device)

    def _check(self, st: int, where: str):
        if st != L.SCDG_OK:
            raise L.ScdgError(st, where, L.last_error(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.scdg_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        self._check(self.lib.scdg_set_stream(self.handle, _stream(stream)), "scdg_set_stream")

    def assemble(self, aii, aib, abi, bb_val, copy: bool = False):
        """Register the blocks: borrowed (kept referenced here until the next
        assemble) or, with copy=True, copied into plan-owned storage."""
        for t in (aii, aib, abi, bb_val):
            if t.dtype != torch.float64:
                raise TypeError("blocks must be float64")
        self._keep = () if copy else (aii, aib, abi, bb_val)
        flags = L.SCDG_COPY if copy else L.SCDG_BORROW
        self._check(self.lib.scdg_assemble(self.handle, _ptr(aii), _ptr(aib), _ptr(abi), _ptr(bb_val), flags),
                    "scdg_assemble")

    def factor(self, precision: str = "fp64"):
        prec = {"fp64": L.SCDG_FP64, "fp32": L.SCDG_FP32}[precision]
        self.precision = precision
        self._check(self.lib.scdg_factor(self.handle, prec), "scdg_factor")

    def factor_info(self):
        e, i = C.c_int64(), C.c_int32()
        self._check(self.lib.scdg_factor_info(self.handle, C.byref(e), C.byref(i)), "scdg_factor_info")
        return e.value, i.value

    def condense(self):
        self._check(self.lib.scdg_condense(self.handle), "scdg_condense")

    def condense_rhs(self, b, bs=None):
        if bs is None:
            bs = torch.empty(self.n1, dtype=torch.float64, device=b.device)
        self._check(self.lib.scdg_condense_rhs(self.handle, _ptr(b), _ptr(bs)), "scdg_condense_rhs")
        return bs

    @staticmethod
    def _opts(**kw) -> L.SolveOpts:
        o = L.SolveOpts()
        o.precond = -1
        solver = kw.pop("solver", "auto")
        o.solver = {"auto": L.SOLVER_AUTO, "dense": L.SOLVER_DENSE, "gmres": L.SOLVER_GMRES}[solver]
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def solve_condensed(self, bs, qb=None, x0=None, check=True, **opts):
        if qb is None:
            qb = torch.empty(self.n1, dtype=torch.float64, device=bs.device)
        o, info = self._opts(**opts), L.SolveInfo()
        st = self.lib.scdg_solve_condensed(self.handle, _ptr(bs), _ptr(qb), _ptr(x0), C.byref(o),
                                           C.byref(info))
        if check:
            self._check(st, "scdg_solve_condensed")
        return qb, info.as_dict() | {"status": st}

    def backsolve(self, b, qb, dq=None):
        if dq is None:
            dq = torch.empty(self.n_dof, dtype=torch.float64, device=b.device)
        self._check(self.lib.scdg_backsolve(self.handle, _ptr(b), _ptr(qb), _ptr(dq)), "scdg_backsolve")
        return dq

    def solve(self, b, dq=None, x0=None, check=True, **opts):
        if dq is None:
            dq = torch.empty(self.n_dof, dtype=torch.float64, device=b.device)
        o, info = self._opts(**opts), L.SolveInfo()
        st = self.lib.scdg_solve(self.handle, _ptr(b), _ptr(dq), _ptr(x0), C.byref(o), C.byref(info))
        if check:
            self._check(st, "scdg_solve")
        return dq, info.as_dict() | {"status": st}

    def residual(self, b, dq, r=None):
        rel = C.c_double()
        self._check(self.lib.scdg_residual(self.handle, _ptr(b), _ptr(dq), _ptr(r), C.byref(rel)),
                    "scdg_residual")
        return r, rel.value

    def _boundary_vectors(self, *vs):
        for v in vs:
            if v.dtype != torch.float64 or v.numel() < self.n1 or not v.is_contiguous():
                raise ValueError(f"boundary vectors are contiguous float64 tensors of at least {self.n1} entries")

    def schur_apply(self, x, y=None):
        if y is None:
            y = torch.empty_like(x)
        self._boundary_vectors(x, y)
        self._check(self.lib.scdg_schur_apply(self.handle, _ptr(x), _ptr(y)), "scdg_schur_apply")
        return y

    def schur_apply_transpose(self, x, y=None):
        """y = S^T x (scdg_schur_apply_transpose; assembled form)."""
        if y is None:
            y = torch.empty_like(x)
        self._boundary_vectors(x, y)
        self._check(self.lib.scdg_schur_apply_transpose(self.handle, _ptr(x), _ptr(y)),
                    "scdg_schur_apply_transpose")
        return y

    def guess_schur_loss(self, y, t, stats, scale: float = 1.0, dy=None, loss=None, grad: bool = True):
        """Condensed-residual loss scale ||S P_b (rc (y - t))||^2 of a normalised
        guess y against its target t (float32 natural vectors, either None for
        zero), and its gradient dy with respect to y when grad
        (scdg_guess_schur_loss; assembled form).  Returns (loss, dy), loss a
        one-element device double."""
        for name, v in (("y", y), ("t", t), ("dy", dy if grad else None)):
            if v is not None and (v.dtype != torch.float32 or v.numel() < self.n_dof or not v.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float32 tensor of at least {self.n_dof} entries")
        if stats.dtype != torch.float64 or stats.numel() < 25 or not stats.is_contiguous():
            raise ValueError("stats must be a contiguous float64 tensor of 25 entries")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=stats.device)
        elif loss.dtype != torch.float64 or loss.numel() < 1:
            raise ValueError("loss must be a float64 tensor")
        if grad and dy is None:
            dy = torch.empty(self.n_dof, dtype=torch.float32, device=stats.device)
        self._check(self.lib.scdg_guess_schur_loss(self.handle, _ptr(y), _ptr(t), _ptr(stats), float(scale),
                                                   _ptr(dy) if grad else None, _ptr(loss)),
                    "scdg_guess_schur_loss")
        return loss, (dy if grad else None)

    def newton_step(self, dg, q_s, inv_dt: float, q, check=True, **opts):
        """Newton iterations of one backward-Euler step (scdg_newton_step): each
        iteration is one replay of a captured graph.  q holds the starting state on
        entry and the new state on return (updated in place); q_s is unchanged.
        Options: newton_tol, lin_tol, forcing, eta_max, restart, cycles, precond,
        max_newton (unset ones take the library defaults)."""
        for t, name in ((q_s, "q_s"), (q, "q")):
            if t.dtype != torch.float64 or t.numel() != self.n_dof or not t.is_contiguous():
                raise ValueError(f"{name}: expected {self.n_dof} contiguous float64 values")
        o = L.NewtonOpts()
        o.forcing = -1.0
        o.precond = -1
        for k, v in opts.items():
            setattr(o, k, v)
        info = L.NewtonInfo()
        st = self.lib.scdg_newton_step(self.handle, dg.handle, _ptr(q_s), float(inv_dt), _ptr(q), C.byref(o),
                                       C.byref(info))
        if check:
            self._check(st, "scdg_newton_step")
        return info.as_dict() | {"status": st}

    def set_krylov_mode(self, mode: str):
        """'host' (Givens on the host), 'device' (device-resident cycle) or 'graph'
        (device-resident cycle replayed from a HIP graph)."""
        m = {"host": 0, "device": 1, "graph": 2}[mode]
        self._check(self.lib.scdg_set_krylov_mode(self.handle, m), "scdg_set_krylov_mode")

    def set_schur_mode(self, mode: str):
        """'assembled' (Schur products through the element blocks T_e),
        'matrix_free' (through X_e, A_bi and A_bb; T_e never formed) or
        'matrix_free_sparse' (through the nonzero 5x5 blocks of A_ib and A_bi,
        A_ii^-1 and A_bb).  A condensed plan needs condense() again after a
        change."""
        m = {"assembled": 0, "matrix_free": 1, "matrix_free_sparse": 2}[mode]
        self._check(self.lib.scdg_set_schur_mode(self.handle, m), "scdg_set_schur_mode")

    def schur_mode(self) -> str:
        out = C.c_int32()
        self._check(self.lib.scdg_get_schur_mode(self.handle, C.byref(out)), "scdg_get_schur_mode")
        return ["assembled", "matrix_free", "matrix_free_sparse"][out.value]

    def set_inverse_mode(self, mode: str):
        """'auto', 'single' (one workgroup per element), 'blocked' or 'resident'
        (one workgroup per element with a wide outer panel in LDS)."""
        m = {"auto": 0, "single": 1, "blocked": 2, "resident": 3}[mode]
        self._check(self.lib.scdg_set_inverse_mode(self.handle, m), "scdg_set_inverse_mode")

    def inverse_mode_used(self) -> str:
        v = C.c_int32()
        self._check(self.lib.scdg_get_inverse_mode(self.handle, C.byref(v)), "scdg_get_inverse_mode")
        return {0: "none", 1: "single", 2: "blocked", 3: "resident"}[v.value]

    def enable_timing(self, on: bool = True):
        self._check(self.lib.scdg_enable_timing(self.handle, int(on)), "scdg_enable_timing")

    def phase_times(self) -> dict:
        n = len(L.PHASES)
        ms = (C.c_double * n)()
        cnt = (C.c_int32 * n)()
        self._check(self.lib.scdg_phase_times(self.handle, ms, cnt, n), "scdg_phase_times")
        return {name: {"ms": ms[i], "count": cnt[i]} for i, name in enumerate(L.PHASES)}

    def problem_signature(self) -> str:
        """Key of this plan's GEMM problems in the autotune cache (sizes, factor
        precision, device, configuration list)."""
        order = self._host["order"].astype(np.int64)
        n_i = 5 * (order - 1) ** 3
        n_c = 5 * np.diff(self._host["c_ptr"])
        dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
        return tuning.problem_signature(n_i, n_c, getattr(self, "precision", "fp64"), dev, L.GEMM_CONFIGS)

    def autotune(self, cache: str | None = None) -> dict:
        """Time every GEMM tile configuration on this plan's problems; keep the
        fastest.  With a cache file (argument, else $SCDG_AUTOTUNE_CACHE), a plan
        whose problem signature is stored takes the stored choice untimed, and a
        new choice is stored."""
        cache = cache or tuning.default_path()
        key = self.problem_signature()
        hit = tuning.lookup(cache, key)
        if hit is not None and hit["x"] in L.GEMM_CONFIGS and hit["s"] in L.GEMM_CONFIGS:
            self.set_gemm_config(hit["x"], hit["s"])
            return dict(hit, cached=True)
        n = len(L.GEMM_CONFIGS)
        mx, ms = (C.c_double * n)(), (C.c_double * n)()
        self._check(self.lib.scdg_autotune(self.handle, mx, ms, n), "scdg_autotune")
        cx, cs = self.gemm_config()
        out = {"x": L.GEMM_CONFIGS[cx], "s": L.GEMM_CONFIGS[cs],
               "ms_x": dict(zip(L.GEMM_CONFIGS, list(mx))), "ms_s": dict(zip(L.GEMM_CONFIGS, list(ms)))}
        tuning.store(cache, key, out)
        return dict(out, cached=False)

    def gemm_config(self):
        cx, cs = C.c_int32(), C.c_int32()
        self._check(self.lib.scdg_get_gemm_config(self.handle, C.byref(cx), C.byref(cs)),
                    "scdg_get_gemm_config")
        return cx.value, cs.value

    def set_gemm_config(self, cfg_x, cfg_s):
        conv = lambda c: L.GEMM_CONFIGS.index(c) if isinstance(c, str) else int(c)
        self._check(self.lib.scdg_set_gemm_config(self.handle, conv(cfg_x), conv(cfg_s)),
                    "scdg_set_gemm_config")

    def export(self, what: str, count: int, dtype=torch.float64, device="cuda"):
        code = {"aii_inv": L.EXPORT_AII_INV, "schur": L.EXPORT_SCHUR, "x": L.EXPORT_X}[what]
        out = torch.empty(count, dtype=dtype, device=device)
        self._check(self.lib.scdg_export(self.handle, code, _ptr(out), out.numel() * out.element_size()),
                    "scdg_export")
        return out
