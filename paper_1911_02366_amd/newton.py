"""Backward-Euler time stepping by Newton's method on the condensed system,
with an optional learned initial guess.

Each implicit step solves R(Q) = M (Q - Q_s)/dt + H(Q) = 0 (paper, eq.
ImplicitDisc and eq. NeqtonEq) by Newton iterations A dQ = -R(Q~) (eq.
NewtonLinSys1), where A is the Jacobian at the start of the step (it is
refreshed once per step and kept for the step's later iterations), every
linear system is solved by the statically condensed GMRES of the library
(Section 3), and R is evaluated by the device residual kernels.  The step
stops when ||R|| <= newton_tol ||R(Q_s)||.  With `forcing`, each linear
solve is taken only to the relative tolerance that target needs
(0.5 newton_tol ||R(Q_s)|| / ||R(Q~)||, clipped to [lin_tol, 0.1]), an
inexact-Newton choice in the spirit of Eisenstat and Walker.  The Jacobian
itself comes from a caller-supplied function of the state, returning device
blocks in the layout of scdg_assemble.  Given node positions `xyz`, the
residual runs on curved hexahedra (metric terms and the mass J w_i w_j w_k);
the condensed solve is the same, since it takes the Jacobian blocks as given.

The learned guess (an addition; the paper has no learned component) is a
per-element network trained on the solver's own (state, previous increment,
increment) triples.  Its prediction enters either as the GMRES initial guess
of the step's first linear solve (mode "gmres", boundary part only, dropped
by the library when worse than zero) or as the Newton starting point (mode
"newton", dropped when R at the predicted state exceeds R at Q_s).  The
Newton stop test is the same in every mode, so every step converges to the
same FP64 residual with or without the network.

Host orchestration only: every arithmetic step runs in libscdg.so.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .dg import DgResidual
from .mlp import Mlp
from .plan import Plan


class ImplicitStepper:
    def __init__(self, structure: dict, k_elem: int, order: int, mach: float, reynolds: float, dt: float,
                 jacobian, lin_tol: float = 1e-10, newton_tol: float = 1e-8, max_newton: int = 10,
                 restart: int = 30, precond: int = 1, precision: str = "fp64", autotune: bool = True,
                 forcing: bool = True, fp32_inner_tol: float = 1e-4, graph: bool = False,
                 graph_cycles: int = 8, autotune_cache: str | None = None, xyz=None,
                 schur_mode: str = "assembled", viscous: str = "br1"):
        self.plan = Plan.from_structure(structure)
        self.plan.set_schur_mode(schur_mode)     # "matrix_free": Schur products through X_e, A_bi, A_bb
        self.dg = DgResidual(k_elem, order, mach=mach, reynolds=reynolds, viscous=viscous)
        if xyz is not None:
            self.dg.set_geometry(xyz)            # curved hexahedra: the residual takes the metric terms
        self.dt = dt
        # jacobian: a callable q -> blocks, or "device" for the library's own
        # blocks (scdg_dg_jacobian_blocks; Cartesian cubes, Bassi-Rebay 1)
        if isinstance(jacobian, str):
            if jacobian != "device":
                raise ValueError("jacobian: a callable or 'device'")
            jacobian = lambda q: self.dg.jacobian_blocks(self.plan, q, 1.0 / self.dt)
        self.jacobian = jacobian
        self.lin_tol, self.newton_tol, self.max_newton = lin_tol, newton_tol, max_newton
        self.restart, self.precond, self.precision = restart, precond, precision
        self._tune = autotune
        self.autotune_cache = autotune_cache
        self.forcing = forcing
        self.fp32_inner_tol = fp32_inner_tol
        self._blocks = None
        self.n_elem = len(structure["order"])
        # graph path: one captured Newton iteration replayed per iteration; the
        # Jacobian blocks and the state vectors live in buffers that keep their
        # addresses from step to step, so the graph is captured once
        self.graph, self.graph_cycles = graph, graph_cycles
        self._persist = None
        self._q_buf = self._qs_buf = None

    def prepare(self, q_s: torch.Tensor, blocks: dict | None = None) -> float:
        """Jacobian at q_s (or the given blocks of it), factor and condense; returns
        the factor+condense seconds."""
        blk = self.jacobian(q_s) if blocks is None else blocks
        if self.graph:
            if self._persist is None:
                self._persist = {k: torch.empty_like(blk[k]) for k in ("aii", "aib", "abi", "bb_val")}
            for k, v in self._persist.items():
                v.copy_(blk[k])
            blk = self._persist
        self._blocks = blk                       # the plan borrows these until the next assemble
        self.plan.assemble(blk["aii"], blk["aib"], blk["abi"], blk["bb_val"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.plan.factor(self.precision)
        if self._tune:
            self.plan.autotune(cache=self.autotune_cache)
            self._tune = False
        self.plan.condense()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def solve_step(self, q_s: torch.Tensor, guess: torch.Tensor | None = None, mode: str = "gmres",
                   graph: bool | None = None, keep_first: bool = False):
        """Newton iterations of one step from a prepared Jacobian; returns (q, info).
        graph (default: the stepper's setting) runs every Newton iteration as one
        replay of the library's captured iteration (scdg_newton_step); there the
        guess can only enter as the Newton starting state.  keep_first returns
        the first Newton correction (the solution of the step's first linear
        system) as info["first_dq"] (host-driven iterations only)."""
        if self.graph if graph is None else graph:
            if keep_first:
                raise ValueError("the captured Newton iteration does not return its first correction")
            return self._solve_step_graph(q_s, guess, mode)
        inv_dt = 1.0 / self.dt
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = self.dg.residual(q_s, q_s, inv_dt)
        r0 = float(torch.linalg.vector_norm(r))
        q = q_s.clone()
        rnorm = r0
        rejected = 0
        if guess is not None and mode == "newton":
            q_try = q_s + guess
            r_try = self.dg.residual(q_try, q_s, inv_dt)
            n_try = float(torch.linalg.vector_norm(r_try))
            if n_try < r0:
                q, r, rnorm = q_try, r_try, n_try
            else:
                rejected = 1
        gmres_iters, first_iters, newton, guess_res = 0, None, 0, 1.0
        first_dq = None
        while rnorm > self.newton_tol * r0 and newton < self.max_newton:
            x0 = guess if (guess is not None and mode == "gmres" and newton == 0) else None
            tol = self.lin_tol
            if self.forcing:
                # inexact Newton: solve only as far as the step's target needs
                tol = min(0.1, max(self.lin_tol, 0.5 * self.newton_tol * r0 / rnorm))
            if self.precision == "fp32":
                # FP32 factors: loose inner GMRES, FP64 refinement on the full system to tol
                ir = dict(ir_tol=tol, ir_max=20)
                inner = max(tol, self.fp32_inner_tol)
            else:
                ir = dict(ir_tol=1.0, ir_max=1)     # FP64 factors: the GMRES tolerance decides
                inner = tol
            dq, info = self.plan.solve(-r, x0=x0, solver="gmres", tol=inner, restart=self.restart,
                                       precond=self.precond, check=False, **ir)
            if info["status"] not in (0,):
                raise RuntimeError(f"condensed solve failed: {info}")
            if x0 is not None and info["guess_rejected"]:
                rejected = 1
            gmres_iters += info["iters"]
            if first_iters is None:
                first_iters = info["iters"]
                guess_res = info["rel_res_guess"]
                if keep_first:
                    first_dq = dq.clone()
            q += dq
            r = self.dg.residual(q, q_s, inv_dt)
            rnorm = float(torch.linalg.vector_norm(r))
            newton += 1
        torch.cuda.synchronize()
        out = dict(newton=newton, gmres=gmres_iters, first_gmres=first_iters or 0,
                   rel_res=rnorm / r0 if r0 > 0 else 0.0, guess_rejected=rejected,
                   guess_res=guess_res,
                   seconds=time.perf_counter() - t0, converged=rnorm <= self.newton_tol * r0)
        if keep_first:
            out["first_dq"] = first_dq if first_dq is not None else torch.zeros_like(q_s)
        return q, out

    def _solve_step_graph(self, q_s: torch.Tensor, guess: torch.Tensor | None, mode: str):
        if guess is not None and mode != "newton":
            raise ValueError("the captured Newton iteration takes a guess only as the starting state")
        if self._q_buf is None:
            self._q_buf = torch.empty_like(q_s)
            self._qs_buf = torch.empty_like(q_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self._qs_buf.copy_(q_s)
        if guess is None:
            self._q_buf.copy_(q_s)
        else:
            torch.add(q_s, guess, out=self._q_buf)
        lin_tol = self.lin_tol if self.precision == "fp64" else max(self.lin_tol, self.fp32_inner_tol)
        info = self.plan.newton_step(self.dg, self._qs_buf, 1.0 / self.dt, self._q_buf, check=False,
                                     newton_tol=self.newton_tol, lin_tol=lin_tol,
                                     forcing=0.5 if self.forcing else 0.0, restart=self.restart,
                                     cycles=self.graph_cycles, precond=self.precond,
                                     max_newton=self.max_newton)
        if info["status"] not in (0, -6):
            raise RuntimeError(f"scdg_newton_step failed: {info}")
        q = self._q_buf.clone()
        torch.cuda.synchronize()
        return q, dict(newton=info["newton"], gmres=info["gmres"], first_gmres=info["first_gmres"],
                       rel_res=info["rel_res"], guess_rejected=info["start_rejected"] if guess is not None else 0,
                       guess_res=1.0, lin_unconverged=info["lin_unconverged"],
                       seconds=time.perf_counter() - t0, converged=bool(info["converged"]))

    def close(self):
        self.plan.close()
        self.dg.close()


class LearnedGuess:
    """Training set, network and optimizer state of the learned initial guess.

    Scales change by orders of magnitude over a run (an initial transient
    decays), so every step is normalized by its own field statistics: the
    features by the step's mean/std of Q and rms of dQprev (and of R(Q_s), the
    step's right-hand side, for a network that takes it), the target (the
    correction dQ - dQprev) by the rms rc of that step's correction.  At
    prediction time the correction of the step is not known yet; the rms of
    the last known correction stands in for it.  A shrinkage factor alpha in
    [0, 1], fitted by least squares on a validation step that training did not
    use, scales the learned correction (alpha = 0 reproduces the previous
    increment); the hold-out step after it is scored only."""

    def __init__(self, n_elem: int, dofs_per_elem: int, capacity: int, hidden: int = 256, layers: int = 2,
                 seed: int = 0, batch: int = 1024, device="cuda", compute: str = "fp32",
                 use_residual: bool = False):
        self.n_elem, self.dpe = n_elem, dofs_per_elem
        self.batch = batch
        # inputs: state and previous increment, plus R(Q_s) when use_residual
        self.use_residual = use_residual
        self.nx = (3 if use_residual else 2) * dofs_per_elem
        self.net = Mlp(self.nx, hidden, layers, dofs_per_elem, max_batch=max(n_elem, batch))
        self.net.set_compute(compute)          # 'fp32' or 'bf16' matrix products
        self.w = self.net.init_params(seed, device, zero_output=True)
        self.m1 = torch.zeros_like(self.w)
        self.m2 = torch.zeros_like(self.w)
        self.adam_step = 0
        self.rng = np.random.default_rng(seed + 1)
        self.alpha = 1.0
        self.capacity = capacity            # number of stored steps
        self.x = torch.empty(capacity * n_elem * self.nx, dtype=torch.float32, device=device)
        self.t = torch.empty(capacity * n_elem * dofs_per_elem, dtype=torch.float32, device=device)
        self.count = 0                      # stored rows
        self.step_stats = []                # field statistics of every stored step (25 device doubles)
        self.dev = device

    def correction_rms(self, q_s, dq_prev, dq):
        """Per-variable rms of dq - dq_prev (5 device doubles)."""
        return self.net.guess_stats(q_s, dq_prev, dq)[15:20].clone()

    def _r(self, r):
        if self.use_residual and r is None:
            raise ValueError("this network takes the residual R(Q_s) as an input")
        return r if self.use_residual else None

    def record(self, q_s, dq_prev, dq, r=None):
        """Add one step's (state, previous increment[, residual R(Q_s)]) -> increment samples."""
        if self.count + self.n_elem > self.capacity * self.n_elem:
            raise RuntimeError("training set is full")
        r = self._r(r)
        stats = self.net.guess_stats(q_s, dq_prev, dq, r)
        nx, nt = self.nx, self.dpe
        self.net.features(q_s, dq_prev, stats, self.n_elem,
                          x=self.x[self.count * nx:(self.count + self.n_elem) * nx], r=r)
        self.net.target(dq, dq_prev, stats, self.n_elem,
                        t=self.t[self.count * nt:(self.count + self.n_elem) * nt])
        self.step_stats.append(stats.clone())
        self.count += self.n_elem

    def copy_samples(self, other: "LearnedGuess"):
        """Take over another instance's stored training rows (same sizes)."""
        if ((other.n_elem, other.dpe, other.nx) != (self.n_elem, self.dpe, self.nx)
                or other.count > self.capacity * self.n_elem):
            raise ValueError("sample sets differ in size")
        nx, nt = self.nx, self.dpe
        self.x[:other.count * nx].copy_(other.x[:other.count * nx])
        self.t[:other.count * nt].copy_(other.t[:other.count * nt])
        self.step_stats = [st.clone() for st in other.step_stats]
        self.count = other.count

    def train(self, epochs: int, lr: float = 1e-3, holdout_rows: int = 0, alpha_rows: int | None = None):
        """Adam on minibatches of a seeded permutation; returns per-epoch mean losses
        (train) and the hold-out loss of the last `holdout_rows` stored rows.

        With a hold-out, the stored rows split into three disjoint parts: the
        training rows, then `alpha_rows` validation rows (default: as many as the
        hold-out) on which the shrinkage alpha is fitted, then the hold-out rows,
        which neither the network nor alpha has seen and which alone are scored."""
        if alpha_rows is None:
            alpha_rows = holdout_rows
        if not holdout_rows:
            alpha_rows = 0
        n_train = self.count - holdout_rows - alpha_rows
        if n_train < self.batch:
            raise ValueError("too few stored rows for training after the validation and hold-out splits")
        nx, nt = self.nx, self.dpe
        xb = torch.empty(self.batch * nx, dtype=torch.float32, device=self.dev)
        tb = torch.empty(self.batch * nt, dtype=torch.float32, device=self.dev)
        dy = torch.empty(self.batch * nt, dtype=torch.float32, device=self.dev)
        loss = torch.empty(1, dtype=torch.float64, device=self.dev)
        history = []
        for _ in range(epochs):
            perm = torch.tensor(self.rng.permutation(n_train).astype(np.int32), device=self.dev)
            total, nb = 0.0, 0
            for s in range(0, n_train - self.batch + 1, self.batch):
                idx = perm[s:s + self.batch]
                self.net.gather(self.x, nx, idx, self.batch, xb)
                self.net.gather(self.t, nt, idx, self.batch, tb)
                y = self.net.forward(self.w, xb, self.batch)
                self.net.mse(y, tb, self.batch * nt, dy=dy, loss=loss)
                dw = self.net.backward(self.w, xb, dy, self.batch)
                self.adam_step += 1
                self.net.adam(self.w, dw, self.m1, self.m2, lr=lr, step=self.adam_step)
                total += float(loss)
                nb += 1
            history.append(total / max(nb, 1))
        hold = None
        if holdout_rows:
            self.alpha = self.fit_alpha(n_train, n_train + alpha_rows)
            hold = self.loss_on(self.count - holdout_rows, self.count)
        return history, hold

    def _sums(self, row0: int, row1: int):
        """sum t^2, sum y^2 and sum t y over stored rows (from loss kernels)."""
        nx, nt = self.nx, self.dpe
        loss = torch.empty(1, dtype=torch.float64, device=self.dev)
        stt = syy = sty = 0.0
        for s in range(row0, row1, self.batch):
            b = min(self.batch, row1 - s)
            n = b * nt
            t = self.t[s * nt:(s + b) * nt]
            y = self.net.forward(self.w, self.x[s * nx:(s + b) * nx], b)
            zero = torch.zeros(n, dtype=torch.float32, device=self.dev)
            lt = float(self.net.mse(t, zero, n, loss=loss)) * n
            ly = float(self.net.mse(y, zero, n, loss=loss)) * n
            lty = float(self.net.mse(y, t, n, loss=loss)) * n
            stt, syy, sty = stt + lt, syy + ly, sty + 0.5 * (lt + ly - lty)
        return stt, syy, sty

    def fit_alpha(self, row0: int, row1: int) -> float:
        _, syy, sty = self._sums(row0, row1)
        return float(min(1.0, max(0.0, sty / syy))) if syy > 0 else 0.0

    def loss_on(self, row0: int, row1: int, zero: bool = False) -> float:
        """Mean squared error of alpha * y over stored rows [row0, row1); zero=True
        scores the zero correction, i.e. the previous increment as the prediction."""
        stt, syy, sty = self._sums(row0, row1)
        n = (row1 - row0) * self.dpe
        if zero:
            return stt / n
        a = self.alpha
        return (stt - 2 * a * sty + a * a * syy) / n

    # ---- training against the condensed residual the guess leaves ----

    def _step_rows(self, k: int):
        n, nx, nt = self.n_elem, self.nx, self.dpe
        return self.x[k * n * nx:(k + 1) * n * nx], self.t[k * n * nt:(k + 1) * n * nt]

    def _condensed_abc(self, plan, k: int):
        """For stored step k: A = |S e(y, 0)|^2, B = <S e(y, 0), S e(0, t)> and
        C = |S e(0, t)|^2 with e(y, t) = P_b (rc (y - t)), so that the loss of the
        shrunk output a y is a^2 A - 2 a B + C (three library loss evaluations)."""
        x, t = self._step_rows(k)
        st = self.step_stats[k]
        y = self.net.forward(self.w, x, self.n_elem)
        a = float(plan.guess_schur_loss(y, None, st, grad=False)[0])
        c = float(plan.guess_schur_loss(None, t, st, grad=False)[0])
        lyt = float(plan.guess_schur_loss(y, t, st, grad=False)[0])
        return a, 0.5 * (a + c - lyt), c

    def condensed_loss_on(self, plan, k: int) -> float:
        """||S P_b (rc (alpha y - t))||^2 / ||S P_b (rc t)||^2 for stored step k,
        S the plan's condensed operator (the zero correction, i.e. the previous
        increment, scores 1)."""
        a, b, c = self._condensed_abc(plan, k)
        al = self.alpha
        return (al * al * a - 2.0 * al * b + c) / c

    def train_condensed(self, plan, epochs: int, lr: float = 1e-3, holdout_steps: int = 1,
                        alpha_steps: int = 1):
        """Adam on the condensed-residual loss: GMRES started from the guess x0
        begins at b_S - S x0_b = S (Q_b - x0_b), so each stored step's loss is
        ||S P_b (rc (y - t))||^2 divided by that of the zero correction (an
        untrained network scores 1).  S couples neighbouring elements, so a batch
        is one whole step (every element), the training steps visited in a seeded
        random order each epoch.  The plan's condensed operator (the step it was
        last condensed at) weights every stored step: one S per step would not
        fit in memory at the sizes this is used at.  The last stored steps split
        as with train(): alpha_steps validation steps fit the shrinkage alpha (by
        the same weighted least squares), then holdout_steps are scored only.
        Returns per-epoch mean losses and the mean hold-out loss."""
        if not holdout_steps:
            alpha_steps = 0
        n_steps = self.count // self.n_elem
        n_train = n_steps - holdout_steps - alpha_steps
        if n_train < 1 or (holdout_steps and alpha_steps < 1):
            raise ValueError("too few stored steps for training after the validation and hold-out splits")
        den = [float(plan.guess_schur_loss(None, self._step_rows(k)[1], self.step_stats[k], grad=False)[0])
               for k in range(n_steps)]
        dy = torch.empty(self.n_elem * self.dpe, dtype=torch.float32, device=self.dev)
        loss = torch.empty(1, dtype=torch.float64, device=self.dev)
        history = []
        for _ in range(epochs):
            total = 0.0
            for k in self.rng.permutation(n_train):
                x, t = self._step_rows(int(k))
                y = self.net.forward(self.w, x, self.n_elem)
                plan.guess_schur_loss(y, t, self.step_stats[k], scale=1.0 / den[k], dy=dy, loss=loss)
                dw = self.net.backward(self.w, x, dy, self.n_elem)
                self.adam_step += 1
                self.net.adam(self.w, dw, self.m1, self.m2, lr=lr, step=self.adam_step)
                total += float(loss)
            history.append(total / n_train)
        hold = None
        if holdout_steps:
            # minimise the sum over the validation steps of (a^2 A - 2 a B + C) / C
            sa = sb = 0.0
            for k in range(n_train, n_train + alpha_steps):
                a, b, c = self._condensed_abc(plan, k)
                sa, sb = sa + a / c, sb + b / c
            self.alpha = float(min(1.0, max(0.0, sb / sa))) if sa > 0 else 0.0
            hold = float(np.mean([self.condensed_loss_on(plan, k)
                                  for k in range(n_steps - holdout_steps, n_steps)]))
        return history, hold

    def predict(self, q_s, dq_prev, rc_prev, r=None):
        """Predicted increment of the step from q_s (natural DOF order); rc_prev is
        the rms of the last known correction (see correction_rms); r = R(Q_s) for a
        network with the residual input."""
        r = self._r(r)
        stats = self.net.guess_stats(q_s, dq_prev, r=r)
        stats[15:20] = self.alpha * rc_prev
        x = self.net.features(q_s, dq_prev, stats, self.n_elem, r=r)
        y = torch.empty(self.n_elem * self.dpe, dtype=torch.float32, device=self.dev)
        mb = self.net.max_batch
        nx, nt = self.nx, self.dpe
        for s in range(0, self.n_elem, mb):
            b = min(mb, self.n_elem - s)
            self.net.forward(self.w, x[s * nx:(s + b) * nx], b, y[s * nt:(s + b) * nt])
        return self.net.apply(dq_prev, y, stats, self.n_elem)

    def close(self):
        self.net.close()
