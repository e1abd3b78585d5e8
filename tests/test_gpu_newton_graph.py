"""Newton iterations of a backward-Euler step replayed from a captured HIP graph
(scdg_newton_step): one replay = condensed right-hand side of R(Q), GMRES
restart cycles with device-side stopping, back-substitution, Q update and the
device residual R(Q).

* The result equals the host-orchestrated Newton loop (same Jacobian, same
  forcing tolerances) and the oracle's Newton step (oracle residual, global
  Jacobian from the same blocks, SuperLU).
* The graph is captured once and replayed over several steps, with eager
  library work between the steps; every replayed step is checked against the
  eager (host-orchestrated) step from the same state.
* FP32 factors: the FP64 nonlinear residual drives the iteration to the same
  tolerance.
* Starting-state rejection, the Newton budget, a GMRES cycle budget that
  leaves linear solves unconverged, and argument errors.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from gpu_common import DEV, to_np
from oracle import dgsem as od
from paper_1911_02366_amd import _lib as L
from paper_1911_02366_amd.dg import DgResidual
from paper_1911_02366_amd.newton import ImplicitStepper
from workload.cases import build_case, jacobian_blocks

pytestmark = pytest.mark.gpu


def _stepper(case, **kw):
    mesh, prm, dt = case.mesh, case.prm, case.dt
    jac = lambda q: jacobian_blocks(q, mesh, prm, dt)
    return ImplicitStepper(case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt, jac, **kw)


def _rel(a, b):
    return float((a - b).norm() / b.norm())


def test_graph_step_matches_oracle_newton():
    case = build_case(2, 3, 100.0, 1e-2, seed=5, device=DEV)
    st = _stepper(case, newton_tol=1e-10, lin_tol=1e-12, graph=True)
    q_s = case.q_state.reshape(-1).contiguous()
    st.prepare(q_s)
    q1, info = st.solve_step(q_s)
    print("graph step", info, flush=True)
    assert info["converged"] and info["newton"] >= 1, info
    grid, flow = od.Grid(2, 3), od.Flow(case.prm.mach, case.prm.reynolds)
    blk = {k: to_np(v) for k, v in jacobian_blocks(q_s.cpu(), case.mesh, case.prm, case.dt).items()}
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col,
                               blk["bb_val"], blk["aii"], blk["aib"], blk["abi"])
    lu = spla.splu(a.tocsc())
    qs = to_np(q_s).reshape(grid.k_elem, grid.k_elem, grid.k_elem, 4, 4, 4, 5)
    q = qs.copy()
    r0 = np.linalg.norm(od.residual(q, grid, flow, qs, case.dt))
    for _ in range(20):
        r = od.residual(q, grid, flow, qs, case.dt)
        if np.linalg.norm(r) <= 1e-13 * r0:
            break
        q = q + lu.solve(-r.reshape(-1)).reshape(q.shape)
    dq_o = (q - qs).reshape(-1)
    dq = to_np(q1 - q_s)
    assert np.linalg.norm(dq - dq_o) <= 1e-8 * np.linalg.norm(dq_o)
    st.close()


def test_graph_replays_match_eager_steps():
    case = build_case(3, 3, 400.0, 1e-2, seed=2, device=DEV)
    st = _stepper(case, newton_tol=1e-10, lin_tol=1e-12, graph=True, autotune=False)
    q = case.q_state.reshape(-1).contiguous()
    for step in range(4):
        st.prepare(q)
        q_h, info_h = st.solve_step(q, graph=False)      # eager library work between replays
        q_g, info_g = st.solve_step(q, graph=True)
        print(f"step {step}: host {info_h} graph {info_g}", flush=True)
        assert info_h["converged"] and info_g["converged"]
        assert abs(info_g["newton"] - info_h["newton"]) <= 1
        assert abs(info_g["gmres"] - info_h["gmres"]) <= 2 * info_h["newton"]
        assert _rel(q_g - q, q_h - q) <= 1e-8
        q = q_g
    # the graph was captured once: the key (buffers, options) never changed
    st.close()


def test_graph_fp32_factors_reach_fp64_tolerance():
    case = build_case(3, 4, 400.0, 1e-2, seed=3, device=DEV)
    q_s = case.q_state.reshape(-1).contiguous()
    ref = _stepper(case, newton_tol=1e-11, lin_tol=1e-12, autotune=False)
    ref.prepare(q_s)
    q_ref, _ = ref.solve_step(q_s)
    ref.close()
    st = _stepper(case, newton_tol=1e-8, lin_tol=1e-10, precision="fp32", graph=True, autotune=False)
    st.prepare(q_s)
    q1, info = st.solve_step(q_s)
    print("fp32 graph step", info, flush=True)
    assert info["converged"] and info["rel_res"] <= 1e-8
    # the Newton stop test bounds the state error by about kappa * 1e-8 of the increment
    assert _rel(q1 - q_s, q_ref - q_s) <= 1e-5
    st.close()


def test_graph_start_rejected_and_accepted():
    case = build_case(2, 3, 100.0, 1e-2, seed=7, device=DEV)
    st = _stepper(case, newton_tol=1e-10, lin_tol=1e-12, graph=True, autotune=False)
    q_s = case.q_state.reshape(-1).contiguous()
    st.prepare(q_s)
    q_ref, _ = st.solve_step(q_s)
    bad = torch.full_like(q_s, 0.3)
    q_b, info_b = st.solve_step(q_s, guess=bad, mode="newton")
    assert info_b["guess_rejected"] == 1 and info_b["converged"]
    assert _rel(q_b - q_s, q_ref - q_s) <= 1e-8
    good = 0.9 * (q_ref - q_s)
    q_g, info_g = st.solve_step(q_s, guess=good, mode="newton")
    assert info_g["guess_rejected"] == 0 and info_g["converged"]
    assert _rel(q_g - q_s, q_ref - q_s) <= 1e-8
    with pytest.raises(ValueError):
        st.solve_step(q_s, guess=good, mode="gmres")
    st.close()


def test_graph_budgets():
    case = build_case(2, 3, 100.0, 1e-2, seed=5, device=DEV)
    st = _stepper(case, graph=True, autotune=False)
    q_s = case.q_state.reshape(-1).contiguous()
    st.prepare(q_s)
    q = q_s.clone()
    # one Newton iteration cannot reach 1e-14
    info = st.plan.newton_step(st.dg, q_s, 1.0 / case.dt, q, check=False, newton_tol=1e-14, lin_tol=1e-12,
                               max_newton=1)
    assert info["status"] == -6 and info["newton"] == 1 and not info["converged"]
    assert 0 < info["rel_res"] < 1
    # one cycle of GMRES(4) per Newton iteration leaves the linear solves short of
    # their tolerance; the chord iteration still converges, in more iterations
    q.copy_(q_s)
    info = st.plan.newton_step(st.dg, q_s, 1.0 / case.dt, q, newton_tol=1e-9, lin_tol=1e-12, forcing=0.0,
                               restart=4, cycles=1, max_newton=200)
    print("cycle budget", info, flush=True)
    assert info["converged"] and info["lin_unconverged"] >= 1
    assert info["gmres"] <= 4 * info["newton"]
    st.close()


def test_graph_argument_errors():
    case = build_case(2, 3, 100.0, 1e-2, seed=5, device=DEV)
    st = _stepper(case, graph=True, autotune=False)
    q_s = case.q_state.reshape(-1).contiguous()
    q = q_s.clone()
    # before scdg_condense
    info = st.plan.newton_step(st.dg, q_s, 1.0 / case.dt, q, check=False)
    assert info["status"] == -2
    st.prepare(q_s)
    lib = L.load()
    o, inf = L.NewtonOpts(), L.NewtonInfo()
    # q aliasing q_s
    assert lib.scdg_newton_step(st.plan.handle, st.dg.handle, q_s.data_ptr(), 100.0, q_s.data_ptr(),
                                C.byref(o), C.byref(inf)) == -1
    # restart above 63
    o.restart = 64
    assert lib.scdg_newton_step(st.plan.handle, st.dg.handle, q_s.data_ptr(), 100.0, q.data_ptr(),
                                C.byref(o), C.byref(inf)) == -1
    # residual object of another size
    other = DgResidual(3, 3, mach=case.prm.mach, reynolds=case.prm.reynolds)
    o.restart = 0
    assert lib.scdg_newton_step(st.plan.handle, other.handle, q_s.data_ptr(), 100.0, q.data_ptr(),
                                C.byref(o), C.byref(inf)) == -1
    other.close()
    st.close()
