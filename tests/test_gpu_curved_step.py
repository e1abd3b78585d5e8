"""Backward-Euler steps on curved hexahedra: the device residual with metric
terms (scdg_dg_set_geometry) drives Newton iterations whose linear systems use
the statically condensed solve of the complex-step Jacobian of the curved
discretization.

* One step equals the oracle's Newton step (oracle curved residual, global
  Jacobian from the same blocks, SuperLU) on both perturbed maps.
* Steps replayed from the captured Newton graph equal the host-orchestrated
  steps, over several steps with a fresh Jacobian each.
* FP32 factors reach the FP64 tolerance on the curved mesh.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from gpu_common import DEV, to_np
from oracle import dgsem as od
from paper_1911_02366_amd.newton import ImplicitStepper
from workload.cases import build_curved_case, curved_jacobian_blocks
from workload.curved import CurvedGeometry

pytestmark = pytest.mark.gpu


def _case(k, n, re, dt, seed, kind):
    # the generator runs on the CPU; the blocks and states move to the device
    return build_curved_case(k, n, re, dt, seed=seed, kind=kind)


def _stepper(case, **kw):
    geo = CurvedGeometry(case.mesh, case.xyz)

    def jac(q):
        blk = curved_jacobian_blocks(q.cpu(), geo, case.prm, case.dt)
        return {k: v.to(DEV) for k, v in blk.items()}
    return ImplicitStepper(case.structure(), case.mesh.k_elem, case.mesh.order, case.prm.mach,
                           case.prm.reynolds, case.dt, jac, xyz=case.xyz, **kw)


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("kind", ["sine", "skew"])
def test_curved_step_matches_oracle_newton(kind):
    case = _case(2, 3, 100.0, 1e-2, 5, kind)
    print("curved step", kind, flush=True)
    st = _stepper(case, newton_tol=1e-10, lin_tol=1e-12)
    q_s = case.q_state.reshape(-1).to(DEV).contiguous()
    st.prepare(q_s)
    q1, info = st.solve_step(q_s)
    print(info, flush=True)
    assert info["converged"] and info["newton"] >= 1, info
    grid, flow = od.Grid(2, 3), od.Flow(case.prm.mach, case.prm.reynolds)
    ja, jac = od.metric_terms(case.xyz, grid)
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col,
                               case.bb_val.numpy(), case.aii.numpy(), case.aib.numpy(), case.abi.numpy())
    lu = spla.splu(a.tocsc())
    qs = case.q_state.numpy().reshape(case.mesh.shape())
    q = qs.copy()
    r0 = np.linalg.norm(od.residual_curved(q, grid, flow, ja, jac, qs, case.dt))
    for _ in range(20):
        r = od.residual_curved(q, grid, flow, ja, jac, qs, case.dt)
        if np.linalg.norm(r) <= 1e-13 * r0:
            break
        q = q + lu.solve(-r.reshape(-1)).reshape(q.shape)
    dq_o = (q - qs).reshape(-1)
    dq = to_np(q1 - q_s)
    assert np.linalg.norm(dq - dq_o) <= 1e-8 * np.linalg.norm(dq_o)
    st.close()


def test_curved_graph_steps_match_eager_steps():
    case = _case(3, 2, 400.0, 1e-2, 2, "skew")
    st = _stepper(case, newton_tol=1e-10, lin_tol=1e-12, graph=True, autotune=False)
    q = case.q_state.reshape(-1).to(DEV).contiguous()
    for step in range(3):
        st.prepare(q)
        q_h, info_h = st.solve_step(q, graph=False)
        q_g, info_g = st.solve_step(q, graph=True)
        print(f"step {step}: host {info_h} graph {info_g}", flush=True)
        assert info_h["converged"] and info_g["converged"]
        assert abs(info_g["newton"] - info_h["newton"]) <= 1
        assert _rel(q_g - q, q_h - q) <= 1e-8
        q = q_g
    st.close()


def test_curved_fp32_factors_reach_fp64_tolerance():
    case = _case(2, 3, 400.0, 1e-2, 3, "sine")
    q_s = case.q_state.reshape(-1).to(DEV).contiguous()
    ref = _stepper(case, newton_tol=1e-11, lin_tol=1e-12, autotune=False)
    ref.prepare(q_s)
    q_ref, _ = ref.solve_step(q_s)
    ref.close()
    st = _stepper(case, newton_tol=1e-8, lin_tol=1e-10, precision="fp32", autotune=False)
    st.prepare(q_s)
    q1, info = st.solve_step(q_s)
    print("fp32 curved step", info, flush=True)
    assert info["converged"] and info["rel_res"] <= 1e-8
    assert _rel(q1 - q_s, q_ref - q_s) <= 1e-5
    st.close()


def test_graph_follows_geometry_changes():
    """Captured Newton iterations must be recaptured when the residual's geometry
    changes under the same scdg_dg object, plan and buffers: Cartesian, then
    curved (scdg_dg_set_geometry(xyz)), then Cartesian again (set_geometry(NULL)
    frees the metric terms).  Each graph step equals the host-driven step and
    zeroes the oracle's residual of the geometry in force."""
    from workload.cases import jacobian_blocks
    case = _case(2, 3, 100.0, 1e-2, 5, "sine")
    geo = CurvedGeometry(case.mesh, case.xyz)
    cart = lambda q: jacobian_blocks(q, case.mesh, case.prm, case.dt)

    def curved(q):
        blk = curved_jacobian_blocks(q.cpu(), geo, case.prm, case.dt)
        return {k: v.to(DEV) for k, v in blk.items()}

    st = ImplicitStepper(case.structure(), case.mesh.k_elem, case.mesh.order, case.prm.mach,
                         case.prm.reynolds, case.dt, cart, newton_tol=1e-10, lin_tol=1e-12, graph=True,
                         autotune=False)
    grid, flow = od.Grid(2, 3), od.Flow(case.prm.mach, case.prm.reynolds)
    ja, jac = od.metric_terms(case.xyz, grid)
    q_s = case.q_state.reshape(-1).to(DEV).contiguous()
    qs_np = to_np(q_s).reshape(case.mesh.shape())
    for phase, xyz in (("cartesian", None), ("curved", case.xyz), ("cartesian again", None)):
        print("geometry phase:", phase, flush=True)
        st.dg.set_geometry(xyz)
        st.jacobian = curved if xyz is not None else cart
        st.prepare(q_s)
        q_h, info_h = st.solve_step(q_s, graph=False)
        q_g, info_g = st.solve_step(q_s, graph=True)
        print(phase, info_h, info_g, flush=True)
        assert info_h["converged"] and info_g["converged"]
        assert _rel(q_g - q_s, q_h - q_s) <= 1e-8
        qg = to_np(q_g).reshape(case.mesh.shape())
        if xyz is None:
            r, r0 = od.residual(qg, grid, flow, qs_np, case.dt), od.residual(qs_np, grid, flow, qs_np, case.dt)
        else:
            r = od.residual_curved(qg, grid, flow, ja, jac, qs_np, case.dt)
            r0 = od.residual_curved(qs_np, grid, flow, ja, jac, qs_np, case.dt)
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(r0), phase
    st.close()
