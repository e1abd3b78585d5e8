"""The symmetric interior penalty (SIPG) viscous flux on the device: the
residual R(Q) and the Newton-matrix product A v (scdg_dg_* with
SCDG_VISCOUS_SIPG) against the oracle, the condensed solve of the SIPG
Jacobian against the oracle's uncondensed solve, and implicit Newton steps
with the SIPG residual against the oracle's Newton step.

Tolerances as for the Bassi-Rebay 1 operators: residual 1e-11 and products
1e-12 of the largest entry (both sides FP64, sums in different orders);
condensed solve 1e-10 relative; Newton steps 1e-8 of the increment."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from gpu_common import DEV, rel, to_np
from oracle import dgsem as od
from paper_1911_02366_amd import DgResidual, Plan
from paper_1911_02366_amd import _lib as L
from paper_1911_02366_amd.newton import ImplicitStepper
from workload import dgsem as wd
from workload.curved import CurvedGeometry, CurvedJacobianParts
from workload.physics import FlowParams
from workload.walls import partition_general

pytestmark = pytest.mark.gpu

CASES = [(2, 3, 100.0, 0.1, 1), (3, 2, 1600.0, 0.1, 2), (2, 5, 1600.0, 0.1, 3), (2, 7, 400.0, 0.3, 4),
         (3, 4, 1600.0, 0.2, 5)]


def _maxrel(got, want):
    return float(np.abs(got.reshape(-1) - want.reshape(-1)).max() / np.abs(want).max())


@pytest.mark.parametrize("k,n,re,mach,seed", CASES)
def test_sipg_residual_and_product_match_oracle(k, n, re, mach, seed):
    print(f"sipg residual K={k} N={n} Re={re} Ma={mach}", flush=True)
    mesh = wd.Mesh(k, n)
    q = wd.taylor_green_state(mesh, FlowParams(mach, re), seed)
    qs = wd.taylor_green_state(mesh, FlowParams(mach, re), seed + 9)
    v = np.random.default_rng(seed + 50).standard_normal(q.shape)
    grid, flow = od.Grid(k, n), od.Flow(mach, re)
    dg = DgResidual(k, n, mach=mach, reynolds=re, viscous="sipg")
    qd, qsd, vd = (torch.tensor(a.reshape(-1), device=DEV) for a in (q, qs, v))
    r = to_np(dg.residual(qd, qsd, 1.0 / 0.01))
    assert _maxrel(r, od.residual(q, grid, flow, qs, 0.01, viscous="sipg")) <= 1e-11
    av = to_np(dg.jacobian_apply(qd, vd, 1.0 / 0.25))
    assert _maxrel(av, od.jacobian_apply(q, v, grid, flow, 0.25, viscous="sipg")) <= 1e-12
    # BR1 and SIPG differ on these discontinuous states
    br = DgResidual(k, n, mach=mach, reynolds=re)
    assert _maxrel(to_np(br.residual(qd, qsd, 100.0)), r) > 1e-8
    br.close()
    # the allocation-free product covers the Bassi-Rebay 1 flux only
    out = torch.empty_like(qd)
    st = L.load().scdg_dg_jacobian_apply_noalloc(dg.handle, C.c_void_p(qd.data_ptr()), C.c_void_p(vd.data_ptr()),
                                                 C.c_double(1.0), C.c_void_p(out.data_ptr()))
    assert st == -8
    dg.close()


def _sipg_blocks(case_q, mesh, prm, dt):
    geo = CurvedGeometry(mesh, wd.curved_node_coordinates(mesh, 0.0), device=DEV)
    parts = CurvedJacobianParts(case_q.to(DEV), geo, prm, dt, viscous="sipg")
    return partition_general(parts.own, parts.couplings(), mesh.order, np.zeros(mesh.n_elem, dtype=np.uint8))


@pytest.mark.parametrize("k,n", [(2, 3), (3, 4)])
def test_sipg_condensed_solve_matches_oracle(k, n):
    print(f"sipg condensed solve K={k} N={n}", flush=True)
    mesh, prm, dt = wd.Mesh(k, n), FlowParams(0.1, 400.0), 1e-2
    q = torch.tensor(wd.taylor_green_state(mesh, prm, 7), dtype=torch.float64)
    blk = _sipg_blocks(q, mesh, prm, dt)
    b = -od.residual(q.numpy(), od.Grid(k, n), od.Flow(0.1, 400.0), viscous="sipg").reshape(-1)
    order = np.full(mesh.n_elem, n, dtype=np.int32)
    ni, nc = blk["n_i"], blk["n_c"]
    oi, oc = np.concatenate([[0], np.cumsum(ni * ni)]), np.concatenate([[0], np.cumsum(ni * nc)])
    t = lambda x: to_np(x)
    aii = [t(blk["aii"])[oi[e]:oi[e + 1]].reshape(ni[e], ni[e]) for e in range(mesh.n_elem)]
    aib = [t(blk["aib"])[oc[e]:oc[e + 1]].reshape(ni[e], nc[e]) for e in range(mesh.n_elem)]
    abi = [t(blk["abi"])[oc[e]:oc[e + 1]].reshape(nc[e], ni[e]) for e in range(mesh.n_elem)]
    a = oracle.assemble_global(order, blk["c_ptr"], blk["c_node"], blk["bb_rowptr"], blk["bb_col"],
                               t(blk["bb_val"]), aii, aib, abi)
    ref = oracle.solve_sparse(a, b)
    plan = Plan(order, blk["c_ptr"], blk["c_node"], blk["bb_rowptr"], blk["bb_col"])
    plan.assemble(blk["aii"], blk["aib"], blk["abi"], blk["bb_val"])
    plan.factor("fp64")
    plan.condense()
    bd = torch.tensor(b, device=DEV)
    for solver in ("dense", "gmres"):
        if solver == "dense" and plan.n1 > 8192:
            continue
        dq, info = plan.solve(bd, solver=solver, tol=1e-13, ir_tol=1e-12)
        print(solver, info, flush=True)
        assert rel(to_np(dq), ref) <= 1e-10
    # the blocks the plan condenses are the device SIPG Newton matrix
    dg = DgResidual(k, n, mach=0.1, reynolds=400.0, viscous="sipg")
    v = torch.randn(mesh.n_dof, dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(3))
    av = dg.jacobian_apply(q.reshape(-1).to(DEV), v, 1.0 / dt)
    r = torch.empty_like(v)
    plan.residual(torch.zeros_like(v), v, r)                     # r = 0 - A v
    assert float((av + r).abs().max() / av.abs().max()) <= 1e-11
    dg.close()
    plan.close()


def test_sipg_newton_step_matches_oracle():
    k, n, dt = 2, 3, 1e-2
    mesh, prm = wd.Mesh(k, n), FlowParams(0.1, 100.0)
    q0 = torch.tensor(wd.taylor_green_state(mesh, prm, 5), dtype=torch.float64)

    def jac(q):
        blk = _sipg_blocks(q.detach().cpu().reshape(mesh.shape()), mesh, prm, dt)
        return {key: blk[key] for key in ("aii", "aib", "abi", "bb_val")}

    blk0 = _sipg_blocks(q0, mesh, prm, dt)
    st = dict(order=np.full(mesh.n_elem, n, dtype=np.int32), c_ptr=blk0["c_ptr"], c_node=blk0["c_node"],
              bb_rowptr=blk0["bb_rowptr"], bb_col=blk0["bb_col"])
    q_s = q0.reshape(-1).to(DEV).contiguous()
    grid, flow = od.Grid(k, n), od.Flow(0.1, 100.0)
    for graph in (False, True):
        stp = ImplicitStepper(st, k, n, 0.1, 100.0, dt, jac, newton_tol=1e-10, lin_tol=1e-12, graph=graph,
                              autotune=False, viscous="sipg")
        stp.prepare(q_s)
        q1, info = stp.solve_step(q_s)
        print("sipg step graph" if graph else "sipg step host", info, flush=True)
        assert info["converged"]
        a = oracle.assemble_global(st["order"], st["c_ptr"], st["c_node"], st["bb_rowptr"], st["bb_col"],
                                   *_host_blocks(blk0))
        lu = spla.splu(a.tocsc())
        qs = q0.numpy()
        q = qs.copy()
        r0 = np.linalg.norm(od.residual(q, grid, flow, qs, dt, viscous="sipg"))
        for _ in range(20):
            r = od.residual(q, grid, flow, qs, dt, viscous="sipg")
            if np.linalg.norm(r) <= 1e-13 * r0:
                break
            q = q + lu.solve(-r.reshape(-1)).reshape(q.shape)
        dq_o = (q - qs).reshape(-1)
        assert np.linalg.norm(to_np(q1 - q_s) - dq_o) <= 1e-8 * np.linalg.norm(dq_o)
        stp.close()


def _host_blocks(blk):
    ni, nc = blk["n_i"], blk["n_c"]
    ne = len(ni)
    oi, oc = np.concatenate([[0], np.cumsum(ni * ni)]), np.concatenate([[0], np.cumsum(ni * nc)])
    t = lambda x: to_np(x)
    return (t(blk["bb_val"]), [t(blk["aii"])[oi[e]:oi[e + 1]].reshape(ni[e], ni[e]) for e in range(ne)],
            [t(blk["aib"])[oc[e]:oc[e + 1]].reshape(ni[e], nc[e]) for e in range(ne)],
            [t(blk["abi"])[oc[e]:oc[e + 1]].reshape(nc[e], ni[e]) for e in range(ne)])
