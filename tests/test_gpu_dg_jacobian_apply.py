"""GPU parity of the Newton-matrix product A v = M v inv_dt + dH/dQ(q) v
(scdg_dg_jacobian_apply, dual-number differentiation of the residual
kernels) against the oracle's complex-step product (oracle.dgsem.
jacobian_apply*), on perturbed Taylor-Green states (faces discontinuous, so
the Lax-Friedrichs and BR1 jump terms and their derivatives are exercised)
and random directions.

Tolerance: both sides are exact to rounding and sum the same FP64 terms in
different orders (weak form in the oracle, strong form in the kernels), as
for the residual itself; 1e-12 of max |A v| (measured: 2e-16 to 2e-15)."""
import numpy as np
import pytest
import torch

from gpu_common import DEV, to_np
from oracle import dgsem as od
from paper_1911_02366_amd import DgResidual, ScdgError
from workload import dgsem as wd
from workload.physics import FlowParams

pytestmark = pytest.mark.gpu

RTOL = 1e-12

# (elements per direction, order, Reynolds, Mach, seed)
CASES = [(2, 3, 100.0, 0.1, 1), (3, 2, 1600.0, 0.1, 2), (2, 5, 1600.0, 0.1, 3),
         (2, 7, 400.0, 0.3, 4), (3, 4, 1600.0, 0.2, 5)]
CURVED = [(2, 3, 100.0, 0.1, 6, "sine"), (3, 4, 1600.0, 0.1, 7, "skew")]


def _rel(got, want):
    return float(np.abs(got.reshape(-1) - want.reshape(-1)).max() / np.abs(want).max())


def _state(mesh, mach, re, seed, xyz=None):
    q = wd.taylor_green_state(mesh, FlowParams(mach, re), seed, coords=xyz)
    v = np.random.default_rng(seed + 50).standard_normal(q.shape)
    return q, v


@pytest.mark.parametrize("k,n,re,mach,seed", CASES)
def test_matches_oracle(k, n, re, mach, seed):
    print(f"dg jacobian_apply K={k} N={n} Re={re} Ma={mach} seed={seed}", flush=True)
    mesh = wd.Mesh(k, n)
    q, v = _state(mesh, mach, re, seed)
    grid, flow = od.Grid(k, n), od.Flow(mach, re)
    dg = DgResidual(k, n, mach=mach, reynolds=re)
    qd, vd = torch.tensor(q.reshape(-1), device=DEV), torch.tensor(v.reshape(-1), device=DEV)
    for dt in (0.25, None):
        got = to_np(dg.jacobian_apply(qd, vd, 0.0 if dt is None else 1.0 / dt))
        want = od.jacobian_apply(q, v, grid, flow, dt)
        err = _rel(got, want)
        print(f"  dt={dt} max rel err {err:.2e}", flush=True)
        assert err <= RTOL
    dg.close()


@pytest.mark.parametrize("k,n,re,mach,seed,kind", CURVED)
def test_curved_matches_oracle(k, n, re, mach, seed, kind):
    print(f"dg jacobian_apply curved {kind} K={k} N={n} seed={seed}", flush=True)
    mesh = wd.Mesh(k, n)
    xyz = wd.curved_node_coordinates(mesh, 0.05, kind)
    q, v = _state(mesh, mach, re, seed, xyz)
    grid, flow = od.Grid(k, n), od.Flow(mach, re)
    ja, jac = od.metric_terms(xyz, grid)
    dg = DgResidual(k, n, mach=mach, reynolds=re)
    dg.set_geometry(xyz)
    got = to_np(dg.jacobian_apply(torch.tensor(q.reshape(-1), device=DEV),
                                  torch.tensor(v.reshape(-1), device=DEV), 4.0))
    want = od.jacobian_apply_curved(q, v, grid, flow, ja, jac, 0.25)
    err = _rel(got, want)
    print(f"  max rel err {err:.2e}", flush=True)
    assert err <= RTOL
    dg.close()


def test_full_size_8cubed_n5():
    # the 553k-DOF order-5 workload of the implicit-step benchmark
    k, n, re, mach = 8, 5, 1600.0, 0.1
    print("dg jacobian_apply full size K=8 N=5", flush=True)
    mesh = wd.Mesh(k, n)
    q, v = _state(mesh, mach, re, 0)
    dg = DgResidual(k, n, mach=mach, reynolds=re)
    got = to_np(dg.jacobian_apply(torch.tensor(q.reshape(-1), device=DEV),
                                  torch.tensor(v.reshape(-1), device=DEV), 200.0))
    want = od.jacobian_apply(q, v, od.Grid(k, n), od.Flow(mach, re), 1.0 / 200.0)
    assert _rel(got, want) <= RTOL
    dg.close()


def test_linear_in_the_direction_and_zero_direction():
    k, n, re, mach = 2, 4, 1600.0, 0.1
    mesh = wd.Mesh(k, n)
    q, v = _state(mesh, mach, re, 9)
    dg = DgResidual(k, n, mach=mach, reynolds=re)
    qd, vd = torch.tensor(q.reshape(-1), device=DEV), torch.tensor(v.reshape(-1), device=DEV)
    a1 = dg.jacobian_apply(qd, vd, 3.0).clone()
    a2 = dg.jacobian_apply(qd, 2.0 * vd, 3.0)
    assert torch.equal(a2, 2.0 * a1)                    # scaling by 2 is exact in every dual operation
    assert bool((dg.jacobian_apply(qd, torch.zeros_like(vd), 3.0) == 0).all())
    # the residual's gradient workspace now holds the lifted gradient of q
    g = to_np(dg.gradient())
    assert _rel(g, od.lifted_gradient(q, od.Grid(k, n))) <= 1e-11
    with pytest.raises(ScdgError):
        dg.jacobian_apply(qd, vd, -1.0)
    with pytest.raises(ValueError):
        dg.jacobian_apply(qd, vd, 1.0, out=vd)
    dg.close()


@pytest.mark.parametrize("curved", [False, True])
def test_plan_blocks_are_the_derivative_of_the_device_residual(curved):
    """The element blocks a plan condenses (here from the generator, applied by
    scdg_residual with B = 0, r = -A v) and the device product agree: the
    linear solve and the nonlinear residual of a Newton step see one matrix."""
    from gpu_common import device_case, make_plan
    from workload.cases import build_case, build_curved_case
    dt = 1e-2
    case = build_curved_case(2, 3, 100.0, dt, seed=3, kind="skew") if curved else build_case(2, 3, 100.0, dt, seed=1)
    print(f"plan blocks vs dg product, curved={curved}", flush=True)
    plan = make_plan(case, device_case(case))
    q = case.q_state.to(DEV).reshape(-1).contiguous()
    v = torch.tensor(np.random.default_rng(21).standard_normal(case.n_dof), device=DEV)
    r = torch.empty_like(v)
    plan.residual(torch.zeros_like(v), v, r)
    dg = DgResidual(case.mesh.k_elem, case.mesh.order, mach=case.prm.mach, reynolds=case.prm.reynolds)
    if curved:
        dg.set_geometry(case.xyz)
    av = dg.jacobian_apply(q, v, 1.0 / dt)
    assert _rel(to_np(av), -to_np(r)) <= 1e-11
    dg.close()
    plan.close()
