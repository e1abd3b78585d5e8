"""Pins of the oracle's Newton-matrix product A v = (M/dt + dH/dQ) v
(oracle.dgsem.jacobian_apply, complex step through the residual of
eq. DGSEMsystem): it must agree with
  * the analytic chain-rule Jacobian blocks of the workload generator
    (independent code: pointwise flux Jacobians and the linear GL operators),
    assembled into the global matrix, to rounding;
  * central differences of the real-valued oracle residual, to truncation;
  * M v / dt exactly where H is flat (a uniform state moved uniformly);
and the curved form agrees with the coloured complex-step blocks of the
curved generator and with central differences.  A planted mistake (the plain
modulus in the Lax-Friedrichs speed, whose complex-step derivative is wrong)
fails the pins."""
import numpy as np
import pytest

import oracle
from oracle import dgsem as od
from workload import dgsem as wd
from workload.cases import build_case, build_curved_case
from workload.physics import FlowParams


def _global(case):
    return oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col,
                                  case.bb_val.numpy(), case.aii.numpy(), case.aib.numpy(), case.abi.numpy())


def _rel(a, b):
    return float(np.abs(a.reshape(-1) - b.reshape(-1)).max() / np.abs(b).max())


@pytest.mark.parametrize("k,n,re,seed", [(2, 3, 100.0, 1), (3, 2, 1600.0, 2)])
def test_matches_the_analytic_jacobian_blocks(k, n, re, seed):
    dt = 1e-2
    case = build_case(k, n, re, dt, seed=seed)
    q = case.q_state.numpy().reshape(case.mesh.shape())
    v = np.random.default_rng(seed + 7).standard_normal(q.shape)
    grid, flow = od.Grid(k, n), od.Flow(case.prm.mach, re)
    want = _global(case) @ v.reshape(-1)
    assert _rel(od.jacobian_apply(q, v, grid, flow, dt), want) <= 1e-12
    # without dt: the operator's Jacobian alone (the mass term removed)
    h_only = want - (np.repeat(case.mass, 5) * v.reshape(-1)) / dt
    assert _rel(od.jacobian_apply(q, v, grid, flow), h_only) <= 1e-11


def _central(fun, q, v, eps):
    return (fun(q + eps * v) - fun(q - eps * v)) / (2 * eps)


def test_matches_central_differences():
    k, n, re = 2, 4, 400.0
    mesh = wd.Mesh(k, n)
    q = wd.taylor_green_state(mesh, FlowParams(0.1, re), 3)
    v = np.random.default_rng(5).standard_normal(q.shape)
    grid, flow = od.Grid(k, n), od.Flow(0.1, re)
    got = od.jacobian_apply(q, v, grid, flow)
    fd = _central(lambda z: od.operator_h(z, grid, flow), q, v, 1e-6)
    assert _rel(got, fd) <= 1e-6
    # the viscous part is visible at this Reynolds number: dropping it is caught
    fd_inviscid = _central(lambda z: od.operator_h(z, grid, od.Flow(0.1, 1e12)), q, v, 1e-6)
    assert _rel(got, fd_inviscid) > 1e-4


def test_uniform_state_moved_uniformly_gives_the_mass_term():
    k, n, dt = 2, 3, 0.05
    mesh = wd.Mesh(k, n)
    q = wd.uniform_state(mesh, FlowParams(0.1, 100.0))
    v = np.broadcast_to(np.array([0.3, -0.2, 0.1, 0.4, 2.0]), q.shape).copy()
    grid, flow = od.Grid(k, n), od.Flow(0.1, 100.0)
    want = od.mass(grid)[..., None] * v / dt
    assert _rel(od.jacobian_apply(q, v, grid, flow, dt), want) <= 1e-12


def test_curved_matches_generator_blocks_and_differences():
    dt = 1e-2
    case = build_curved_case(2, 3, 100.0, dt, seed=3, kind="skew")
    grid, flow = od.Grid(2, 3), od.Flow(0.1, 100.0)
    ja, jac = od.metric_terms(case.xyz, grid)
    q = case.q_state.numpy().reshape(case.mesh.shape())
    v = np.random.default_rng(11).standard_normal(q.shape)
    got = od.jacobian_apply_curved(q, v, grid, flow, ja, jac, dt)
    assert _rel(got, _global(case) @ v.reshape(-1)) <= 1e-11
    fd = _central(lambda z: od.residual_curved(z, grid, flow, ja, jac, q, dt), q, v, 1e-6)
    assert _rel(got, fd) <= 1e-6


def test_planted_plain_modulus_fails_the_pins(monkeypatch):
    # np.abs of a complex-step argument is its modulus: the imaginary part (the
    # derivative of |v.n|) is lost, so the Lax-Friedrichs speed looks constant
    k, n, re, seed, dt = 2, 3, 100.0, 1, 1e-2
    case = build_case(k, n, re, dt, seed=seed)
    q = case.q_state.numpy().reshape(case.mesh.shape())
    v = np.random.default_rng(seed + 7).standard_normal(q.shape)
    grid, flow = od.Grid(k, n), od.Flow(case.prm.mach, re)
    want = _global(case) @ v.reshape(-1)
    monkeypatch.setattr(od, "_abs", np.abs)
    assert _rel(od.jacobian_apply(q, v, grid, flow, dt), want) > 1e-8
