"""Physical boundaries in the oracle and the generator: isothermal no-slip walls
on the two domain faces normal to one direction (Section 2.1.1: the outer state
of a boundary face is a function q^-(q^+) of the inner one; Section 3.2: the
DOFs of nodes lying only on physical faces join Q_i, the achievable ratio).

Pins: the wall state 1/2 (q^+ + q^-) is at rest at the wall temperature for any
inner state; a fluid at rest at the wall temperature stays steady; mass is
conserved exactly (no mass crosses a wall) and the other variables change only
by the wall fluxes; the lifted gradient of a continuous polynomial state that
satisfies the wall condition is exact; the complex-step Jacobian agrees with
central differences; the achievable ratio's closed form equals the node count;
the condensed solve with wall DOFs in Q_i equals the uncondensed brute force;
the generator's residual and Jacobian blocks equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from oracle import dgsem as od
from workload import dgsem as wd
from workload.curved import CurvedGeometry, operator_h as gen_h
from workload.physics import FlowParams
from workload.walls import build_wall_case, interior_mask

FLOW = od.Flow(0.1, 100.0)


def _tgv(k, n, seed=1, re=100.0):
    return wd.taylor_green_state(wd.Mesh(k, n), FlowParams(0.1, re), seed)


def test_wall_state_is_at_rest_at_wall_temperature():
    rng = np.random.default_rng(0)
    q = _tgv(2, 3).reshape(-1, 5)[:50]
    q = q + 0.01 * rng.standard_normal(q.shape) * np.abs(q)
    for t_wall in (1.0, 1.3):
        qw = 0.5 * (q + od.wall_ghost(q, FLOW, t_wall))
        _, vel, _, _, temp = od.primitive(qw, FLOW)
        assert np.abs(vel).max() == 0.0
        assert np.abs(temp - t_wall).max() <= 1e-13
    # planted mistake: momentum copied instead of reversed
    bad = od.wall_ghost(q, FLOW, 1.0)
    bad[:, 1:4] = q[:, 1:4]
    assert np.abs(od.primitive(0.5 * (q + bad), FLOW)[1]).max() > 1e-3


@pytest.mark.parametrize("d", [0, 1, 2])
def test_rest_state_at_wall_temperature_is_steady(d):
    grid = od.Grid(2, 3)
    e_w = 1.0 / (FLOW.gamma * (FLOW.gamma - 1.0) * FLOW.mach ** 2)
    q = np.zeros((2, 2, 2, 4, 4, 4, 5))
    q[..., 0] = 1.2
    q[..., 4] = 1.2 * e_w
    h = od.operator_h(q, grid, FLOW, od.Walls(d, 1.0))
    assert np.abs(h).max() <= 1e-13 * q[..., 4].max()


@pytest.mark.parametrize("d", [0, 2])
def test_mass_conserved_and_wall_flux_balance(d):
    k, n = 3, 3
    grid, walls = od.Grid(k, n), od.Walls(d, 1.0)
    q = _tgv(k, n)
    h = od.operator_h(q, grid, FLOW, walls)
    total = h.reshape(-1, 5).sum(0)
    scale = np.abs(h).reshape(-1, 5).sum(0)
    assert abs(total[0]) <= 1e-13 * scale[0]
    # the other variables change by the fluxes through the two walls alone
    g = od.lifted_gradient(q, grid, walls, FLOW)
    f_hi, f_lo = od.wall_fluxes(q, g, d, FLOW, walls)
    _, w = od.gl_rule(n)
    ct = (grid.h / 2.0) ** 2 * np.outer(w, w)[..., None]
    expected = (ct * f_hi).reshape(-1, 5).sum(0) - (ct * f_lo).reshape(-1, 5).sum(0)
    assert np.all(np.abs(total - expected) <= 1e-12 * scale)
    assert np.abs(expected[1:]).max() > 1e-6          # the walls do act
    # periodic mesh: every variable conserved (the balance reduces to zero)
    hp = od.operator_h(q, grid, FLOW).reshape(-1, 5).sum(0)
    assert np.all(np.abs(hp) <= 1e-12 * scale)


def test_lifted_gradient_exact_for_polynomial_state_meeting_the_wall_condition():
    # at rest at the wall temperature everywhere, density quadratic in the wall
    # direction: continuous across elements and equal to its wall state at the walls
    k, n = 3, 3
    grid, walls = od.Grid(k, n), od.Walls(2, 1.0)
    z = wd.node_coordinates(wd.Mesh(k, n))[..., 2]
    e_w = 1.0 / (FLOW.gamma * (FLOW.gamma - 1.0) * FLOW.mach ** 2)
    rho = 1.0 + 0.1 * z + 0.02 * z * z
    q = np.zeros(z.shape + (5,))
    q[..., 0], q[..., 4] = rho, rho * e_w
    g = od.lifted_gradient(q, grid, walls, FLOW)
    drho = 0.1 + 0.04 * z
    assert np.abs(g[..., 2, 0] - drho).max() <= 1e-12
    assert np.abs(g[..., 2, 4] - e_w * drho).max() <= 1e-12 * e_w
    assert np.abs(g[..., :2, :]).max() <= 1e-12 * e_w
    # the same state on a periodic mesh jumps across the wrap: not exact there
    gp = od.lifted_gradient(q, grid)
    assert np.abs(gp[..., 2, 0] - drho).max() > 1e-3


def test_wall_jacobian_complex_step_matches_central_differences():
    grid, walls = od.Grid(2, 2), od.Walls(2, 1.0)
    q = _tgv(2, 2)
    v = np.random.default_rng(3).standard_normal(q.shape)
    av = od.jacobian_apply(q, v, grid, FLOW, 1e-2, walls)
    eps = 1e-9 * np.abs(q).max() / np.abs(v).max()     # small: |v . n| at a wall is O(1e-3)
    fd = (od.residual(q + eps * v, grid, FLOW, q, 1e-2, walls) -
          od.residual(q - eps * v, grid, FLOW, q, 1e-2, walls)) / (2 * eps)
    assert np.abs(av - fd).max() <= 1e-6 * np.abs(av).max()
    # mass conservation differentiated: the mass rows of dH/dQ sum to zero column by column
    dh = od.jacobian_apply(q, v, grid, FLOW, None, walls)
    assert abs(dh[..., 0].sum()) <= 1e-12 * np.abs(dh[..., 0]).sum()


@pytest.mark.parametrize("k,n", [(2, 3), (4, 5), (8, 5), (3, 7)])
def test_achievable_ratio_closed_form(k, n):
    worst = (6 * n * n + 2) / (n + 1) ** 3                  # Table ratio, d = 3
    assert oracle.achievable_ratio(k, n, ()) == pytest.approx(worst, rel=1e-15)
    # walls normal to one direction: (N - 1)^2 face-interior nodes of each of 2 K^2 wall faces move to Q_i
    closed = (k ** 3 * ((n + 1) ** 3 - (n - 1) ** 3) - 2 * k * k * (n - 1) ** 2) / (k ** 3 * (n + 1) ** 3)
    assert oracle.achievable_ratio(k, n) == pytest.approx(closed, rel=1e-15)
    assert oracle.achievable_ratio(k, n) < worst
    # and from the node sets the condensation uses
    masks = od.wall_face_mask(k, od.Walls(2, 1.0))
    n_int = sum(len(oracle.node_sets(n, int(m)).interior) for m in masks)
    assert 1.0 - n_int / (k ** 3 * (n + 1) ** 3) == pytest.approx(closed, rel=1e-15)


def test_interior_sets_agree_between_oracle_and_generator():
    for n in (2, 3, 5):
        for m in (0, 16, 32, 48, 1 | 8, 63):
            a = np.zeros((n + 1) ** 3, dtype=bool)
            a[oracle.node_sets(n, m).interior] = True
            assert np.array_equal(a, interior_mask(n, m)), (n, m)


@pytest.mark.parametrize("d", [0, 2])
def test_generator_residual_equals_oracle(d):
    k, n = 3, 2
    mesh = wd.Mesh(k, n)
    q = _tgv(k, n)
    geo = CurvedGeometry(mesh, wd.curved_node_coordinates(mesh, 0.0))
    h = gen_h(torch.tensor(q), geo, FlowParams(0.1, 100.0), (d, 1.0)).numpy()
    ho = od.operator_h(q, od.Grid(k, n), FLOW, od.Walls(d, 1.0))
    assert np.abs(h - ho).max() <= 1e-12 * np.abs(ho).max()


@pytest.fixture(scope="module")
def wall_case():
    return build_wall_case(2, 3, 100.0, 1e-2, seed=5)


def test_wall_blocks_linearize_the_oracle_residual(wall_case):
    c = wall_case
    eb = c.element_blocks()
    a = oracle.assemble_global(c.order, c.c_ptr, c.c_node, c.bb_rowptr, c.bb_col, eb["bb_val"], eb["aii"],
                               eb["aib"], eb["abi"], phys=c.phys_faces)
    q = c.q_state.numpy().reshape(c.mesh.shape())
    v = np.random.default_rng(1).standard_normal(q.shape)
    av = od.jacobian_apply(q, v, od.Grid(2, 3), FLOW, c.dt, od.Walls(2, 1.0))
    assert np.abs(a @ v.reshape(-1) - av.reshape(-1)).max() <= 1e-12 * np.abs(av).max()
    b = od.residual(q, od.Grid(2, 3), FLOW, q, c.dt, od.Walls(2, 1.0))
    assert np.abs(c.rhs.numpy() + b.reshape(-1)).max() <= 1e-12 * np.abs(b).max()


def test_wall_condensed_equals_uncondensed(wall_case):
    c = wall_case
    assert c.n1 / (c.n1 + c.n2) == pytest.approx(oracle.achievable_ratio(2, 3), rel=1e-15)
    eb = c.element_blocks()
    args = (c.order, c.c_ptr, c.c_node, c.bb_rowptr, c.bb_col, eb["bb_val"], eb["aii"], eb["aib"], eb["abi"])
    a = oracle.assemble_global(*args, phys=c.phys_faces)
    x = oracle.solve_dense(a, c.rhs.numpy())
    xs = oracle.condensed_solve_dense(*args, c.rhs.numpy(), phys=c.phys_faces)
    assert np.linalg.norm(xs - x) <= 1e-12 * np.linalg.norm(x)
    # planted mistake: wall DOFs classified as boundary with the same blocks -> the maps disagree
    with pytest.raises(Exception):
        oracle.assemble_global(*args)


def test_general_partition_reproduces_the_periodic_partition():
    # no physical face: the pattern-derived coupling sets and blocks equal the
    # closed-form periodic partition of the analytic generator
    from workload.cases import build_case
    from workload.curved import CurvedJacobianParts
    from workload.walls import partition_general
    ref = build_case(2, 3, 100.0, 1e-2, seed=5)
    mesh = ref.mesh
    geo = CurvedGeometry(mesh, wd.curved_node_coordinates(mesh, 0.0))
    parts = CurvedJacobianParts(ref.q_state, geo, ref.prm, ref.dt)
    blk = partition_general(parts.own, parts.couplings(), 3, np.zeros(8, dtype=np.uint8))
    assert np.array_equal(blk["c_ptr"], ref.c_ptr) and np.array_equal(blk["c_node"], ref.c_node)
    assert np.array_equal(blk["bb_rowptr"], ref.bb_rowptr) and np.array_equal(blk["bb_col"], ref.bb_col)
    for k in ("aii", "aib", "abi"):
        r = getattr(ref, k).reshape(-1)
        assert float((blk[k] - r).abs().max()) <= 1e-12 * float(r.abs().max()), k
    assert float((blk["bb_val"] - ref.bb_val).abs().max()) <= 1e-12 * float(ref.bb_val.abs().max())
