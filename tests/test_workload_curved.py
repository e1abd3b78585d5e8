"""The curved-mesh implicit-step generator (workload.curved): H(Q) and the
metric terms equal the oracle's curved residual, and the Jacobian blocks
linearize the oracle's curved R(Q) (central differences), including colour
classes that hold several elements (K = 6)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import dgsem as od
from workload import curved as wc
from workload.cases import build_curved_case, global_matrix_from_parts
from workload.dgsem import Mesh, curved_node_coordinates, taylor_green_state, uniform_state
from workload.jacobian import JacobianParts
from workload.physics import FlowParams


def _fd(q, grid, flow, ja, jac, dt, v, eps=1e-6):
    rp = od.residual_curved(q + eps * v, grid, flow, ja, jac, q, dt)
    rm = od.residual_curved(q - eps * v, grid, flow, ja, jac, q, dt)
    return ((rp - rm) / (2 * eps)).reshape(-1)


@pytest.mark.parametrize("kind", ["sine", "skew"])
def test_curved_h_matches_oracle(kind):
    mesh, prm = Mesh(2, 3), FlowParams(mach=0.1, reynolds=100.0)
    xyz = curved_node_coordinates(mesh, 0.05, kind)
    q = taylor_green_state(mesh, prm, 4, coords=xyz)
    geo = wc.CurvedGeometry(mesh, xyz)
    grid, flow = od.Grid(2, 3), od.Flow(0.1, 100.0)
    ja, jac = od.metric_terms(xyz, grid)
    np.testing.assert_allclose(geo.ja.numpy(), ja, rtol=0, atol=1e-12)
    np.testing.assert_allclose(geo.jac.numpy(), jac, rtol=0, atol=1e-12)
    h_o = od.operator_h_curved(q, grid, flow, ja, jac)
    h_t = wc.operator_h(torch.tensor(q), geo, prm).numpy()
    assert np.abs(h_t - h_o).max() <= 1e-12 * np.abs(h_o).max()
    # batched complex evaluation: the real part is H, per batch entry
    qc = torch.tensor(q).to(torch.complex128).expand((2,) + q.shape)
    np.testing.assert_allclose(wc.operator_h(qc, geo, prm).real.numpy()[1], h_t, rtol=0, atol=1e-12)


def test_curved_jacobian_blocks_linearize_oracle_residual():
    dt = 1e-2
    case = build_curved_case(2, 3, 100.0, dt, seed=3, kind="skew")
    grid, flow = od.Grid(2, 3), od.Flow(0.1, 100.0)
    ja, jac = od.metric_terms(case.xyz, grid)
    q = case.q_state.numpy().reshape(case.mesh.shape())
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col,
                               case.bb_val.numpy(), case.aii.numpy(), case.aib.numpy(), case.abi.numpy())
    v = np.random.default_rng(12).standard_normal(q.shape)
    fd = _fd(q, grid, flow, ja, jac, dt, v)
    av = a @ v.reshape(-1)
    assert np.abs(av - fd).max() <= 1e-6 * np.abs(av).max()
    np.testing.assert_allclose(case.rhs.numpy(), -od.operator_h_curved(q, grid, flow, ja, jac).reshape(-1),
                               rtol=0, atol=1e-12 * np.abs(case.rhs.numpy()).max())
    np.testing.assert_allclose(case.mass, od.curved_mass(grid, jac).reshape(-1), rtol=1e-14)
    # the Cartesian Jacobian of the same state misses the metric terms: the pin sees the geometry
    cart = global_matrix_from_parts(JacobianParts(case.q_state, case.mesh, case.prm, dt))
    assert np.abs(cart @ v.reshape(-1) - fd).max() > 1e-3 * np.abs(av).max()


def test_curved_jacobian_colour_classes_with_several_elements():
    """K = 6: colour classes of 8 elements, 3 elements apart (order 1 keeps it
    small).  The state is a uniform flow with a seeded 1% perturbation, so no
    normal velocity or wave-speed comparison sits at the kink of |.| or max
    within the central-difference step.  Two elements of one class writing to
    the same row would show as O(1) errors against the central differences."""
    dt = 5e-3
    mesh, prm = Mesh(6, 1), FlowParams(mach=0.1, reynolds=400.0)
    assert wc._colour_modulus(6) == 3 and wc._colour_modulus(4) == 4 and wc._colour_modulus(2) == 2
    xyz = curved_node_coordinates(mesh, 0.05, "sine")
    q = uniform_state(mesh, prm) * (1.0 + 0.01 * np.random.default_rng(9).standard_normal(mesh.shape()))
    geo = wc.CurvedGeometry(mesh, xyz)
    a = global_matrix_from_parts(wc.CurvedJacobianParts(torch.tensor(q), geo, prm, dt))
    grid, flow = od.Grid(6, 1), od.Flow(0.1, 400.0)
    ja, jac = od.metric_terms(xyz, grid)
    v = np.random.default_rng(13).standard_normal(q.shape)
    av = a @ v.reshape(-1)
    assert np.abs(av - _fd(q, grid, flow, ja, jac, dt, v)).max() <= 1e-6 * np.abs(av).max()
    # every column of one element reaches rows of its own 3x3x3 neighbourhood only
    p3 = 8
    rows, cols = a.nonzero()
    er, ec = rows // (5 * p3), cols // (5 * p3)
    d = [np.minimum((er // 6 ** s % 6 - ec // 6 ** s % 6) % 6, (ec // 6 ** s % 6 - er // 6 ** s % 6) % 6)
         for s in range(3)]
    assert max(int(x.max()) for x in d) == 1


def test_curved_geometry_rejects_folded_map():
    mesh = Mesh(2, 2)
    xyz = curved_node_coordinates(mesh, 0.05, "sine")
    with pytest.raises(ValueError):
        wc.CurvedGeometry(mesh, xyz[..., ::-1].copy())       # mirrored map: J < 0
    with pytest.raises(ValueError):
        wc.CurvedGeometry(mesh, xyz[:, :, :, :2])
