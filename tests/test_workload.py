"""Pins of the synthetic GL-DGSEM Navier-Stokes system that feeds both the oracle
and the HIP path: free stream, discrete conservation, weak = strong form, exact
lifted gradients, and the analytic Jacobian against complex-step differentiation
of the full residual."""
import json
import os

import numpy as np
import pytest
import torch

from workload import dgsem
from workload.cases import build_case, global_matrix_from_parts
from workload.dgsem import Mesh, residual, taylor_green_state, uniform_state, lifted_gradient
from workload.jacobian import JacobianParts
from workload.partition import coupling_size, local_sets
from workload.physics import FlowParams

PRM = FlowParams(mach=0.1, reynolds=100.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2), (2, 5)])
def test_free_stream_preserved(k, n):
    mesh = Mesh(k, n)
    q = torch.tensor(uniform_state(mesh, PRM))
    h = residual(q, mesh, PRM)
    scale = float(torch.abs(q).max()) * mesh.jac * mesh.scale
    assert float(h.abs().max()) < 1e-13 * scale * 10


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2), (2, 4)])
def test_conservation_and_weak_equals_strong(k, n):
    mesh = Mesh(k, n)
    q = torch.tensor(taylor_green_state(mesh, PRM, seed=3))
    h = residual(q, mesh, PRM)
    hs = residual(q, mesh, PRM, form="strong")
    tot = h.reshape(-1, 5).sum(0)
    mag = h.reshape(-1, 5).abs().sum(0)
    assert torch.all(tot.abs() <= 1e-13 * mag + 1e-15)
    assert float((h - hs).abs().max()) <= 1e-12 * float(h.abs().max())


@pytest.mark.parametrize("n", [2, 3, 4])
def test_lifted_gradient_exact_for_continuous_polynomial(n):
    # q_0 = x^n is continuous across the faces of the middle element column of a
    # 3^3 mesh, so the BR1 lifted gradient there equals the exact derivative.
    mesh = Mesh(3, n)
    xyz = dgsem.node_coordinates(mesh)
    q = np.ones(mesh.shape())
    q[..., 0] = xyz[..., 0] ** n
    q[..., 4] = xyz[..., 1] ** n
    g = lifted_gradient(torch.tensor(q), mesh)
    mid = (slice(None), slice(None), 1)
    np.testing.assert_allclose(g[0][mid][..., 0].numpy(), (n * xyz[..., 0] ** (n - 1))[mid], rtol=1e-11)
    np.testing.assert_allclose(g[1][mid][..., 0].numpy(), 0.0, atol=1e-10)
    midy = (slice(None), 1)
    np.testing.assert_allclose(g[1][midy][..., 4].numpy(), (n * xyz[..., 1] ** (n - 1))[midy], rtol=1e-11)


def _complex_step_jacobian(q, mesh):
    qc = q.to(torch.complex128).reshape(-1)
    n = qc.numel()
    jac = np.zeros((n, n))
    for c in range(n):
        qp = qc.clone()
        qp[c] += 1e-30j
        jac[:, c] = (residual(qp.reshape(mesh.shape()), mesh, PRM).imag / 1e-30).reshape(-1).numpy()
    return jac


@pytest.mark.parametrize("k,n", [(2, 2), pytest.param(3, 2, marks=pytest.mark.slow)])
def test_analytic_jacobian_matches_complex_step(k, n):
    mesh = Mesh(k, n)
    q = torch.tensor(taylor_green_state(mesh, PRM, seed=1))
    parts = JacobianParts(q, mesh, PRM, dt=1.0)
    a = global_matrix_from_parts(parts).toarray()
    m = np.repeat(dgsem.mass_diagonal(mesh).reshape(-1), 5)
    a -= np.diag(m)                       # dt = 1: remove M / dt
    jac = _complex_step_jacobian(q, mesh)
    assert np.abs(a - jac).max() <= 1e-13 * np.abs(jac).max()


def test_jacobian_column_sums_vanish(case_n3k2):
    # differentiating sum_j H_{j,v}(Q) = 0 gives 1_v^T dH/dQ = 0 for every column
    c = case_n3k2
    a = global_matrix_from_parts(c.parts)
    m = np.repeat(c.mass, 5) / c.dt
    dh = a - __import__("scipy.sparse", fromlist=["diags"]).diags(m)
    sums = np.asarray(dh.reshape(-1).tocsr().toarray()) if False else None
    colsum = np.zeros((5, dh.shape[1]))
    coo = dh.tocoo()
    np.add.at(colsum, (coo.row % 5, coo.col), coo.data)
    scale = np.abs(coo.data).max()
    assert np.abs(colsum).max() <= 1e-13 * scale


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7])
def test_coupling_set_size_and_ratio(n):
    golden = json.load(open(os.path.join(GOLDEN, "condensed_ratio.json")))
    ls = local_sets(n)
    nb, ni = len(ls["b_loc"]), len(ls["i_loc"])
    num, den = golden["d3_values"][str(n)]
    assert nb * den == num * (n + 1) ** 3 and nb + ni == (n + 1) ** 3
    assert coupling_size(n) == (n + 1) ** 3 - (n - 1) ** 3 - 8 + 6 * (n - 1) ** 2


@pytest.mark.parametrize("k,n", [(2, 2), (3, 3), (2, 4)])
def test_partition_sizes_and_block_diagonal_aii(k, n):
    # partition() raises if an interior DOF couples across elements or outside C_e
    c = build_case(k, n, 100.0, 1e-2)
    assert c.n_i == 5 * (n - 1) ** 3
    assert c.n_c == 5 * coupling_size(n)
    assert c.n1 * (n + 1) ** 3 == (c.n1 + c.n2) * (6 * n * n + 2)
    assert c.aii.shape == (k ** 3, c.n_i, c.n_i)
    assert c.aib.shape == (k ** 3, c.n_i, c.n_c) and c.abi.shape == (k ** 3, c.n_c, c.n_i)
    # every node of the coupling set carries a nonzero (C_e is tight at node level)
    e = k ** 3
    assert bool((c.aib.reshape(e, c.n_i, -1, 5).abs().sum((1, 3)) > 0).all())
    assert bool((c.abi.reshape(e, -1, 5, c.n_i).abs().sum((2, 3)) > 0).all())


def test_lower_dimensional_ratios_from_node_counts():
    golden = json.load(open(os.path.join(GOLDEN, "condensed_ratio.json")))
    for n, (num, den) in golden["d1_values"].items():
        n = int(n)
        assert 2 * den == num * (n + 1)                       # 1D: 2 boundary nodes of N+1
    for n, (num, den) in golden["d2_values"].items():
        n = int(n)
        assert ((n + 1) ** 2 - (n - 1) ** 2) * den == num * (n + 1) ** 2
