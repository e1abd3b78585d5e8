"""Pins of the oracle functions that the GPU parity tests compare against at
sizes where the global matrix is not formed: the element inverse, the interior
and full residuals taken block by block, and the condensed CPU route (LAPACK LU
of every A_ii, element Schur blocks, point-Jacobi GMRES on S, back-substitution).

Each is pinned against something other than itself: matrix identities
(A A^-1 = I), closed-form inverses, the residual of the assembled global matrix
(a different code path: scatter into CSR, sparse product) and the uncondensed
SuperLU solve of eq. NewtonLinSys1."""
import numpy as np
import pytest

import oracle
from workload.cases import build_case


def _np(c):
    t = lambda x: x.cpu().numpy()
    return dict(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr,
                bb_col=c.bb_col, bb_val=t(c.bb_val), aii=t(c.aii), aib=t(c.aib), abi=t(c.abi),
                b=t(c.rhs))


def _blocks(d):
    return (d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
            d["aii"], d["aib"], d["abi"])


def _assemble(d):
    return oracle.assemble_global(*_blocks(d))


@pytest.fixture(scope="module")
def n4k2():
    return _np(build_case(2, 4, 1600.0, 5e-3, seed=11))


# ---- element inverse -------------------------------------------------------

def test_element_inverse_is_two_sided_inverse(n4k2):
    for e in (0, 5):
        a = n4k2["aii"][e]
        inv = oracle.element_inverse(a)
        eye = np.eye(a.shape[0])
        assert np.abs(a @ inv - eye).max() <= 1e-13
        assert np.abs(inv @ a - eye).max() <= 1e-13


def test_element_inverse_closed_forms():
    rng = np.random.default_rng(3)
    n = 40
    # Householder reflection H = I - 2 u u^T / u^T u is its own inverse
    u = rng.standard_normal(n)
    h = np.eye(n) - 2.0 * np.outer(u, u) / (u @ u)
    assert np.abs(oracle.element_inverse(h) - h).max() <= 1e-14
    # a permutation needs pivoting (zero leading diagonal); its inverse is its transpose
    p = np.eye(n)[rng.permutation(n)]
    p = p[np.r_[1:n, 0]]
    assert p[0, 0] == 0.0
    assert np.array_equal(oracle.element_inverse(p), p.T)
    # Sherman-Morrison: (D + x y^T)^-1 = D^-1 - D^-1 x y^T D^-1 / (1 + y^T D^-1 x)
    d = rng.uniform(1.0, 3.0, n)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    di = 1.0 / d
    ref = np.diag(di) - np.outer(di * x, y * di) / (1.0 + y @ (di * x))
    got = oracle.element_inverse(np.diag(d) + np.outer(x, y))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_element_inverse_planted_transpose_fails(n4k2):
    a = n4k2["aii"][1]
    # the interior blocks are not symmetric: a transposed inverse is not an inverse
    assert np.abs(a @ oracle.element_inverse(a.T) - np.eye(a.shape[0])).max() > 1e-6


# ---- residuals block by block ---------------------------------------------

def test_interior_residual_equals_rows_of_global_residual(n4k2):
    d = n4k2
    a = _assemble(d)
    rng = np.random.default_rng(5)
    dq = rng.standard_normal(d["b"].shape[0])
    r = oracle.full_residual(a, dq, d["b"])
    interior, _ = oracle.dof_maps(d["order"])
    for e in range(len(d["order"])):
        ri = oracle.element_interior_residual(e, d["order"], d["c_ptr"], d["c_node"], d["aii"][e],
                                              d["aib"][e], d["b"], dq)
        assert np.abs(ri - r[interior[e]]).max() <= 1e-13 * np.abs(r).max()


def test_full_residual_blocks_equals_global_residual(n4k2):
    d = n4k2
    a = _assemble(d)
    rng = np.random.default_rng(6)
    dq = rng.standard_normal(d["b"].shape[0])
    r = oracle.full_residual(a, dq, d["b"])
    rb = oracle.full_residual_blocks(*_blocks(d), d["b"], dq)
    assert np.abs(rb - r).max() <= 1e-13 * np.abs(r).max()
    x = oracle.solve_sparse(a, d["b"])
    rx = oracle.full_residual_blocks(*_blocks(d), d["b"], x)
    assert np.linalg.norm(rx) <= 1e-13 * np.linalg.norm(d["b"])
    # planted mistake: A_bi left out of the boundary rows
    bad = oracle.full_residual_blocks(*_blocks(dict(d, abi=0 * d["abi"])), d["b"], x)
    assert np.linalg.norm(bad) > 1e-6 * np.linalg.norm(d["b"])


# ---- the condensed CPU route ----------------------------------------------

@pytest.mark.parametrize("k,n,re,dt", [(2, 3, 100.0, 1e-2), (2, 4, 1600.0, 5e-3), (3, 2, 1600.0, 5e-3)])
def test_condensed_cpu_route_equals_uncondensed(k, n, re, dt):
    d = _np(build_case(k, n, re, dt, seed=k + 2 * n))
    a = _assemble(d)
    ref = oracle.solve_sparse(a, d["b"])
    c = oracle.condense_cpu(*_blocks(d))
    s = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                      d["aii"], d["aib"], d["abi"])
    x = np.random.default_rng(1).standard_normal(s.shape[0])
    assert np.abs(oracle.schur_matvec_cpu(c, x) - s @ x).max() <= 1e-12 * np.abs(s @ x).max()
    assert np.array_equal(c.diag, np.diag(s)) or np.abs(c.diag - np.diag(s)).max() <= 1e-13 * np.abs(c.diag).max()
    dq, it, relres = oracle.condensed_gmres_solve(c, d["b"], tol=1e-13)
    assert relres <= 1e-13 and it > 0
    assert np.linalg.norm(dq - ref) <= 1e-10 * np.linalg.norm(ref)


def test_condensed_cpu_route_planted_sign_fails():
    d = _np(build_case(2, 3, 100.0, 1e-2, seed=4))
    ref = oracle.solve_sparse(_assemble(d), d["b"])
    c = oracle.condense_cpu(*_blocks(d))
    c.schur = -c.schur                     # S = A_bb + sum A_bi A_ii^-1 A_ib: wrong sign
    c.diag = c.abb.diagonal() + (c.diag - c.abb.diagonal()) * -1.0
    dq, _, _ = oracle.condensed_gmres_solve(c, d["b"], tol=1e-13, max_iter=400)
    assert np.linalg.norm(dq - ref) > 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("k,n", [(2, 3), (2, 4)])
def test_uncondensed_element_jacobi_gmres_equals_superlu(k, n):
    d = _np(build_case(k, n, 1600.0, 5e-3, seed=9))
    a = _assemble(d)
    ref = oracle.solve_sparse(a, d["b"])
    x, it, relres = oracle.solve_gmres_element_jacobi(a, d["b"], d["order"], tol=1e-13)
    assert relres <= 1e-13 and it > 0
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # element-block Jacobi is exact on a block-diagonal matrix: one iteration
    import scipy.sparse as sp
    sizes = 5 * (n + 1) ** 3
    a_bd = sp.block_diag([a[e * sizes:(e + 1) * sizes, e * sizes:(e + 1) * sizes] for e in range(k ** 3)]).tocsr()
    x1, it1, _ = oracle.solve_gmres_element_jacobi(a_bd, d["b"], d["order"], tol=1e-12)
    assert it1 == 1
    assert np.linalg.norm(a_bd @ x1 - d["b"]) <= 1e-12 * np.linalg.norm(d["b"])
