"""Pins of the FP64 oracle: brute force, condensed = uncondensed, invariants,
free stream, conservation of the increment, and planted mistakes that must fail."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workload.cases import build_case, global_matrix_from_parts


def _np(c):
    t = lambda x: x.cpu().numpy()
    return dict(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr,
                bb_col=c.bb_col, bb_val=t(c.bb_val), aii=t(c.aii), aib=t(c.aib), abi=t(c.abi),
                b=t(c.rhs))


def _assemble(d):
    return oracle.assemble_global(d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"],
                                  d["bb_val"], d["aii"], d["aib"], d["abi"])


def _condensed(d, **over):
    x = dict(d)
    x.update(over)
    return oracle.condensed_solve_dense(x["order"], x["c_ptr"], x["c_node"], x["bb_rowptr"], x["bb_col"],
                                        x["bb_val"], x["aii"], x["aib"], x["abi"], x["b"])


def test_blocks_reassemble_to_generator_matrix(case_n3k2):
    d = _np(case_n3k2)
    a = _assemble(d)
    a0 = global_matrix_from_parts(case_n3k2.parts)
    assert abs(a - a0).max() == 0.0 and a.nnz == a0.nnz


def test_brute_force_dense_equals_sparse(case_n3k2):
    d = _np(case_n3k2)
    a = _assemble(d)
    x1 = oracle.solve_dense(a, d["b"])
    x2 = oracle.solve_sparse(a, d["b"])
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)
    assert np.linalg.norm(oracle.full_residual(a, x1, d["b"])) <= 1e-13 * np.linalg.norm(d["b"])


@pytest.mark.parametrize("k,n,re", [(2, 3, 100.0), (3, 2, 1600.0), (2, 4, 1600.0)])
def test_condensed_equals_uncondensed(k, n, re):
    c = build_case(k, n, re, 5e-3, seed=k + n)
    d = _np(c)
    a = _assemble(d)
    x = oracle.solve_dense(a, d["b"])
    xs = _condensed(d)
    assert np.linalg.norm(xs - x) <= 1e-12 * np.linalg.norm(x)


def test_planted_mistakes_fail_brute_force(case_n3k2):
    d = _np(case_n3k2)
    x = oracle.solve_dense(_assemble(d), d["b"])
    err = lambda y: np.linalg.norm(y - x) / np.linalg.norm(x)
    # A_bi and A_ib swapped (the paper's subscript convention misread)
    passes = lambda y: bool(err(y) <= 1e-10)   # the bar a correct solve meets
    assert not passes(_condensed(d, aib=d["abi"].transpose(0, 2, 1).copy(),
                                 abi=d["aib"].transpose(0, 2, 1).copy()))
    # A_bb dropped from S
    assert not passes(_condensed(d, bb_val=0 * d["bb_val"]))
    # transposed interior blocks
    assert not passes(_condensed(d, aii=d["aii"].transpose(0, 2, 1).copy()))
    # sign of the Schur term flipped
    s = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                      d["aii"], d["aib"], d["abi"])
    s_bad = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                          d["aii"], -d["aib"], d["abi"])
    bs = oracle.condensed_rhs(d["order"], d["c_ptr"], d["c_node"], d["aii"], d["abi"], d["b"])
    _, bnode = oracle.dof_maps(d["order"])
    qb_good = np.linalg.solve(s, bs)
    assert np.linalg.norm(qb_good - x[bnode.reshape(-1)]) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(np.linalg.solve(s_bad, bs) - x[bnode.reshape(-1)]) > 1e-6 * np.linalg.norm(x)


def test_schur_invariants(case_n3k2):
    d = _np(case_n3k2)
    args = (d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"])
    s_zero = oracle.condensed_matrix_dense(*args, d["aii"], 0 * d["aib"], d["abi"])
    s_bb = oracle.condensed_matrix_dense(*args, d["aii"], d["aib"], 0 * d["abi"])
    np.testing.assert_array_equal(s_zero, s_bb)            # S = A_bb when the coupling vanishes
    e = 3
    s1 = oracle.element_schur(d["aii"][e], d["aib"][e], d["abi"][e])
    s2 = oracle.element_schur(2.5 * d["aii"][e], d["aib"][e], d["abi"][e])
    np.testing.assert_allclose(s2, s1 / 2.5, rtol=1e-13, atol=1e-13 * np.abs(s1).max())


def test_increment_conserves_mass_momentum_energy(case_n3k2):
    # 1_v^T dH/dQ = 0 and 1_v^T H = 0 imply sum_j J_j w_j dQ_{j,v} = 0
    c = case_n3k2
    d = _np(c)
    x = oracle.solve_dense(_assemble(d), d["b"])
    m = np.repeat(c.mass, 5).reshape(-1, 5)
    mx = m * x.reshape(-1, 5)
    assert np.all(np.abs(mx.sum(0)) <= 1e-13 * np.abs(mx).sum(0))


def test_free_stream_gives_zero_increment():
    c = build_case(2, 3, 100.0, 1e-2, state="uniform")
    d = _np(c)
    x = _condensed(d)
    assert np.abs(d["b"]).max() < 1e-10
    assert np.abs(x).max() < 1e-12


def test_gmres_oracle_matches_direct(case_n3k2):
    d = _np(case_n3k2)
    a = _assemble(d)
    x = oracle.solve_dense(a, d["b"])
    diag = a.diagonal()
    y, it, rel = oracle.gmres_mgs(lambda v: a @ v, d["b"], tol=1e-13, restart=30, precond_diag=diag)
    assert rel <= 1e-13 and it > 0
    assert np.linalg.norm(y - x) <= 1e-10 * np.linalg.norm(x)


def test_condensed_system_better_conditioned(case_n3k2):
    # the paper observes kappa(S) < kappa(A) for its example (Section 4); here it is reported and checked
    d = _np(case_n3k2)
    a = _assemble(d).toarray()
    s = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                      d["aii"], d["aib"], d["abi"])
    assert np.linalg.cond(s) < np.linalg.cond(a)
