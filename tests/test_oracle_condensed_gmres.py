"""The paper's Krylov observation (Section 4): GMRES with a point-Jacobi
preconditioner converges far better on the condensed system S than on the
global system A, whose iteration count grows much faster with the time step.
The cylinder case is not available; the analogue here is the Taylor-Green
system at growing time steps, both solves by the oracle's GMRES(30) with
point Jacobi to 1e-10, and the condensed solution back-substituted equals the
global one."""
import numpy as np
import pytest

import oracle
from oracle import linalg as ol
from workload.cases import build_case


def _solves(k, n, dt):
    case = build_case(k, n, 1600.0, dt, seed=0)
    aii, aib, abi, bbv = (x.numpy() for x in (case.aii, case.aib, case.abi, case.bb_val))
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib, abi)
    b = case.rhs.numpy()
    s = ol.condensed_matrix_dense(case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib, abi)
    bs = ol.condensed_rhs(case.order, case.c_ptr, case.c_node, aii, abi, b)
    xa, it_a, ra = ol.gmres_mgs(lambda v: a @ v, b, 1e-10, restart=30, max_iter=3000, precond_diag=a.diagonal())
    qb, it_s, rs = ol.gmres_mgs(lambda v: s @ v, bs, 1e-10, restart=30, max_iter=3000,
                                precond_diag=np.diag(s).copy())
    xs = ol.back_substitute(case.order, case.c_ptr, case.c_node, aii, aib, b, qb)
    return it_a, ra, it_s, rs, xa, xs


@pytest.mark.parametrize("dt,factor", [(5e-3, 1.0), (0.2, 3.0)])
def test_condensed_gmres_needs_fewer_iterations(dt, factor):
    it_a, ra, it_s, rs, xa, xs = _solves(2, 4, dt)
    print(f"dt {dt}: global {it_a} iterations, condensed {it_s}", flush=True)
    assert ra <= 1e-10 and rs <= 1e-10
    assert it_s * factor <= it_a
    assert np.linalg.norm(xs - xa) <= 1e-7 * np.linalg.norm(xa)


@pytest.mark.parametrize("dt", [0.2, 2.0])
def test_condensed_system_is_better_conditioned(dt):
    """The paper compares condition numbers of the global and condensed
    systems (Section 4); on a 2^3 x N = 3 mesh kappa_2(S) < kappa_2(A), and
    after the point-Jacobi scaling that GMRES uses the gap widens with dt."""
    case = build_case(2, 3, 1600.0, dt, seed=0)
    aii, aib, abi, bbv = (x.numpy() for x in (case.aii, case.aib, case.abi, case.bb_val))
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib,
                               abi).toarray()
    s = ol.condensed_matrix_dense(case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib, abi)
    ka, ks = np.linalg.cond(a), np.linalg.cond(s)
    ja, js = np.linalg.cond(a / np.diag(a)[:, None]), np.linalg.cond(s / np.diag(s)[:, None])
    print(f"dt {dt}: kappa A {ka:.3e} S {ks:.3e}; Jacobi-scaled A {ja:.3e} S {js:.3e}", flush=True)
    assert ks < ka and 2.0 * js < ja
