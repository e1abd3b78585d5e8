"""Elements of uneven polynomial order in one plan (orders 2..7 side by side in
every batched launch): interior inverses (both forms), element Schur blocks,
and full solves against the oracle on the mixed-order structure workload
(workload/mixed.py: conforming-style coupling sets across faces of different
order, synthetic diagonally dominant values).  Bars as for the uniform
workloads: 1e-11 per element matrix, 1e-10 on dQ in FP64, 1e-8 full residual
with FP32 factors."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, fold_matrices, rel, to_np
from paper_1911_02366_amd import Plan
from workload.mixed import mixed_order_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mixed():
    torch.cuda.init()
    c = mixed_order_case(2, seed=1)          # orders 5 5 6 7 3 3 7 7
    blocks = c.element_blocks()
    d = dict(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr, bb_col=c.bb_col, **blocks)
    return c, c.to(DEV), d


def _oracle_solve(d, b):
    """Uncondensed oracle solve: GMRES (MGS) on the assembled global matrix to
    1e-14 (the rows are strictly diagonally dominant, so it converges fast)."""
    a = oracle.assemble_global(**d)
    x, _, res = oracle.gmres_mgs(lambda v: a @ v, b, tol=1e-14, restart=50, max_iter=2000)
    assert res <= 1e-14
    return x


def _plan(cd, mode="auto", precision="fp64"):
    plan = Plan.from_structure(cd.structure())
    plan.set_inverse_mode(mode)
    plan.assemble(cd.aii, cd.aib, cd.abi, cd.bb_val)
    plan.factor(precision)
    plan.condense()
    return plan


@pytest.mark.parametrize("mode", ["single", "blocked"])
def test_mixed_inverse_and_schur_blocks(mixed, mode):
    c, cd, d = mixed
    print(f"mixed K=2 orders {c.order.tolist()} inverse {mode}", flush=True)
    plan = _plan(cd, mode)
    assert plan.inverse_mode_used() == mode
    inv = to_np(plan.export("aii_inv", int((c.n_i ** 2).sum())))
    sch = to_np(plan.export("schur", int((c.n_c ** 2).sum())))
    fold = fold_matrices(c)
    oi = np.concatenate([[0], np.cumsum(c.n_i ** 2)])
    oc = np.concatenate([[0], np.cumsum(c.n_c ** 2)])
    for e in range(c.n_elem):
        ni, nc = int(c.n_i[e]), int(c.n_c[e])
        ref = oracle.element_inverse(d["aii"][e])
        assert rel(inv[oi[e]:oi[e + 1]].reshape(ni, ni), ref) <= 1e-11, e
        s_ref = oracle.element_schur(d["aii"][e], d["aib"][e], d["abi"][e])
        assert rel(fold[e] - sch[oc[e]:oc[e + 1]].reshape(nc, nc), s_ref) <= 1e-11, e
    plan.close()


@pytest.mark.parametrize("solver", ["dense", "gmres"])
def test_mixed_full_solve(mixed, solver):
    c, cd, d = mixed
    plan = _plan(cd)
    dq, info = plan.solve(cd.rhs, solver=solver, tol=1e-13)
    ref = _oracle_solve(d, to_np(c.rhs))
    assert rel(to_np(dq), ref) <= 1e-10, info
    plan.close()


def test_mixed_fp32_factors_with_refinement(mixed):
    c, cd, d = mixed
    plan = _plan(cd, precision="fp32")
    dq, info = plan.solve(cd.rhs, solver="gmres", tol=1e-6, ir_tol=1e-8)
    assert info["rel_res_full"] <= 1e-8 and info["ir_sweeps"] >= 2, info
    ref = _oracle_solve(d, to_np(c.rhs))
    assert rel(to_np(dq), ref) <= 1e-7
    plan.close()


def test_mixed_k3_gmres():
    c = mixed_order_case(3, lo=2, hi=5, seed=4)
    print(f"mixed K=3 orders {sorted(set(c.order.tolist()))}", flush=True)
    cd = c.to(DEV)
    plan = _plan(cd)
    dq, info = plan.solve(cd.rhs, solver="gmres", tol=1e-13)
    d = dict(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr, bb_col=c.bb_col,
             **c.element_blocks())
    ref = _oracle_solve(d, to_np(c.rhs))
    assert rel(to_np(dq), ref) <= 1e-10, info
    plan.close()
