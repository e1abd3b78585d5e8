"""Parity at the production size the benchmark times: 8^3 elements of order 5
(552 960 DOFs, n_i = 320, n_c = 1200), the same launch configuration.
The oracle checks sampled element outputs one by one, the full-system FP64
residual, and the discrete conservation of the increment."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, fold_matrices, make_plan, rel, to_np
from workload.cases import named_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    torch.cuda.init()
    print("\n[tgv_n5_k8 generation on device]", flush=True)
    case = named_case("tgv_n5_k8", device=DEV)
    dev = dict(aii=case.aii, aib=case.aib, abi=case.abi, bb_val=case.bb_val, b=case.rhs)
    yield case, dev


def _sample_elements(case):
    return [0, 137, case.n_elem - 1]


def test_full_size_fp64(big):
    case, dev = big
    plan = make_plan(case, dev)
    inv = plan.export("aii_inv", case.n_elem * case.n_i ** 2).view(case.n_elem, case.n_i, case.n_i)
    s = plan.export("schur", case.n_elem * case.n_c ** 2).view(case.n_elem, case.n_c, case.n_c)
    fold = fold_matrices(case, _sample_elements(case))
    for e in _sample_elements(case):
        aii, aib, abi = to_np(case.aii[e]), to_np(case.aib[e]), to_np(case.abi[e])
        assert rel(to_np(inv[e]), oracle.element_inverse(aii)) <= 1e-11
        ref = oracle.element_schur(aii, aib, abi)
        assert rel(fold[e] - to_np(s[e]), ref) <= 1e-11
    del inv, s
    for precond in (1, 2):
        dq, info = plan.solve(dev["b"], solver="gmres", precond=precond, tol=1e-10, ir_tol=1e-8)
        print(precond, info, flush=True)
        assert info["rel_res_full"] <= 1e-8
    dq_np, b_np = to_np(dq), to_np(dev["b"])
    bnorm = np.linalg.norm(b_np)
    for e in _sample_elements(case):
        r = oracle.element_interior_residual(e, case.order, case.c_ptr, case.c_node, to_np(case.aii[e]),
                                             to_np(case.aib[e]), b_np, dq_np)
        assert np.linalg.norm(r) <= 1e-8 * bnorm
    m = np.repeat(case.mass, 5).reshape(-1, 5) * dq_np.reshape(-1, 5)
    assert np.all(np.abs(m.sum(0)) <= 1e-8 * np.abs(m).sum(0))
    plan.close()


def test_full_size_fp32_refinement(big):
    case, dev = big
    plan = make_plan(case, dev, precision="fp32")
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-6, ir_tol=1e-8)
    print(info, flush=True)
    assert info["rel_res_full"] <= 1e-8
    plan.close()
