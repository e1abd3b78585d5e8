"""Edge cases and failure handling of the HIP path (forced from the host; no
kernel is made to fault): zero and free-stream right-hand sides, a singular
interior block, a NaN right-hand side, an exhausted iteration budget, call
order, an exact initial guess, repeatability, and FP32 factors with FP64
iterative refinement."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, device_case, make_plan, oracle_arrays, oracle_matrix, rel, to_np
from paper_1911_02366_amd import Plan, ScdgError
from workload.cases import build_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    torch.cuda.init()
    case = build_case(2, 3, 100.0, 1e-2, seed=11)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = make_plan(case, dev)
    yield case, d, dev, plan
    plan.close()


def test_zero_rhs_gives_zero_increment(small):
    case, d, dev, plan = small
    for solver in ("dense", "gmres"):
        dq, info = plan.solve(torch.zeros_like(dev["b"]), solver=solver)
        assert float(dq.abs().max()) == 0.0
    x0 = torch.randn(case.n_dof, dtype=torch.float64, device=DEV)
    dq, info = plan.solve(torch.zeros_like(dev["b"]), x0=x0, solver="gmres")
    assert float(dq.abs().max()) == 0.0


def test_free_stream_state():
    case = build_case(2, 3, 100.0, 1e-2, state="uniform")
    dev = device_case(case)
    plan = make_plan(case, dev)
    dq, info = plan.solve(dev["b"], solver="gmres", ir_tol=1e-6)
    assert float(dev["b"].abs().max()) < 1e-10
    assert float(dq.abs().max()) < 1e-12
    plan.close()


def test_singular_interior_block_reported(small):
    case, d, dev, plan = small
    bad = dev["aii"].clone()
    bad[3, 7, :] = 0.0                      # zero row: A_ii(3) singular
    p2 = Plan.from_structure(case.structure())
    p2.assemble(bad, dev["aib"], dev["abi"], dev["bb_val"])
    p2.factor("fp64")
    elem, info = p2.factor_info()
    assert elem == 3 and info > 0
    with pytest.raises(ScdgError) as err:
        p2.condense()
    assert err.value.status == -5
    p2.close()


def test_nan_rhs_reported(small):
    case, d, dev, plan = small
    b = dev["b"].clone()
    b[17] = float("nan")
    with pytest.raises(ScdgError) as err:
        plan.solve(b, solver="gmres")
    assert err.value.status == -7


def test_iteration_budget_exhausted(small):
    case, d, dev, plan = small
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-15, max_iters=1, ir_max=1, check=False)
    assert info["status"] == -6 and info["iters"] == 1
    assert np.isfinite(to_np(dq)).all()


def test_call_order_enforced(small):
    case, d, dev, plan = small
    p2 = Plan.from_structure(case.structure())
    with pytest.raises(ScdgError) as err:
        p2.factor("fp64")
    assert err.value.status == -2
    p2.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    with pytest.raises(ScdgError) as err:
        p2.condense()
    assert err.value.status == -2
    with pytest.raises(ScdgError):
        p2.solve(dev["b"])
    p2.close()


def test_exact_guess_needs_no_iteration(small):
    case, d, dev, plan = small
    ref = oracle.solve_dense(oracle_matrix(d), d["b"])
    dq, info = plan.solve(dev["b"], x0=torch.tensor(ref, device=DEV), solver="gmres", tol=1e-8)
    assert info["iters"] == 0
    assert rel(to_np(dq), ref) <= 1e-12


def test_repeatable_bitwise(small):
    case, d, dev, plan = small
    a, _ = plan.solve(dev["b"], solver="gmres", tol=1e-12)
    b, _ = plan.solve(dev["b"], solver="gmres", tol=1e-12)
    assert torch.equal(a, b)
    p2 = make_plan(case, dev)
    s1 = plan.export("schur", case.n_elem * case.n_c ** 2)
    s2 = p2.export("schur", case.n_elem * case.n_c ** 2)
    assert torch.equal(s1, s2)
    p2.close()


@pytest.mark.parametrize("k,n", [(2, 3), (2, 5)])
def test_fp32_factors_with_fp64_refinement(k, n):
    case = build_case(k, n, 1600.0, 5e-3, seed=5)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = make_plan(case, dev, precision="fp32")
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-6, ir_tol=1e-8)
    assert info["rel_res_full"] <= 1e-8, info
    assert info["ir_sweeps"] >= 2
    # error bounded by kappa(A) times the residual; kappa ~ 1e3-1e4 here
    assert rel(to_np(dq), ref) <= 1e-5
    inv = to_np(plan.export("aii_inv", case.n_elem * case.n_i ** 2, dtype=torch.float32))
    inv = inv.reshape(case.n_elem, case.n_i, case.n_i)
    for e in (0, case.n_elem - 1):
        assert rel(inv[e], oracle.element_inverse(d["aii"][e])) <= 1e-4
    plan.close()
