"""Full-solve parity at order 7 with physical values: 2^3 Taylor-Green elements of
order N = 7 (20 480 DOFs, n_i = 1080, n_c = 2520: the N = 7 sizes of the condensed-
size table, Section 3.2), Re 1600, dt 5e-3.  The automatic inverse takes the
blocked form here (n_i > 320).

The expected solution is the oracle's uncondensed solve of eq. NewtonLinSys1:
GMRES on the global matrix with element-block Jacobi, converged to 1e-13 (pinned
against SuperLU on smaller meshes).  FP64: relative error <= 1e-10.  FP32 factors
with FP64 refinement: full-system residual <= 1e-8, computed on the host from the
blocks by the oracle, and error <= 1e-5 (kappa(A) times the residual level)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import device_case, make_plan, oracle_arrays, oracle_matrix, rel, to_np
from workload.cases import build_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def n7():
    torch.cuda.init()
    print("\n[2^3 x N=7 generation + oracle GMRES on A]", flush=True)
    case = build_case(2, 7, 1600.0, 5e-3, seed=0)
    d = oracle_arrays(case)
    ref, it, relres = oracle.solve_gmres_element_jacobi(oracle_matrix(d), d["b"], d["order"], tol=1e-13)
    assert relres <= 1e-13
    yield case, d, device_case(case), ref


def _host_residual(d, dq):
    r = oracle.full_residual_blocks(d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"],
                                    d["bb_val"], d["aii"], d["aib"], d["abi"], d["b"], dq)
    return float(np.linalg.norm(r) / np.linalg.norm(d["b"]))


@pytest.mark.parametrize("precond", [1, 2])
def test_order7_fp64_solve(n7, precond):
    case, d, dev, ref = n7
    assert (case.n_i, case.n_c) == (1080, 2520)
    plan = make_plan(case, dev)
    assert plan.inverse_mode_used() == "blocked"
    dq, info = plan.solve(dev["b"], solver="gmres", precond=precond, tol=1e-13, ir_tol=1e-12)
    print(info, flush=True)
    x = to_np(dq)
    assert rel(x, ref) <= 1e-10, info
    assert _host_residual(d, x) <= 1e-12
    m = np.repeat(case.mass, 5).reshape(-1, 5) * x.reshape(-1, 5)
    assert np.all(np.abs(m.sum(0)) <= 1e-11 * np.abs(m).sum(0))
    plan.close()


def test_order7_fp32_refinement(n7):
    case, d, dev, ref = n7
    plan = make_plan(case, dev, precision="fp32")
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-6, ir_tol=1e-8)
    print(info, flush=True)
    x = to_np(dq)
    res = _host_residual(d, x)
    assert info["rel_res_full"] <= 1e-8 and res <= 1e-8
    assert abs(res - info["rel_res_full"]) <= 1e-3 * res + 1e-14
    assert rel(x, ref) <= 1e-5
    plan.close()
