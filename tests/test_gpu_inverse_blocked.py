"""The blocked form of the batched Gauss-Jordan inverse (outer panels of 128
columns, the rest of the block updated by a batched matrix-core GEMM) against
the oracle's inverse and against the single-kernel form.

Both forms take the same pivots (same elimination), so they agree to
rounding; against the oracle the FP64 bar is 1e-11 relative per element (the
interior blocks are mass-dominated and well conditioned), FP32 5e-5.
Cases: n_i = 40 (a single outer panel: no GEMM), 135 (128 + a ragged panel of
7), 320 (three outer panels), 1080 (order 7: nine outer panels, inner panels
of 8 columns).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, device_case, oracle_arrays, rel, to_np
from paper_1911_02366_amd import Plan
from workload.cases import build_case

pytestmark = pytest.mark.gpu

CASES = [(2, 3), (2, 4), (2, 5), (2, 7)]


def _plan(case, dev, mode, precision):
    plan = Plan.from_structure(case.structure())
    plan.set_inverse_mode(mode)
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    plan.factor(precision)
    return plan


@pytest.mark.parametrize("k,n", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_blocked_inverse_matches_oracle_and_single_kernel(k, n, precision):
    print(f"blocked inverse K={k} N={n} {precision}", flush=True)
    case = build_case(k, n, 1600.0, 5e-3, seed=3)
    d = oracle_arrays(case)
    dev = device_case(case)
    size = case.n_elem * case.n_i ** 2
    out = {}
    for mode in ("blocked", "single"):
        plan = _plan(case, dev, mode, precision)
        assert plan.inverse_mode_used() == mode
        bad, info = plan.factor_info()
        assert bad == -1, (mode, bad, info)
        dtype = torch.float32 if precision == "fp32" else torch.float64
        out[mode] = to_np(plan.export("aii_inv", size, dtype=dtype)).astype(np.float64).reshape(
            case.n_elem, case.n_i, case.n_i)
        plan.close()
    tol = 1e-11 if precision == "fp64" else 5e-5
    for e in range(case.n_elem):
        ref = oracle.element_inverse(d["aii"][e])
        assert rel(out["blocked"][e], ref) <= tol, (e, rel(out["blocked"][e], ref))
        assert rel(out["blocked"][e], out["single"][e]) <= tol


def test_blocked_inverse_full_solve():
    case = build_case(2, 5, 1600.0, 5e-3, seed=4)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = _plan(case, dev, "blocked", "fp64")
    plan.condense()
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-13)
    a = oracle.assemble_global(d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"],
                               d["bb_val"], d["aii"], d["aib"], d["abi"])
    ref = oracle.solve_sparse(a, d["b"])
    assert rel(to_np(dq), ref) <= 1e-10
    plan.close()


def test_blocked_inverse_reports_singular_block():
    case = build_case(2, 4, 1600.0, 5e-3, seed=5)
    dev = device_case(case)
    aii = dev["aii"].clone().reshape(case.n_elem, case.n_i, case.n_i)
    aii[3, :, 130] = 0.0          # a zero column inside the second (ragged) outer panel
    dev["aii"] = aii.reshape(-1).contiguous()
    plan = _plan(case, dev, "blocked", "fp64")
    bad, info = plan.factor_info()
    assert bad == 3 and info == 131     # LAPACK-style: the 1-based column of the zero pivot
    plan.close()
