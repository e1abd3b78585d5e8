"""Parity at the production size the benchmark times: 8^3 elements of order 5
(552 960 DOFs, n_i = 320, n_c = 1200), the same launch configuration.

Checks, all against the oracle on the host:
  * sampled element outputs one by one (inverse, stored Schur block);
  * the whole increment against the oracle's condensed CPU route (LAPACK LU of
    every A_ii, element Schur blocks, point-Jacobi GMRES on S, back-substitution;
    pinned against SuperLU on small meshes), both sides converged to 1e-13:
    relative error <= 1e-10 over all 552 960 DOFs;
  * the full-system FP64 residual B - A dQ formed element by element from the
    blocks (no global matrix) at the benchmark's tolerance: GMRES stops at
    ||b_S - S x|| <= 1e-10 ||b_S||, and the interior rows vanish after
    back-substitution, so ||B - A dQ|| <= 1e-10 ||b_S|| up to rounding;
  * FP32 factors with FP64 refinement: host residual <= 1e-8 and error <= 1e-5;
  * discrete conservation of the increment."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, fold_matrices, make_plan, rel, to_np
from paper_1911_02366_amd import DgResidual, Plan
from workload.cases import named_case

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def big():
    torch.cuda.init()
    print("\n[tgv_n5_k8 generation on device]", flush=True)
    case = named_case("tgv_n5_k8", device=DEV)
    dev = dict(aii=case.aii, aib=case.aib, abi=case.abi, bb_val=case.bb_val, b=case.rhs)
    host = dict(order=case.order, c_ptr=case.c_ptr, c_node=case.c_node, bb_rowptr=case.bb_rowptr,
                bb_col=case.bb_col, bb_val=to_np(case.bb_val), aii=to_np(case.aii), aib=to_np(case.aib),
                abi=to_np(case.abi), b=to_np(case.rhs))
    yield case, dev, host


@pytest.fixture(scope="module")
def oracle_solution(big):
    case, dev, h = big
    print("\n[oracle condensed CPU route, tgv_n5_k8, to 1e-13]", flush=True)
    c = oracle.condense_cpu(h["order"], h["c_ptr"], h["c_node"], h["bb_rowptr"], h["bb_col"], h["bb_val"],
                            h["aii"], h["aib"], h["abi"])
    dq, it, relres = oracle.condensed_gmres_solve(c, h["b"], tol=1e-13)
    print(f"[oracle: {it} GMRES iterations, rel res on S {relres:.2e}]", flush=True)
    assert relres <= 1e-13
    del c
    return dq


def _host_residual(h, dq):
    r = oracle.full_residual_blocks(h["order"], h["c_ptr"], h["c_node"], h["bb_rowptr"], h["bb_col"],
                                    h["bb_val"], h["aii"], h["aib"], h["abi"], h["b"], dq)
    return float(np.linalg.norm(r))


def _sample_elements(case):
    return [0, 137, case.n_elem - 1]


def test_full_size_fp64_blocks_and_residual(big):
    case, dev, h = big
    plan = make_plan(case, dev)
    inv = plan.export("aii_inv", case.n_elem * case.n_i ** 2).view(case.n_elem, case.n_i, case.n_i)
    s = plan.export("schur", case.n_elem * case.n_c ** 2).view(case.n_elem, case.n_c, case.n_c)
    fold = fold_matrices(case, _sample_elements(case))
    for e in _sample_elements(case):
        assert rel(to_np(inv[e]), oracle.element_inverse(h["aii"][e])) <= 1e-11
        ref = oracle.element_schur(h["aii"][e], h["aib"][e], h["abi"][e])
        assert rel(fold[e] - to_np(s[e]), ref) <= 1e-11
    del inv, s
    bs_norm = float(torch.linalg.norm(plan.condense_rhs(dev["b"])))
    bnorm = float(np.linalg.norm(h["b"]))
    for precond in (1, 2):
        dq, info = plan.solve(dev["b"], solver="gmres", precond=precond, tol=1e-10, ir_tol=1e-8)
        print(precond, info, flush=True)
        x = to_np(dq)
        rn = _host_residual(h, x)
        print(f"host residual {rn / bnorm:.3e} (library {info['rel_res_full']:.3e})", flush=True)
        assert rn <= 1.2e-10 * bs_norm + 1e-13 * bnorm
        assert abs(rn / bnorm - info["rel_res_full"]) <= 1e-3 * rn / bnorm + 1e-15
    m = np.repeat(case.mass, 5).reshape(-1, 5) * x.reshape(-1, 5)
    assert np.all(np.abs(m.sum(0)) <= 1e-8 * np.abs(m).sum(0))
    plan.close()


def test_full_size_fp64_matches_oracle_everywhere(big, oracle_solution):
    case, dev, h = big
    plan = make_plan(case, dev)
    dq, info = plan.solve(dev["b"], solver="gmres", precond=1, tol=1e-13, ir_tol=1e-12, max_iters=3000)
    print(info, flush=True)
    x = to_np(dq)
    err = rel(x, oracle_solution)
    print(f"full-size FP64 error vs oracle {err:.3e}", flush=True)
    assert err <= 1e-10
    # element by element as well: no element's increment is off by more than the bar
    x_e, o_e = x.reshape(case.n_elem, -1), oracle_solution.reshape(case.n_elem, -1)
    worst = np.max(np.linalg.norm(x_e - o_e, axis=1) / np.linalg.norm(o_e, axis=1))
    assert worst <= 1e-9
    plan.close()


def test_full_size_fp32_refinement(big, oracle_solution):
    case, dev, h = big
    plan = make_plan(case, dev, precision="fp32")
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-6, ir_tol=1e-8)
    print(info, flush=True)
    x = to_np(dq)
    res = _host_residual(h, x) / float(np.linalg.norm(h["b"]))
    assert info["rel_res_full"] <= 1e-8 and res <= 1e-8
    err = rel(x, oracle_solution)
    print(f"full-size FP32 + refinement: host residual {res:.3e}, error vs oracle {err:.3e}", flush=True)
    assert err <= 1e-5
    plan.close()


def test_full_size_device_jacobian_blocks(big):
    """The library's own Newton-matrix blocks (scdg_dg_jacobian_blocks) equal the
    generator's over all 512 elements, every entry, 1e-12 of the largest entry."""
    case, dev, h = big
    dg = DgResidual(case.mesh.k_elem, case.mesh.order, mach=case.prm.mach, reynolds=case.prm.reynolds)
    plan = Plan.from_structure(case.structure())
    blk = dg.jacobian_blocks(plan, case.q_state.reshape(-1).contiguous(), 1.0 / case.dt)
    for name in ("aii", "aib", "abi", "bb_val"):
        ref = dev[name] if name in dev else getattr(case, name)
        ref = ref.reshape(-1)
        err = float((blk[name] - ref).abs().max() / ref.abs().max())
        print(f"full-size device blocks {name}: {err:.2e}", flush=True)
        assert err <= 1e-12
    del blk
    plan.close()
    dg.close()
