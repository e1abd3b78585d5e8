"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: FP64 results must match the oracle to 1e-10 relative (the
target for the plain form).  Per-element matrices are compared at 1e-11
relative: the interior blocks are well conditioned (mass-dominated), so the
Gauss-Jordan inverse and the Schur products carry errors of a few n eps kappa.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import (DEV, device_case, fold_matrices, make_plan, oracle_arrays, oracle_matrix,
                        rel, to_np)
from workload.cases import build_case, named_case

pytestmark = pytest.mark.gpu

CASES = {
    "n3k2": dict(k_elem=2, order=3, reynolds=100.0, dt=1e-2),     # the 2x2x2 N=3 workload
    "n2k3": dict(k_elem=3, order=2, reynolds=1600.0, dt=5e-3),
    "n4k2": dict(k_elem=2, order=4, reynolds=1600.0, dt=5e-3),    # n_i = 135: ragged MFMA tiles
    "n5k2": dict(k_elem=2, order=5, reynolds=1600.0, dt=5e-3),    # n_i = 320, n_c = 1200
}


@pytest.fixture(scope="module", params=list(CASES))
def setup(request):
    torch.cuda.init()
    print(f"\n[case {request.param}]", flush=True)
    case = build_case(seed=7, **CASES[request.param])
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = make_plan(case, dev)
    yield request.param, case, d, dev, plan
    plan.close()


def test_inverse_parity(setup):
    name, case, d, dev, plan = setup
    inv = to_np(plan.export("aii_inv", case.n_elem * case.n_i ** 2)).reshape(case.n_elem, case.n_i, case.n_i)
    for e in range(case.n_elem):
        ref = oracle.element_inverse(d["aii"][e])
        assert rel(inv[e], ref) <= 1e-11, (name, e)


def test_schur_block_parity(setup):
    # stored element block T_e = F_e - A_bi(e) A_ii(e)^-1 A_ib(e), F_e the folded A_bb blocks
    name, case, d, dev, plan = setup
    s = to_np(plan.export("schur", case.n_elem * case.n_c ** 2)).reshape(case.n_elem, case.n_c, case.n_c)
    fold = fold_matrices(case)
    for e in range(case.n_elem):
        ref = oracle.element_schur(d["aii"][e], d["aib"][e], d["abi"][e])
        assert rel(fold[e] - s[e], ref) <= 1e-11, (name, e)


def test_condensed_rhs_parity(setup):
    name, case, d, dev, plan = setup
    bs = plan.condense_rhs(dev["b"])
    ref = oracle.condensed_rhs(d["order"], d["c_ptr"], d["c_node"], d["aii"], d["abi"], d["b"])
    assert rel(to_np(bs), ref) <= 1e-12


def test_schur_apply_parity(setup):
    name, case, d, dev, plan = setup
    s = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                      d["aii"], d["aib"], d["abi"])
    x = np.random.default_rng(3).standard_normal(s.shape[0])
    y = plan.schur_apply(torch.tensor(x, device=DEV))
    assert rel(to_np(y), s @ x) <= 1e-12


def test_backsolve_parity(setup):
    name, case, d, dev, plan = setup
    qb = np.random.default_rng(4).standard_normal(case.n1)
    dq = plan.backsolve(dev["b"], torch.tensor(qb, device=DEV))
    ref = oracle.back_substitute(d["order"], d["c_ptr"], d["c_node"], d["aii"], d["aib"], d["b"], qb)
    assert rel(to_np(dq), ref) <= 1e-12


def test_residual_parity(setup):
    name, case, d, dev, plan = setup
    a = oracle_matrix(d)
    x = np.random.default_rng(5).standard_normal(case.n_dof)
    r = torch.empty(case.n_dof, dtype=torch.float64, device=DEV)
    _, relv = plan.residual(dev["b"], torch.tensor(x, device=DEV), r)
    ref = oracle.full_residual(a, x, d["b"])
    assert rel(to_np(r), ref) <= 1e-13
    assert abs(relv - np.linalg.norm(ref) / np.linalg.norm(d["b"])) <= 1e-12 * relv


@pytest.mark.parametrize("solver,precond", [("dense", 1), ("gmres", 1), ("gmres", 2), ("gmres", 0)])
def test_full_solve_parity(setup, solver, precond):
    name, case, d, dev, plan = setup
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    dq, info = plan.solve(dev["b"], solver=solver, precond=precond, tol=1e-13, ir_tol=1e-12)
    assert rel(to_np(dq), ref) <= 1e-10, info
    assert info["rel_res_full"] <= 1e-12
    # discrete conservation of the increment: sum_j J_j w_j dQ_{j,v} = 0
    m = np.repeat(case.mass, 5).reshape(-1, 5) * to_np(dq).reshape(-1, 5)
    assert np.all(np.abs(m.sum(0)) <= 1e-11 * np.abs(m).sum(0))


def test_condensed_pipeline_by_stages(setup):
    name, case, d, dev, plan = setup
    bs = plan.condense_rhs(dev["b"])
    qb, info = plan.solve_condensed(bs, solver="gmres", tol=1e-13)
    dq = plan.backsolve(dev["b"], qb)
    ref = oracle.condensed_solve_dense(d["order"], d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"],
                                       d["bb_val"], d["aii"], d["aib"], d["abi"], d["b"])
    assert rel(to_np(dq), ref) <= 1e-10, info


@pytest.mark.parametrize("cfg", list(range(9)))
def test_every_gemm_tile_config(setup, cfg):
    name, case, d, dev, plan = setup
    plan.set_gemm_config(cfg, cfg)
    plan.condense()
    x = to_np(plan.export("x", case.n_elem * case.n_i * case.n_c)).reshape(case.n_elem, case.n_i, case.n_c)
    s = to_np(plan.export("schur", case.n_elem * case.n_c ** 2)).reshape(case.n_elem, case.n_c, case.n_c)
    fold = fold_matrices(case, [0, case.n_elem - 1])
    for e in (0, case.n_elem - 1):
        assert rel(x[e], np.linalg.solve(d["aii"][e], d["aib"][e])) <= 1e-11, (name, cfg, e)
        ref = oracle.element_schur(d["aii"][e], d["aib"][e], d["abi"][e])
        assert rel(fold[e] - s[e], ref) <= 1e-11, (name, cfg, e)


def test_autotune_keeps_results(setup, tmp_path):
    name, case, d, dev, plan = setup
    cache = str(tmp_path / "autotune.json")
    tuned = plan.autotune(cache=cache)
    assert not tuned["cached"]
    assert tuned["x"] in tuned["ms_x"] and tuned["ms_s"][tuned["s"]] > 0
    # a second plan of the same problems takes the stored choice without timing
    other = make_plan(case, dev)
    other.set_gemm_config(0, 0)
    again = other.autotune(cache=cache)
    assert again["cached"] and (again["x"], again["s"]) == (tuned["x"], tuned["s"])
    assert other.gemm_config() == plan.gemm_config()
    other.close()
    plan.condense()
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-13, ir_tol=1e-12)
    assert rel(to_np(dq), ref) <= 1e-10
