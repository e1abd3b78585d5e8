"""The three ways of running the GMRES cycle (host Givens; device-resident;
device-resident replayed from a HIP graph) give the same solutions and the
same iteration counts, against the oracle.

Graph replays are checked the way captured work has to be: several solves in
a row on one plan (each replays the graph once per restart cycle), with eager
library work between them, every result compared with the host-driven solve
of the same right-hand side; after a re-assembly with new blocks the graph is
recaptured."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, device_case, oracle_arrays, oracle_matrix, rel, to_np
from paper_1911_02366_amd import Plan, ScdgError
from workload.cases import build_case

pytestmark = pytest.mark.gpu

MODES = ["host", "device", "graph"]


def _plan(case, dev, mode, precision="fp64"):
    plan = Plan.from_structure(case.structure())
    plan.set_krylov_mode(mode)
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    plan.factor(precision)
    plan.condense()
    return plan


@pytest.mark.parametrize("k,n,restart", [(2, 3, 30), (2, 5, 30), (2, 4, 5)])
def test_modes_agree_with_oracle(k, n, restart):
    print(f"krylov modes K={k} N={n} restart {restart}", flush=True)
    case = build_case(k, n, 1600.0, 5e-3, seed=2)
    d = oracle_arrays(case)
    dev = device_case(case)
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    iters = {}
    for mode in MODES:
        plan = _plan(case, dev, mode)
        dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=restart)
        assert rel(to_np(dq), ref) <= 1e-10, (mode, info)
        iters[mode] = info["iters"]
        plan.close()
    assert abs(iters["device"] - iters["host"]) <= 1 and iters["graph"] == iters["device"], iters


def test_graph_replays_between_eager_work():
    case = build_case(2, 4, 1600.0, 5e-3, seed=6)
    dev = device_case(case)
    host = _plan(case, dev, "host")
    graph = _plan(case, dev, "graph")
    gen = torch.Generator(device=DEV)
    gen.manual_seed(1)
    for rep in range(4):
        b = torch.randn(case.n_dof, generator=gen, dtype=torch.float64, device=DEV)
        dq_h, info_h = host.solve(b, solver="gmres", tol=1e-11, restart=8)
        dq_g, info_g = graph.solve(b, solver="gmres", tol=1e-11, restart=8)
        assert info_g["restarts"] >= 2          # several graph launches per solve
        assert rel(to_np(dq_g), to_np(dq_h)) <= 1e-10, (rep, info_h, info_g)
        # eager library work on the same plan between replays
        bs = graph.condense_rhs(b)
        y = graph.schur_apply(bs)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    host.close()
    graph.close()


def test_graph_recaptured_after_new_blocks_and_precision():
    case = build_case(2, 3, 100.0, 1e-2, seed=8)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = _plan(case, dev, "graph")
    dq, _ = plan.solve(dev["b"], solver="gmres", tol=1e-12)
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    assert rel(to_np(dq), ref) <= 1e-10
    # new blocks (a second case with the same structure) in new buffers
    case2 = build_case(2, 3, 100.0, 1e-2, seed=9)
    d2 = oracle_arrays(case2)
    dev2 = device_case(case2)
    plan.assemble(dev2["aii"], dev2["aib"], dev2["abi"], dev2["bb_val"])
    plan.factor("fp64")
    plan.condense()
    dq2, _ = plan.solve(dev2["b"], solver="gmres", tol=1e-12)
    assert rel(to_np(dq2), oracle.solve_sparse(oracle_matrix(d2), d2["b"])) <= 1e-10
    # FP32 factors with FP64 refinement through the graph
    plan.factor("fp32")
    plan.condense()
    dq3, info3 = plan.solve(dev2["b"], solver="gmres", tol=1e-6, ir_tol=1e-10)
    assert info3["rel_res_full"] <= 1e-10
    plan.close()


def test_device_mode_budget_and_zero_rhs():
    case = build_case(2, 4, 1600.0, 5e-3, seed=3)
    dev = device_case(case)
    for mode in ("device", "graph"):
        plan = _plan(case, dev, mode)
        bs = plan.condense_rhs(dev["b"])
        qb, info = plan.solve_condensed(bs, solver="gmres", tol=1e-14, max_iters=3, restart=30, check=False)
        assert info["status"] == -6 and info["iters"] == 3, (mode, info)
        z = torch.zeros_like(dev["b"])
        dq, info = plan.solve(z, solver="gmres")
        assert float(dq.abs().max()) == 0.0
        plan.close()
