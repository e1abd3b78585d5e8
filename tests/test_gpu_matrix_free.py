"""Matrix-free Schur products without forming T_e: form 1, S x = A_bb x -
sum_e P_e A_bi(e) (X_e x[C_e]); form 2, the same through the nonzero 5x5
blocks of A_ib and A_bi and A_ii^-1 (the block pattern found from the values).

* One product equals the assembled product to rounding, on random vectors.
* Solves equal the oracle's sparse LU to the FP64 bar, with the same GMRES
  iteration counts as the assembled form under both Jacobi preconditioners
  (the Jacobi blocks are formed from diag(A_bb) and the diagonal blocks of
  A_bi X_e instead of from T_e).
* FP32 factors with FP64 refinement, mixed orders, the captured GMRES cycle,
  and the state rules (re-condense after a change; dense solve and the Schur
  export refused).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, device_case, oracle_arrays, oracle_matrix, rel, to_np
from paper_1911_02366_amd import Plan, ScdgError
from workload.cases import build_case
from workload.mixed import mixed_order_case

pytestmark = pytest.mark.gpu


def _plan(case, dev, mode, precision="fp64", krylov="host"):
    plan = Plan.from_structure(case.structure())
    plan.set_schur_mode(mode)
    plan.set_krylov_mode(krylov)
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    plan.factor(precision)
    plan.condense()
    return plan


MF = ["matrix_free", "matrix_free_sparse"]


@pytest.mark.parametrize("mode", MF)
@pytest.mark.parametrize("k,n", [(2, 3), (2, 5), (3, 4)])
def test_product_equals_assembled(k, n, mode):
    print(f"{mode} product K={k} N={n}", flush=True)
    case = build_case(k, n, 1600.0, 5e-3, seed=4)
    dev = device_case(case)
    asm = _plan(case, dev, "assembled")
    mf = _plan(case, dev, mode)
    assert mf.schur_mode() == mode and asm.schur_mode() == "assembled"
    gen = torch.Generator(device=DEV)
    gen.manual_seed(3)
    for _ in range(3):
        x = torch.randn(case.n1, generator=gen, dtype=torch.float64, device=DEV)
        ya, ym = asm.schur_apply(x), mf.schur_apply(x)
        torch.cuda.synchronize()
        assert rel(to_np(ym), to_np(ya)) <= 1e-12
    asm.close()
    mf.close()


@pytest.mark.parametrize("precond", [1, 2])
@pytest.mark.parametrize("k,n", [(2, 3), (2, 5)])
def test_solve_matches_oracle_and_assembled_iterations(k, n, precond):
    print(f"matrix-free solves K={k} N={n} precond {precond}", flush=True)
    case = build_case(k, n, 1600.0, 5e-3, seed=2)
    d = oracle_arrays(case)
    dev = device_case(case)
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    its = {}
    for mode in ["assembled"] + MF:
        plan = _plan(case, dev, mode)
        dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-12, precond=precond)
        assert rel(to_np(dq), ref) <= 1e-10, (mode, info)
        assert info["rel_res_full"] <= 1e-10
        its[mode] = info["iters"]
        plan.close()
    assert abs(its["matrix_free"] - its["assembled"]) <= 1, its
    assert abs(its["matrix_free_sparse"] - its["assembled"]) <= 1, its


@pytest.mark.parametrize("mode", MF)
def test_fp32_refinement_and_mixed_orders(mode):
    case = build_case(2, 5, 1600.0, 5e-3, seed=7)
    d = oracle_arrays(case)
    dev = device_case(case)
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    plan = _plan(case, dev, mode, precision="fp32")
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-6, ir_tol=1e-10)
    print("fp32 matrix-free", info, flush=True)
    assert info["rel_res_full"] <= 1e-10 and rel(to_np(dq), ref) <= 1e-7
    plan.close()
    # uneven orders (the mixed-order structure workload, orders 5 5 6 7 3 3 7 7)
    c = mixed_order_case(2, seed=1)
    cd = c.to(DEV)
    a = oracle.assemble_global(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr,
                               bb_col=c.bb_col, **c.element_blocks())
    mref = oracle.solve_sparse(a, to_np(c.rhs))
    plan = Plan.from_structure(cd.structure())
    plan.set_schur_mode(mode)
    plan.assemble(cd.aii, cd.aib, cd.abi, cd.bb_val)
    plan.factor("fp64")
    plan.condense()
    dq, info = plan.solve(cd.rhs, solver="gmres", tol=1e-13)
    assert rel(to_np(dq), mref) <= 1e-10, info
    plan.close()


@pytest.mark.parametrize("mode", MF)
def test_captured_cycle_and_state_rules(mode):
    case = build_case(2, 4, 1600.0, 5e-3, seed=6)
    d = oracle_arrays(case)
    dev = device_case(case)
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    plan = _plan(case, dev, mode, krylov="graph")
    for _ in range(2):
        dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=8)
        assert info["restarts"] >= 2 and rel(to_np(dq), ref) <= 1e-10, info
    # the dense solve and the Schur export need the assembled form
    with pytest.raises(ScdgError) as err:
        plan.solve(dev["b"], solver="dense")
    assert err.value.status == -2
    with pytest.raises(ScdgError) as err:
        plan.export("schur", case.n_elem * case.n_c * case.n_c)
    assert err.value.status == -2
    # a change of form sends the plan back to the factored state
    plan.set_schur_mode("assembled")
    with pytest.raises(ScdgError) as err:
        plan.solve(dev["b"], solver="gmres")
    assert err.value.status == -2
    plan.condense()
    dq, info = plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=8)
    assert rel(to_np(dq), ref) <= 1e-10, info
    plan.set_schur_mode(mode)
    plan.condense()
    dq, info = plan.solve(dev["b"], solver="auto", tol=1e-12)
    assert info["solver_used"] == 2 and rel(to_np(dq), ref) <= 1e-10, info
    with pytest.raises(KeyError):
        plan.set_schur_mode("other")
    plan.close()


@pytest.mark.parametrize("mode", MF)
def test_newton_steps_in_matrix_free_form(mode):
    """Captured Newton iterations (scdg_newton_step) with matrix-free products
    equal the host-driven ones and the assembled form's step."""
    from paper_1911_02366_amd.newton import ImplicitStepper
    from workload.cases import jacobian_blocks
    case = build_case(3, 3, 400.0, 1e-2, seed=2, device=DEV)
    mesh, prm, dt = case.mesh, case.prm, case.dt
    jac = lambda q: jacobian_blocks(q, mesh, prm, dt)
    q = case.q_state.reshape(-1).contiguous()
    ref = ImplicitStepper(case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt, jac,
                          newton_tol=1e-10, lin_tol=1e-12, autotune=False)
    ref.prepare(q)
    q_ref, info_ref = ref.solve_step(q)
    ref.close()
    st = ImplicitStepper(case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt, jac,
                         newton_tol=1e-10, lin_tol=1e-12, autotune=False, graph=True, schur_mode=mode)
    assert st.plan.schur_mode() == mode
    for step in range(2):
        st.prepare(q)
        q_h, info_h = st.solve_step(q, graph=False)
        q_g, info_g = st.solve_step(q, graph=True)
        print(f"step {step}: host {info_h} graph {info_g}", flush=True)
        assert info_h["converged"] and info_g["converged"]
        assert rel(to_np(q_g - q), to_np(q_h - q)) <= 1e-8
        if step == 0:
            assert rel(to_np(q_g - q), to_np(q_ref - q)) <= 1e-8, (info_g, info_ref)
        q = q_g
    st.close()


def test_sparse_form_follows_a_changed_block_pattern():
    """New blocks with a different zero pattern (one nonzero block of every
    element's A_ib and A_bi zeroed) are found at the next condense, the block
    lists are rebuilt and the captured cycle is recaptured."""
    case = build_case(2, 4, 1600.0, 5e-3, seed=9)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = _plan(case, dev, "matrix_free_sparse", krylov="graph")
    dq, _ = plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=8)
    assert rel(to_np(dq), oracle.solve_sparse(oracle_matrix(d), d["b"])) <= 1e-10
    aib, abi = d["aib"].copy(), d["abi"].copy()
    for e in range(aib.shape[0]):
        nz = np.argwhere(np.abs(aib[e].reshape(aib.shape[1] // 5, 5, -1, 5)).max(axis=(1, 3)) > 0)
        rb, cb = nz[len(nz) // 2]
        aib[e, 5 * rb:5 * rb + 5, 5 * cb:5 * cb + 5] = 0.0
        nz = np.argwhere(np.abs(abi[e].reshape(abi.shape[1] // 5, 5, -1, 5)).max(axis=(1, 3)) > 0)
        rb, cb = nz[len(nz) // 3]
        abi[e, 5 * rb:5 * rb + 5, 5 * cb:5 * cb + 5] = 0.0
    d2 = dict(d, aib=aib, abi=abi)
    aib_d = torch.tensor(aib, device=DEV)
    abi_d = torch.tensor(abi, device=DEV)
    plan.assemble(dev["aii"], aib_d, abi_d, dev["bb_val"])
    plan.factor("fp64")
    plan.condense()
    dq2, info = plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=8)
    assert rel(to_np(dq2), oracle.solve_sparse(oracle_matrix(d2), d["b"])) <= 1e-10, info
    plan.close()


def test_captured_cycle_follows_new_caller_blocks():
    """The plain matrix-free form reads the caller's A_bi inside the captured
    GMRES cycle: new blocks in new buffers recapture it (the cycle's key holds
    the caller's block addresses)."""
    case = build_case(2, 4, 1600.0, 5e-3, seed=10)
    dev = device_case(case)
    plan = _plan(case, dev, "matrix_free", krylov="graph")
    plan.solve(dev["b"], solver="gmres", tol=1e-12, restart=8)
    case2 = build_case(2, 4, 1600.0, 5e-3, seed=11)
    d2 = oracle_arrays(case2)
    dev2 = device_case(case2)
    plan.assemble(dev2["aii"], dev2["aib"], dev2["abi"], dev2["bb_val"])
    plan.factor("fp64")
    plan.condense()
    dq, info = plan.solve(dev2["b"], solver="gmres", tol=1e-12, restart=8)
    assert info["restarts"] >= 2
    assert rel(to_np(dq), oracle.solve_sparse(oracle_matrix(d2), d2["b"])) <= 1e-10, info
    plan.close()


@pytest.mark.parametrize("mode", ["assembled"] + MF)
def test_fp32_products_match_fp64_to_single_precision(mode):
    """With FP32 factors every form streams FP32 blocks (T_e and the A_bb
    remainder; X_e, A_bi and A_bb; or the nonzero blocks, A_ii^-1 and A_bb),
    accumulating in FP64: the product agrees with the FP64 assembled one to a
    few FP32 roundings of the blocks."""
    case = build_case(2, 5, 1600.0, 5e-3, seed=12)
    dev = device_case(case)
    ref = _plan(case, dev, "assembled")
    p32 = _plan(case, dev, mode, precision="fp32")
    gen = torch.Generator(device=DEV)
    gen.manual_seed(5)
    x = torch.randn(case.n1, generator=gen, dtype=torch.float64, device=DEV)
    y64, y32 = ref.schur_apply(x), p32.schur_apply(x)
    torch.cuda.synchronize()
    err = rel(to_np(y32), to_np(y64))
    print(f"{mode}: FP32 product rel. error {err:.2e}", flush=True)
    assert 1e-9 < err <= 2e-5
    ref.close()
    p32.close()
