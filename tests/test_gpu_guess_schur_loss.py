"""Condensed-residual loss of a predicted increment (scdg_guess_schur_loss)
against the oracle's definition on its dense S: loss to 1e-12 and gradient to
1e-6 (the gradient is returned in FP32) with FP64 Schur blocks, 5e-6 / 1e-5
with FP32 blocks; meshes with two and three elements per direction; the loss
alone (no gradient), a zero output, the scale argument, and refusal in the
matrix-free forms and for bad arguments."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as om
from gpu_common import DEV, device_case, make_plan, oracle_arrays, rel, to_np
from paper_1911_02366_amd import ScdgError
from workload.cases import build_case

pytestmark = pytest.mark.gpu


def _inputs(n_dof, seed):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(n_dof).astype(np.float32)
    t = rng.standard_normal(n_dof).astype(np.float32)
    stats = rng.uniform(-1.0, 1.0, 25)
    stats[15:20] = rng.uniform(0.1, 4.0, 5)
    return y, t, stats


def _dev(*arrs):
    return [torch.tensor(a, device=DEV) for a in arrs]


@pytest.mark.parametrize("k,n", [(2, 3), (3, 3), (2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_loss_and_gradient_match_oracle(k, n, precision):
    case = build_case(k, n, 1600.0, 5e-3, seed=51 + k + n)
    d = oracle_arrays(case)
    plan = make_plan(case, device_case(case), precision=precision)
    s = oracle.condensed_matrix_dense(d["c_ptr"], d["c_node"], d["bb_rowptr"], d["bb_col"], d["bb_val"],
                                      d["aii"], d["aib"], d["abi"])
    _, bnode = oracle.dof_maps(d["order"])
    y, t, stats = _inputs(plan.n_dof, 7 + k)
    want, gwant = om.condensed_loss(s, bnode, y, t, stats[15:20])
    yd, td, sd = _dev(y, t, stats)
    scale = 0.37
    loss, dy = plan.guess_schur_loss(yd, td, sd, scale=scale)
    got = float(loss)
    g = to_np(dy).astype(np.float64)
    tol_l, tol_g = (1e-12, 1e-6) if precision == "fp64" else (5e-6, 1e-5)
    print(f"K={k} N={n} {precision}: loss {abs(got / scale - want) / want:.2e}, "
          f"gradient {rel(g / scale, gwant):.2e}", flush=True)
    assert abs(got - scale * want) <= tol_l * scale * want
    assert rel(g, scale * gwant) <= tol_g
    # the loss alone, and a zero output (y = None): ||S P_b rc t||^2
    loss2, none = plan.guess_schur_loss(yd, td, sd, grad=False)
    assert none is None and abs(float(loss2) - want) <= tol_l * want
    want0, _ = om.condensed_loss(s, bnode, np.zeros_like(y), t, stats[15:20])
    loss0, _ = plan.guess_schur_loss(None, td, sd, grad=False)
    assert abs(float(loss0) - want0) <= tol_l * want0
    plan.close()


def test_gradient_is_zero_on_interior_dofs_and_at_the_target():
    case = build_case(2, 3, 400.0, 1e-2, seed=60)
    plan = make_plan(case, device_case(case))
    d = oracle_arrays(case)
    _, bnode = oracle.dof_maps(d["order"])
    y, t, stats = _inputs(plan.n_dof, 3)
    yd, td, sd = _dev(y, t, stats)
    _, dy = plan.guess_schur_loss(yd, td, sd)
    interior = np.setdiff1d(np.arange(plan.n_dof), bnode.reshape(-1))
    assert interior.size > 0 and not to_np(dy)[interior].any()
    loss, dy = plan.guess_schur_loss(td, td, sd)
    assert float(loss) == 0.0 and not to_np(dy).any()
    plan.close()


def test_refusals():
    case = build_case(2, 3, 100.0, 1e-2, seed=61)
    plan = make_plan(case, device_case(case))
    y, t, stats = _inputs(plan.n_dof, 4)
    yd, td, sd = _dev(y, t, stats)
    with pytest.raises(ScdgError) as err:
        plan.guess_schur_loss(None, None, sd)
    assert err.value.status == -1
    with pytest.raises(ScdgError) as err:
        plan.guess_schur_loss(yd, td, sd, scale=-1.0)
    assert err.value.status == -1
    plan.set_schur_mode("matrix_free")
    plan.condense()
    with pytest.raises(ScdgError) as err:
        plan.guess_schur_loss(yd, td, sd)
    assert err.value.status == -2
    plan.close()


def test_mixed_orders_against_oracle():
    """Elements of orders 2..5 in one plan: the restriction to the boundary
    vector follows each element's own node sets."""
    from paper_1911_02366_amd import Plan
    from workload.mixed import mixed_order_case
    c = mixed_order_case(2, lo=2, hi=5, seed=4)
    blocks = c.element_blocks()
    cd = c.to(DEV)
    plan = Plan.from_structure(cd.structure())
    plan.assemble(cd.aii, cd.aib, cd.abi, cd.bb_val)
    plan.factor("fp64")
    plan.condense()
    s = oracle.condensed_matrix_dense(c.c_ptr, c.c_node, c.bb_rowptr, c.bb_col, blocks["bb_val"],
                                      blocks["aii"], blocks["aib"], blocks["abi"])
    _, bnode = oracle.dof_maps(c.order)
    y, t, stats = _inputs(plan.n_dof, 12)
    want, gwant = om.condensed_loss(s, bnode, y, t, stats[15:20])
    yd, td, sd = _dev(y, t, stats)
    loss, dy = plan.guess_schur_loss(yd, td, sd)
    assert abs(float(loss) - want) <= 1e-12 * want
    assert rel(to_np(dy).astype(np.float64), gwant) <= 1e-6
    plan.close()


def test_follows_a_new_jacobian():
    """After new blocks are assembled and condensed, the loss uses the new S."""
    case = build_case(2, 3, 400.0, 1e-2, seed=62)
    dev = device_case(case)
    plan = make_plan(case, dev)
    y, t, stats = _inputs(plan.n_dof, 5)
    yd, td, sd = _dev(y, t, stats)
    l1 = float(plan.guess_schur_loss(yd, td, sd, grad=False)[0])
    scaled = {k: (v * 2.0).contiguous() for k, v in dev.items() if k != "b"}
    plan.assemble(scaled["aii"], scaled["aib"], scaled["abi"], scaled["bb_val"], copy=True)
    plan.factor("fp64")
    plan.condense()
    l2 = float(plan.guess_schur_loss(yd, td, sd, grad=False)[0])
    # every block doubled: S doubles, the loss grows by exactly 4 (up to rounding)
    assert abs(l2 / l1 - 4.0) <= 1e-12
    plan.close()
