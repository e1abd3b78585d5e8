"""The resident-panel form of the batched Gauss-Jordan inverse (one workgroup
per element holding an outer panel of 48 FP64 / 64 FP32 columns in LDS, 32
FP64 columns when some n_i exceeds 320,
16-column inner panels eliminated in registers, one matrix-core pass over the
rest of the block per outer panel) against the oracle's inverse and against
the single-kernel form.

Bars as for the other forms: 1e-11 relative per element in FP64, 5e-5 in FP32
(the interior blocks are mass-dominated and well conditioned).  Cases:
n_i = 5, 40, 135, 320 (one, one, three and seven FP64 outer panels; ragged last
outer and inner panels at 5, 40 and 135), a mixed-order plan with orders 2..5
in one launch, wall elements with n_i = 400 beside inner ones with 320, blocks whose rows are permuted so that the pivots are off the
diagonal, and singular and NaN blocks, which must be reported through
scdg_factor_info like the other forms do."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, device_case, oracle_arrays, oracle_matrix, rel, to_np
from paper_1911_02366_amd import Plan
from workload.cases import build_case
from workload.mixed import mixed_order_case

pytestmark = pytest.mark.gpu


def _inverse(structure, aii, aib, abi, bb_val, mode, precision, n_elem, n_i):
    plan = Plan.from_structure(structure)
    plan.set_inverse_mode(mode)
    plan.assemble(aii, aib, abi, bb_val)
    plan.factor(precision)
    assert plan.inverse_mode_used() == mode
    bad, info = plan.factor_info()
    dtype = torch.float32 if precision == "fp32" else torch.float64
    out = None
    if bad == -1:
        size = int(np.sum(np.asarray(n_i) ** 2)) if np.ndim(n_i) else n_elem * n_i ** 2
        out = to_np(plan.export("aii_inv", size, dtype=dtype)).astype(np.float64)
    plan.close()
    return out, bad, info


@pytest.mark.parametrize("k,n", [(2, 2), (2, 3), (2, 4), (2, 5)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resident_inverse_matches_oracle_and_single_kernel(k, n, precision):
    print(f"resident inverse K={k} N={n} {precision}", flush=True)
    case = build_case(k, n, 1600.0, 5e-3, seed=5)
    d = oracle_arrays(case)
    dev = device_case(case)
    args = (case.structure(), dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    res, bad, _ = _inverse(*args, "resident", precision, case.n_elem, case.n_i)
    assert bad == -1
    single, bad, _ = _inverse(*args, "single", precision, case.n_elem, case.n_i)
    assert bad == -1
    res = res.reshape(case.n_elem, case.n_i, case.n_i)
    single = single.reshape(case.n_elem, case.n_i, case.n_i)
    tol = 1e-11 if precision == "fp64" else 5e-5
    worst = 0.0
    for e in range(case.n_elem):
        ref = oracle.element_inverse(d["aii"][e])
        worst = max(worst, rel(res[e], ref))
        assert rel(res[e], single[e]) <= tol
    print(f"  worst element error vs oracle {worst:.2e}", flush=True)
    assert worst <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resident_inverse_mixed_orders(precision):
    c = mixed_order_case(2, lo=2, hi=5, seed=3)
    print(f"mixed orders {c.order.tolist()} {precision}", flush=True)
    assert len(set(c.n_i.tolist())) >= 3
    blocks = c.element_blocks()
    cd = c.to(DEV)
    res, bad, _ = _inverse(cd.structure(), cd.aii, cd.aib, cd.abi, cd.bb_val, "resident", precision,
                           c.n_elem, c.n_i)
    assert bad == -1
    tol = 1e-11 if precision == "fp64" else 5e-5
    off = 0
    for e in range(c.n_elem):
        m = int(c.n_i[e])
        got = res[off:off + m * m].reshape(m, m)
        off += m * m
        assert rel(got, oracle.element_inverse(blocks["aii"][e])) <= tol, e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resident_inverse_off_diagonal_pivots(precision):
    """Rows of every block permuted at random: the diagonal no longer holds the
    pivots, so almost every column exchanges rows (implicitly)."""
    case = build_case(2, 5, 1600.0, 5e-3, seed=6)
    rng = np.random.default_rng(11)
    aii = to_np(case.aii).reshape(case.n_elem, case.n_i, case.n_i)
    perm = np.stack([rng.permutation(case.n_i) for _ in range(case.n_elem)])
    aii_p = np.stack([aii[e][perm[e]] for e in range(case.n_elem)])
    dev = device_case(case)
    res, bad, _ = _inverse(case.structure(), torch.from_numpy(aii_p.reshape(-1)).to(DEV), dev["aib"], dev["abi"],
                           dev["bb_val"], "resident", precision, case.n_elem, case.n_i)
    assert bad == -1
    res = res.reshape(case.n_elem, case.n_i, case.n_i)
    tol = 1e-11 if precision == "fp64" else 5e-5
    for e in range(case.n_elem):
        assert rel(res[e], oracle.element_inverse(aii_p[e])) <= tol, e


def test_resident_inverse_reports_singular_and_nan_blocks():
    case = build_case(2, 4, 1600.0, 5e-3, seed=7)
    dev = device_case(case)
    zero = dev["aii"].clone().view(case.n_elem, case.n_i, case.n_i)
    zero[3, 7, :] = 0.0
    _, bad, info = _inverse(case.structure(), zero.reshape(-1), dev["aib"], dev["abi"], dev["bb_val"], "resident",
                            "fp64", case.n_elem, case.n_i)
    assert bad == 3 and info > 0
    nan = dev["aii"].clone().view(case.n_elem, case.n_i, case.n_i)
    nan[5, 2, 3] = float("nan")
    _, bad, info = _inverse(case.structure(), nan.reshape(-1), dev["aib"], dev["abi"], dev["bb_val"], "resident",
                            "fp64", case.n_elem, case.n_i)
    assert bad == 5 and 0 < info <= case.n_i


def test_resident_inverse_full_solve():
    case = build_case(2, 5, 1600.0, 5e-3, seed=8)
    d = oracle_arrays(case)
    dev = device_case(case)
    plan = Plan.from_structure(case.structure())
    plan.set_inverse_mode("resident")
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    plan.factor("fp64")
    plan.condense()
    dq, info = plan.solve(dev["b"], solver="gmres", precond=1, tol=1e-13, ir_tol=1e-12, max_iters=2000)
    assert plan.inverse_mode_used() == "resident"
    ref = oracle.solve_sparse(oracle_matrix(d), d["b"])
    err = rel(to_np(dq), ref)
    print(f"resident-inverse solve vs oracle {err:.2e}", flush=True)
    assert err <= 1e-10
    plan.close()


def test_resident_form_refuses_large_blocks():
    case = build_case(2, 6, 1600.0, 5e-3, seed=9)     # n_i = 625
    dev = device_case(case)
    plan = Plan.from_structure(case.structure())
    plan.set_inverse_mode("resident")
    plan.assemble(dev["aii"], dev["aib"], dev["abi"], dev["bb_val"])
    with pytest.raises(Exception) as err:
        plan.factor("fp64")
    assert getattr(err.value, "status", None) == -8
    plan.close()


def test_resident_inverse_wall_elements():
    """Elements with n_i = 320 and 400 in one launch: 3^3 x N = 5 with
    isothermal walls normal to z, whose wall-face nodes join the interior of
    the two outer element layers (the layout up to n_i = 400: 32-column FP64
    and 64-column FP32 outer panels, 25 column tiles).  Inverse against the
    oracle's per element in both precisions, and a full FP64 solve whose
    residual the oracle forms from the blocks (<= 1e-12 relative)."""
    from workload.walls import build_wall_case
    print("[3^3 x N = 5 wall case: generation on the device]", flush=True)
    case = build_wall_case(k_elem=3, order=5, reynolds=1600.0, dt=5e-3, seed=2, device=DEV)
    assert sorted(set(case.n_i.tolist())) == [320, 400]
    eb = case.element_blocks()
    for precision, tol in (("fp64", 1e-11), ("fp32", 5e-5)):
        res, bad, _ = _inverse(case.structure(), case.aii, case.aib, case.abi, case.bb_val, "resident",
                               precision, case.n_elem, case.n_i)
        assert bad == -1
        off, worst = 0, 0.0
        for e in range(case.n_elem):
            m = int(case.n_i[e])
            worst = max(worst, rel(res[off:off + m * m].reshape(m, m), oracle.element_inverse(eb["aii"][e])))
            off += m * m
        print(f"  {precision}: worst element error vs oracle {worst:.2e}", flush=True)
        assert worst <= tol
    plan = Plan.from_structure(case.structure())
    plan.assemble(case.aii, case.aib, case.abi, case.bb_val)
    plan.factor("fp64")
    assert plan.inverse_mode_used() == "resident"
    plan.condense()
    dq, _ = plan.solve(case.rhs, solver="gmres", precond=1, tol=1e-13, ir_tol=1e-12, max_iters=4000)
    # the full residual formed by the oracle block by block (a sparse LU of
    # this 29k-DOF system takes minutes on the host)
    b = to_np(case.rhs)
    r = oracle.full_residual_blocks(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col,
                                    eb["bb_val"], eb["aii"], eb["aib"], eb["abi"], b, to_np(dq),
                                    phys=case.phys_faces)
    res = float(np.linalg.norm(r) / np.linalg.norm(b))
    print(f"  wall solve with the resident inverse: oracle full residual {res:.2e}", flush=True)
    assert res <= 1e-12
    plan.close()
