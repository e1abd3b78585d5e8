"""Element blocks of the backward-Euler Newton matrix formed on the device
(scdg_dg_jacobian_blocks: pointwise flux Jacobians on dual numbers, summed by a
term template of mesh coefficients) against the generator and the oracle.

  * Against the generator (workload/jacobian.py: the same chain rule with
    complex-step pointwise Jacobians in PyTorch, partitioned by
    workload/partition.py): every entry of A_ii, A_ib, A_bi and A_bb, bar 1e-12
    of the largest entry of each array (both sides exact to rounding).
  * Against the oracle: A v with A assembled on the host from the device
    blocks (oracle.assemble_global) equals the oracle's complex-step
    Newton-matrix product (oracle.dgsem.jacobian_apply) plus M v / dt, 1e-12 of
    max |A v|.  The generator is not involved in this check.
  * A Newton step whose Jacobian comes from the library alone reaches the same
    state as the step with the generator's Jacobian.
  * Unsupported configurations (curved elements, the interior-penalty flux, a
    plan of another mesh) are refused."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, oracle_arrays, oracle_matrix, to_np
from oracle import dgsem as od
from paper_1911_02366_amd import DgResidual, Plan, ScdgError
from workload.cases import build_case

pytestmark = pytest.mark.gpu

CASES = [(2, 2, 100.0, 1e-2, 1), (2, 3, 100.0, 1e-2, 2), (3, 3, 1600.0, 5e-3, 3), (2, 4, 1600.0, 5e-3, 4),
         (3, 4, 400.0, 2e-2, 5), (2, 5, 1600.0, 5e-3, 6)]


def _rel(got, want):
    return float(np.abs(np.asarray(got) - np.asarray(want)).max() / max(np.abs(np.asarray(want)).max(), 1e-300))


def _device_blocks(case, k, n, re, dt):
    dg = DgResidual(k, n, mach=0.1, reynolds=re)
    plan = Plan.from_structure(case.structure())
    blk = dg.jacobian_blocks(plan, case.q_state.reshape(-1).to(DEV).contiguous(), 1.0 / dt)
    return dg, plan, blk


@pytest.mark.parametrize("k,n,re,dt,seed", CASES)
def test_blocks_match_generator(k, n, re, dt, seed):
    print(f"device Jacobian blocks K={k} N={n} Re={re} dt={dt}", flush=True)
    case = build_case(k, n, re, dt, seed=seed, device=DEV)
    dg, plan, blk = _device_blocks(case, k, n, re, dt)
    for name in ("aii", "aib", "abi", "bb_val"):
        ref = getattr(case, name).reshape(-1)
        got = blk[name].reshape(-1)
        assert got.numel() == ref.numel(), name
        err = _rel(to_np(got), to_np(ref))
        print(f"  {name}: {got.numel()} entries, max error {err:.2e} of the largest entry", flush=True)
        assert err <= 1e-12, name
    plan.close()
    dg.close()


@pytest.mark.parametrize("k,n,re,dt,seed", [(2, 3, 100.0, 1e-2, 7), (2, 4, 1600.0, 5e-3, 8)])
def test_blocks_times_vector_match_oracle(k, n, re, dt, seed):
    case = build_case(k, n, re, dt, seed=seed, device=DEV)
    dg, plan, blk = _device_blocks(case, k, n, re, dt)
    d = oracle_arrays(case)
    for name in ("aii", "aib", "abi", "bb_val"):
        d[name] = to_np(blk[name]).reshape(d[name].shape)
    a = oracle_matrix(d)
    q = to_np(case.q_state).reshape(-1)
    v = np.random.default_rng(seed).standard_normal(q.size)
    # the oracle's product in its natural DOF order; the assembled matrix is in the same order
    want = od.jacobian_apply(q.reshape(k, k, k, n + 1, n + 1, n + 1, 5), v.reshape(k, k, k, n + 1, n + 1, n + 1, 5),
                             od.Grid(k, n), od.Flow(0.1, re), dt).reshape(-1)
    got = a @ v
    err = _rel(got, want)
    print(f"A v from device blocks vs oracle complex step: {err:.2e}", flush=True)
    assert err <= 1e-12
    plan.close()
    dg.close()


def test_newton_step_with_device_jacobian():
    from paper_1911_02366_amd.newton import ImplicitStepper
    k, n, re, dt = 2, 4, 1600.0, 5e-3
    case = build_case(k, n, re, dt, seed=9, device=DEV)
    q_s = case.q_state.reshape(-1).to(DEV).contiguous()
    gen = lambda q: {key: getattr(case, key) for key in ("aii", "aib", "abi", "bb_val")}
    out = {}
    for name, jac in (("generator", gen), ("device", "device")):
        st = ImplicitStepper(case.structure(), k, n, mach=0.1, reynolds=re, dt=dt, jacobian=jac, autotune=False,
                             newton_tol=1e-10, lin_tol=1e-12)
        st.prepare(q_s)
        q, info = st.solve_step(q_s)
        out[name] = to_np(q)
        print(name, info, flush=True)
    err = _rel(out["device"], out["generator"])
    print(f"Newton step, device vs generator Jacobian: {err:.2e}", flush=True)
    assert err <= 1e-12


def test_unsupported_configurations_refused():
    k, n, re, dt = 2, 3, 100.0, 1e-2
    case = build_case(k, n, re, dt, seed=10, device=DEV)
    q = case.q_state.reshape(-1).to(DEV).contiguous()
    plan = Plan.from_structure(case.structure())
    sipg = DgResidual(k, n, mach=0.1, reynolds=re, viscous="sipg")
    with pytest.raises(ScdgError) as err:
        sipg.jacobian_blocks(plan, q, 1.0 / dt)
    assert err.value.status == -8
    other = DgResidual(3, n, mach=0.1, reynolds=re)
    with pytest.raises(ValueError):
        other.jacobian_blocks(plan, q, 1.0 / dt)      # state of the wrong size
    q3 = torch.zeros(other.n_dof, dtype=torch.float64, device=DEV)
    with pytest.raises(ScdgError) as err:
        other.jacobian_blocks(plan, q3, 1.0 / dt)     # plan of a 2^3 mesh, object of a 3^3 mesh
    assert err.value.status == -8
    for o in (plan, sipg, other):
        o.close()


def _pattern_blocks(rowptr, col, val):
    """{(row, col): 5x5 block} of an A_bb pattern."""
    val = to_np(val).reshape(-1, 5, 5)
    out = {}
    for r in range(len(rowptr) - 1):
        for j in range(rowptr[r], rowptr[r + 1]):
            out[(r, int(col[j]))] = val[j]
    return out


def test_plan_pattern_without_room_and_with_extra_blocks():
    """Whether the plan holds a place for every block the Jacobian can fill is
    checked once per plan (the call is asynchronous afterwards when it does;
    otherwise each call checks the values): a plan whose A_bb pattern lacks a
    nonzero block is refused (SCDG_ERR_ARG), one whose pattern has an extra
    block gets zeros there and the same values everywhere else; alternating
    between plans on one DG object gives bitwise the same blocks each time."""
    k, n, re, dt = 3, 3, 400.0, 1e-2
    case = build_case(k, n, re, dt, seed=12, device=DEV)
    q = case.q_state.reshape(-1).to(DEV).contiguous()
    dg = DgResidual(k, n, mach=0.1, reynolds=re)
    st = case.structure()
    plan = Plan.from_structure(st)
    ref = dg.jacobian_blocks(plan, q, 1.0 / dt)
    rowptr, col = np.asarray(st["bb_rowptr"], dtype=np.int64), np.asarray(st["bb_col"], dtype=np.int32)
    blocks = _pattern_blocks(rowptr, col, ref["bb_val"])
    # drop the largest off-diagonal block of row 0
    r0 = 0
    js = [j for j in range(rowptr[r0], rowptr[r0 + 1]) if col[j] != r0]
    jd = max(js, key=lambda j: np.abs(blocks[(r0, int(col[j]))]).max())
    assert np.abs(blocks[(r0, int(col[jd]))]).max() > 0
    col_less = np.delete(col, jd)
    rowptr_less = rowptr.copy()
    rowptr_less[r0 + 1:] -= 1
    less = Plan.from_structure(dict(st, bb_rowptr=rowptr_less, bb_col=col_less))
    with pytest.raises(ScdgError) as err:
        dg.jacobian_blocks(less, q, 1.0 / dt)
    assert err.value.status == -1
    # add a block to row 1 in a column it does not couple to
    r1 = 1
    present = set(int(c) for c in col[rowptr[r1]:rowptr[r1 + 1]])
    extra = next(c for c in range(int(col.max()) + 1) if c not in present)
    row_cols = sorted(present | {extra})
    col_more = np.concatenate([col[:rowptr[r1]], np.array(row_cols, dtype=np.int32), col[rowptr[r1 + 1]:]])
    rowptr_more = rowptr.copy()
    rowptr_more[r1 + 1:] += 1
    more = Plan.from_structure(dict(st, bb_rowptr=rowptr_more, bb_col=col_more))
    got = dg.jacobian_blocks(more, q, 1.0 / dt)
    for name in ("aii", "aib", "abi"):
        assert torch.equal(got[name], ref[name]), name
    gb = _pattern_blocks(rowptr_more, col_more, got["bb_val"])
    assert not gb.pop((r1, extra)).any()
    assert gb.keys() == blocks.keys()
    assert all(np.array_equal(gb[key], blocks[key]) for key in blocks)
    # back to the first plan, then the extended one again: same blocks bitwise
    again = dg.jacobian_blocks(plan, q, 1.0 / dt)
    for name in ("aii", "aib", "abi", "bb_val"):
        assert torch.equal(again[name], ref[name]), name
    got2 = dg.jacobian_blocks(more, q, 1.0 / dt)
    for name in ("aii", "aib", "abi", "bb_val"):
        assert torch.equal(got2[name], got[name]), name
    for o in (plan, less, more, dg):
        o.close()
