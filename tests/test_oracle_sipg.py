"""Pins of the symmetric interior penalty (SIPG) viscous flux, the paper's
choice for its example (Section 4; the compact-flux class of the sparsity
analysis, Section 3.1), in the oracle and the generator.

  * free stream steady, discrete conservation on a discontinuous state;
  * on states continuous across faces (the nodal interpolant of a smooth
    periodic field) jumps vanish and the broken gradient equals the lifted
    one, so SIPG and BR1 give the same H to rounding;
  * the broken gradient is the exact derivative of each element's own
    polynomial, also for a state that jumps between elements;
  * spectral convergence to the closed-form shear and heat-conduction
    divergences;
  * the penalty damps a momentum jump (a planted sign error grows it);
  * complex-step Jacobian = central differences; the generator's residual
    and Jacobian blocks equal the oracle's;
  * compactness: the A_bb pattern of SIPG is a strict subset of BR1's.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import dgsem as od
from workload import dgsem as wd
from workload.curved import CurvedGeometry, CurvedJacobianParts, operator_h as gen_h
from workload.physics import FlowParams
from workload.walls import partition_general

from test_oracle_dgsem import _coords, _rel_err, _state

FLOW = od.Flow(0.1, 100.0)


def _tgv(k, n, seed=1, amplitude=1e-3):
    return wd.taylor_green_state(wd.Mesh(k, n), FlowParams(0.1, 100.0), seed, amplitude=amplitude)


def test_sipg_free_stream_and_conservation():
    g = od.Grid(3, 3)
    q = _state(1.1, 0.3, -0.2, 0.1, 1.0 / (1.4 * 0.01))
    q = np.broadcast_to(q, (3, 3, 3, 4, 4, 4, 5)).copy()
    assert np.abs(od.operator_h(q, g, FLOW, viscous="sipg")).max() <= 1e-11
    h = od.operator_h(_tgv(3, 3), g, FLOW, viscous="sipg")
    tot, scale = h.reshape(-1, 5).sum(0), np.abs(h).reshape(-1, 5).sum(0)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


@pytest.mark.parametrize("k,n", [(2, 3), (3, 4)])
def test_sipg_equals_br1_on_continuous_states(k, n):
    q = _tgv(k, n, amplitude=0.0)          # interpolant of a smooth periodic field: no jumps
    g = od.Grid(k, n)
    h_s = od.operator_h(q, g, FLOW, viscous="sipg")
    h_b = od.operator_h(q, g, FLOW)
    assert np.abs(h_s - h_b).max() <= 1e-11 * np.abs(h_b).max()
    assert np.abs(od.broken_gradient(q, g) - od.lifted_gradient(q, g)).max() <= 1e-10
    # with the seeded jumps the two fluxes differ
    qp = _tgv(k, n)
    assert np.abs(od.operator_h(qp, g, FLOW, viscous="sipg") - od.operator_h(qp, g, FLOW)).max() \
        > 1e-4 * np.abs(h_b).max()


def test_broken_gradient_is_elementwise_derivative():
    k, n = 2, 4
    g = od.Grid(k, n)
    x, y, z = _coords(g)
    ex = np.arange(k)[None, None, :, None, None, None] + 0 * x          # element index along x
    q = np.stack([1 + 0.1 * x ** 2 * (1 + ex), 0.2 * y * z, x * y * z, 0.5 + ex * z ** 3, 2.0 + 0 * x], -1)
    gb = od.broken_gradient(q, g)
    want = np.zeros(gb.shape)
    want[..., 0, 0] = 0.2 * x * (1 + ex)
    want[..., 1, 1], want[..., 2, 1] = 0.2 * z, 0.2 * y
    want[..., 0, 2], want[..., 1, 2], want[..., 2, 2] = y * z, x * z, x * y
    want[..., 2, 3] = 3 * ex * z ** 2
    assert np.abs(gb - want).max() <= 1e-10 * np.abs(want).max()
    # the lifted gradient sees the jumps between elements
    assert np.abs(od.lifted_gradient(q, g) - want).max() > 1e-3


def test_sipg_closed_form_shear_and_heat_conduction():
    flow = od.Flow(mach=0.3, reynolds=1.0)
    u0, p0 = 0.4, 1.0 / (1.4 * 0.09)
    errs = []
    for n in (3, 5, 7):
        g = od.Grid(4, n)
        _, y, _ = _coords(g)
        q = _state(1.0, u0 * np.sin(y), 0.0, 0.0, p0)
        want = np.stack([0 * y, u0 * np.sin(y), 0 * y, 0 * y, -u0 ** 2 * np.cos(2 * y)], axis=-1)
        errs.append(_rel_err(od.operator_h(q, g, flow, viscous="sipg"), g, want))
    assert errs[0] < 0.25 and errs[1] < 8e-3 and errs[2] < 1e-4, errs


def test_penalty_damps_a_momentum_jump(monkeypatch):
    # rest state with x-momentum only in element (0, 0, 0): the penalty's share of H at
    # that element's face nodes has the sign of the bump (it pulls the bump down)
    g = od.Grid(2, 3)
    p0 = 1.0 / (1.4 * 0.01)
    q = np.broadcast_to(_state(1.0, 0.0, 0.0, 0.0, p0), (2, 2, 2, 4, 4, 4, 5)).copy()
    q[0, 0, 0, ..., 1] += 0.05

    def penalty_part():
        h1 = od.operator_h(q, g, FLOW, viscous="sipg")
        monkeypatch.setattr(od, "SIPG_ETA", 0.0)
        h0 = od.operator_h(q, g, FLOW, viscous="sipg")
        monkeypatch.undo()
        return (h1 - h0)[0, 0, 0, ..., 1]

    dp = penalty_part()
    face = dp[:, :, 3]                  # +x face nodes of the bumped element (i = N)
    assert face.min() > 0
    # planted mistake: the penalty with the wrong sign
    good = od.sipg_viscous_flux
    monkeypatch.setattr(od, "sipg_viscous_flux",
                        lambda qi, gi, qo, go, d, fl, s: 2 * (0.5 * (od.viscous_flux(qi, gi, d, fl) +
                                                                     od.viscous_flux(qo, go, d, fl)))
                        - good(qi, gi, qo, go, d, fl, s))
    h_bad = od.operator_h(q, g, FLOW, viscous="sipg")
    monkeypatch.undo()
    monkeypatch.setattr(od, "SIPG_ETA", 0.0)
    h_zero = od.operator_h(q, g, FLOW, viscous="sipg")
    monkeypatch.undo()
    assert (h_bad - h_zero)[0, 0, 0, :, :, 3, 1].max() < 0


def test_sipg_jacobian_complex_step_matches_central_differences():
    g = od.Grid(2, 2)
    q = _tgv(2, 2)
    v = np.random.default_rng(3).standard_normal(q.shape)
    av = od.jacobian_apply(q, v, g, FLOW, 1e-2, viscous="sipg")
    eps = 1e-9 * np.abs(q).max() / np.abs(v).max()
    fd = (od.residual(q + eps * v, g, FLOW, q, 1e-2, viscous="sipg") -
          od.residual(q - eps * v, g, FLOW, q, 1e-2, viscous="sipg")) / (2 * eps)
    assert np.abs(av - fd).max() <= 1e-6 * np.abs(av).max()


@pytest.fixture(scope="module")
def sipg_and_br1_blocks():
    k, n = 3, 2
    mesh = wd.Mesh(k, n)
    prm = FlowParams(0.1, 100.0)
    q = torch.tensor(_tgv(k, n))
    geo = CurvedGeometry(mesh, wd.curved_node_coordinates(mesh, 0.0))
    out = {}
    for visc in ("sipg", "br1"):
        parts = CurvedJacobianParts(q, geo, prm, 1e-2, viscous=visc)
        out[visc] = partition_general(parts.own, parts.couplings(), n, np.zeros(k ** 3, dtype=np.uint8))
    return mesh, q, out


def test_generator_sipg_residual_equals_oracle():
    k, n = 3, 2
    mesh = wd.Mesh(k, n)
    q = _tgv(k, n)
    geo = CurvedGeometry(mesh, wd.curved_node_coordinates(mesh, 0.0))
    h = gen_h(torch.tensor(q), geo, FlowParams(0.1, 100.0), viscous="sipg").numpy()
    ho = od.operator_h(q, od.Grid(k, n), FLOW, viscous="sipg")
    assert np.abs(h - ho).max() <= 1e-12 * np.abs(ho).max()


def test_sipg_blocks_linearize_the_oracle_residual_and_are_compact(sipg_and_br1_blocks):
    mesh, q, out = sipg_and_br1_blocks
    blk = out["sipg"]
    order = np.full(mesh.n_elem, mesh.order, dtype=np.int32)
    ni, nc = blk["n_i"], blk["n_c"]
    oi, oc = np.concatenate([[0], np.cumsum(ni * ni)]), np.concatenate([[0], np.cumsum(ni * nc)])
    t = lambda x: x.numpy()
    aii = [t(blk["aii"])[oi[e]:oi[e + 1]].reshape(ni[e], ni[e]) for e in range(mesh.n_elem)]
    aib = [t(blk["aib"])[oc[e]:oc[e + 1]].reshape(ni[e], nc[e]) for e in range(mesh.n_elem)]
    abi = [t(blk["abi"])[oc[e]:oc[e + 1]].reshape(nc[e], ni[e]) for e in range(mesh.n_elem)]
    a = oracle.assemble_global(order, blk["c_ptr"], blk["c_node"], blk["bb_rowptr"], blk["bb_col"],
                               t(blk["bb_val"]), aii, aib, abi)
    v = np.random.default_rng(2).standard_normal(q.shape)
    av = od.jacobian_apply(q.numpy(), v, od.Grid(mesh.k_elem, mesh.order), FLOW, 1e-2, viscous="sipg")
    assert np.abs(a @ v.reshape(-1) - av.reshape(-1)).max() <= 1e-12 * np.abs(av).max()
    # compact flux: same coupling sets, and the A_bb pattern a strict subset of BR1's
    br1 = out["br1"]
    assert np.array_equal(blk["c_node"], br1["c_node"])
    nb = blk["bb_rowptr"].shape[0] - 1
    key = lambda b: set((np.repeat(np.arange(nb), np.diff(b["bb_rowptr"])) * nb + b["bb_col"]).tolist())
    ks, kb = key(blk), key(br1)
    assert ks < kb
    print(f"A_bb node blocks: SIPG {len(ks)}, BR1 {len(kb)}")
