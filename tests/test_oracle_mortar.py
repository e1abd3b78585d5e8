"""Pins of the mixed-order mortar oracle (oracle/mortar.py), against what the
mathematics fixes rather than against itself:

* one order everywhere: the mortar is the identity and the residual equals the
  conforming curved oracle's (eq. DGSEMsystem), an implementation with no
  mortar code;
* free stream: a uniform state is steady (H = 0, lifted gradient 0) on a
  mixed-order mesh of displaced (non-affine) elements with p-nonconforming
  faces, which needs the discrete metric identities and the same normal on both
  sides of every mortar;
* conservation: the residual summed over every node of the periodic mesh
  vanishes for each conserved variable (each face flux enters both sides with
  opposite signs after its projection);
* the BR1 gradient of a state linear in x is exact, across p-nonconforming
  faces, on the element of a 3^3 mesh whose faces do not wrap;
* the complex-step Newton matrix product equals central differences;
* mortar algebra: interpolation is exact for polynomials of the side's degree
  and the mortar integral of such a product is the exact integral;
* planted mistakes in the mortar (no quadrature weights, collocation instead
  of projection) each break one of the pins above.
"""
import math

import numpy as np
import pytest

from oracle import dgsem as od
from oracle import mortar as om

FLOW = od.Flow(0.1, 400.0)


def _state(geo, rng, amp=0.1):
    parts = om.split(np.zeros(geo.mesh.n_dof), geo)
    for p in parts:
        rho = 1.0 + amp * rng.random(p.shape[:-1])
        vel = amp * rng.standard_normal(p.shape[:-1] + (3,))
        pres = 1.0 / (FLOW.gamma * FLOW.mach ** 2) * (1.0 + amp * rng.random(p.shape[:-1]))
        p[..., 0] = rho
        p[..., 1:4] = rho[..., None] * vel
        p[..., 4] = pres / (FLOW.gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return om.join(parts)


def _uniform(geo, rho=1.2, vel=(0.3, -0.2, 0.1), pres=None):
    pres = 1.0 / (FLOW.gamma * FLOW.mach ** 2) if pres is None else pres
    vel = np.array(vel)
    q = np.array([rho, *(rho * vel), pres / (FLOW.gamma - 1.0) + 0.5 * rho * vel @ vel])
    return np.concatenate([np.tile(q, (el.order + 1) ** 3) for el in geo.elems])


MIXED = (5, 5, 6, 7, 3, 3, 7, 7)           # a 2^3 draw from {3..7}: faces 3|5, 3|7, 5|6, 6|7, 7|7, ...


def test_one_order_equals_the_conforming_curved_oracle():
    mesh = om.MortarMesh(2, (3,) * 8, amplitude=0.05)
    geo = om.build_geometry(mesh)
    xyz = np.stack([om.element_nodes(mesh, e) for e in range(8)]).reshape(2, 2, 2, 4, 4, 4, 3)
    grid = od.Grid(2, 3)
    ja, jac = od.metric_terms(xyz, grid)
    q = _state(geo, np.random.default_rng(0))
    ref = od.operator_h_curved(q.reshape(2, 2, 2, 4, 4, 4, 5), grid, FLOW, ja, jac).reshape(-1)
    h = om.residual(q, geo, FLOW)
    assert np.max(np.abs(h - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and the gradient
    g_ref = od.lifted_gradient_curved(q.reshape(2, 2, 2, 4, 4, 4, 5), grid, ja, jac)
    g = om.lifted_gradient(om.split(q, geo), geo)
    g = np.stack(g).reshape(g_ref.shape)
    assert np.max(np.abs(g - g_ref)) <= 1e-12 * np.max(np.abs(g_ref))


def test_geometry_is_non_affine_and_watertight():
    mesh = om.MortarMesh(2, MIXED)
    geo = om.build_geometry(mesh)
    # the Jacobian varies inside an element (not a parallelepiped)
    jac = geo.elems[0].jac
    assert np.ptp(jac) > 1e-3 * np.mean(jac)
    # shared faces: both sides' node positions lie on the same bilinear face
    for f in geo.faces:
        xl = om.element_nodes(mesh, f.left)
        xr = om.element_nodes(mesh, f.right)
        fl = np.take(xl, mesh.orders[f.left], axis=2 - f.d)
        fr = np.take(xr, 0, axis=2 - f.d)
        if (f.left // mesh.k_elem ** f.d) % mesh.k_elem == mesh.k_elem - 1:
            fr = fr.copy()
            fr[..., f.d] += mesh.length            # the periodic wrap
        ml = _face_map_points(fl, f.il)
        mr = _face_map_points(fr, f.ir)
        assert np.max(np.abs(ml - mr)) <= 1e-12


def _face_map_points(pts, im):
    return np.einsum("ma,nb,abc->mnc", im, im, pts)


def test_free_stream_is_steady_on_mixed_orders():
    geo = om.build_geometry(om.MortarMesh(2, MIXED, amplitude=0.05))
    q = _uniform(geo)
    g = om.lifted_gradient(om.split(q, geo), geo)
    # rounding only (the sums are divided by the mass J w_i w_j w_k, down to 2e-4 at N = 7)
    assert max(np.max(np.abs(x)) for x in g) <= 1e-11 * np.max(np.abs(q))
    h = om.residual(q, geo, FLOW)
    scale = np.max(np.abs(q)) * max(np.max(np.abs(el.ja)) for el in geo.elems)
    assert np.max(np.abs(h)) <= 1e-13 * scale


def test_conservation_on_mixed_orders():
    geo = om.build_geometry(om.MortarMesh(2, MIXED))
    q = _state(geo, np.random.default_rng(1))
    h = om.residual(q, geo, FLOW)
    total = sum(x.reshape(-1, 5).sum(axis=0) for x in om.split(h, geo))
    assert np.max(np.abs(total)) <= 1e-12 * np.max(np.abs(h))


def test_lifted_gradient_of_a_linear_state_is_exact_across_mortars():
    orders = tuple(int(n) for n in np.random.default_rng(4).integers(3, 8, 27))
    mesh = om.MortarMesh(3, orders, amplitude=0.05)
    geo = om.build_geometry(mesh)
    centre = 1 + 3 + 9
    nbrs = {orders[mesh.neighbour(centre, d, s)] for d in range(3) for s in (1, -1)}
    assert nbrs - {orders[centre]}, "the centre element needs a p-nonconforming face"
    slope = np.array([[0.3, -0.1, 0.2, 0.05, 0.7],
                      [0.1, 0.4, -0.3, 0.2, -0.5],
                      [-0.2, 0.1, 0.6, -0.4, 0.3]])                 # d q_v / d x_k
    base = np.array([1.0, 0.2, -0.1, 0.3, 50.0])
    parts = [base + om.element_nodes(mesh, e) @ slope for e in range(mesh.n_elem)]
    g = om.lifted_gradient(parts, geo)
    ref = np.broadcast_to(slope, g[centre].shape)
    assert np.max(np.abs(g[centre] - ref)) <= 1e-11 * max(np.max(np.abs(p)) for p in parts)
    # an element with a periodic wrap face sees the jump of the linear state there
    assert np.max(np.abs(g[0] - np.broadcast_to(slope, g[0].shape))) > 1e-3


def test_complex_step_product_equals_central_differences():
    geo = om.build_geometry(om.MortarMesh(2, (3, 4, 3, 5, 4, 3, 3, 4)))
    rng = np.random.default_rng(2)
    q = _state(geo, rng)
    v = rng.standard_normal(q.shape)
    dt = 5e-3
    av = om.jacobian_apply(q, v, geo, FLOW, dt)
    eps = 1e-6
    fd = (om.residual(q + eps * v, geo, FLOW, q, dt) - om.residual(q - eps * v, geo, FLOW, q, dt)) / (2 * eps)
    assert np.linalg.norm(av - fd) <= 1e-7 * np.linalg.norm(av)
    # batched directions give the same products
    vb = np.stack([v, 2.0 * v])
    avb = om.jacobian_apply(q, vb, geo, FLOW, dt)
    assert np.array_equal(avb[0], av)
    assert np.allclose(avb[1], 2.0 * av, rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("n,m", [(3, 3), (3, 5), (4, 7), (2, 6)])
def test_mortar_interpolation_and_integral_are_exact(n, m):
    x_n, w_n = od.gl_rule(n)
    x_m, w_m = od.gl_rule(m)
    im = om.interpolation_matrix(x_n, x_m)
    if n == m:
        assert np.array_equal(im, np.eye(n + 1))
    rng = np.random.default_rng(n * 10 + m)
    c = rng.standard_normal(n + 1)
    poly = lambda x: np.polynomial.polynomial.polyval(x, c)          # degree n
    assert np.allclose(im @ poly(x_n), poly(x_m), rtol=0, atol=1e-13)
    # the mortar integral of a degree-n function against each basis function of the
    # side: exact when the mortar is finer (degree 2n <= 2m - 1), the side's own
    # Gauss-Lobatto sum w_a f_a on a conforming face
    f = np.outer(poly(x_m), poly(x_m))
    s = om._to_side(f[..., None], im, w_m, 1)[..., 0]
    if m > n:
        xg, wg = np.polynomial.legendre.leggauss(n + 2)
        lag = om.interpolation_matrix(x_n, xg)                          # l_a at Gauss points
        ref_1d = (wg * poly(xg)) @ lag
    else:
        ref_1d = w_n * poly(x_n)
    assert np.allclose(s, np.outer(ref_1d, ref_1d), rtol=1e-13, atol=1e-13)
    # and sums to the mortar quadrature of f (what the other side receives)
    assert math.isclose(s.sum(), float(w_m @ f @ w_m), rel_tol=1e-13)


def _planted(monkeypatch, wrong):
    monkeypatch.setattr(om, "_to_side", wrong)


def test_planted_mortar_mistakes_break_a_pin(monkeypatch):
    geo = om.build_geometry(om.MortarMesh(2, MIXED))
    q_free = _uniform(geo)
    q = _state(geo, np.random.default_rng(3))
    right = om._to_side

    def no_weights(fm, im, wm, tail):
        return right(fm, im, np.ones_like(wm), tail)

    def collocation(fm, im, wm, tail):
        # the mortar values taken at the side's nodes (nearest mortar node) with the side's weights
        n = im.shape[1] - 1
        x_n, w_n = od.gl_rule(n)
        x_m, _ = od.gl_rule(len(wm) - 1)
        pick = np.array([int(np.argmin(np.abs(x_m - x))) for x in x_n])
        src = (fm.ndim - 2 - tail, fm.ndim - 1 - tail)
        g = np.moveaxis(fm, src, (-2, -1))[..., pick, :][..., :, pick] * np.outer(w_n, w_n)
        return np.moveaxis(g, (-2, -1), src)

    for wrong in (no_weights, collocation):
        _planted(monkeypatch, wrong)
        h_free = om.residual(q_free, geo, FLOW)
        h = om.residual(q, geo, FLOW)
        total = sum(x.reshape(-1, 5).sum(axis=0) for x in om.split(h, geo))
        free_ok = np.max(np.abs(h_free)) <= 1e-9
        cons_ok = np.max(np.abs(total)) <= 1e-12 * np.max(np.abs(h))
        assert not (free_ok and cons_ok), wrong.__name__
    monkeypatch.setattr(om, "_to_side", right)


def test_mass_integrates_the_volume_of_the_torus():
    """sum_j J_j w_j over every node is the volume L^3: the displacement is periodic,
    so the displaced elements still tile the periodic box, and J (degree <= 2 per
    direction on a trilinear element) is integrated exactly at every order >= 2."""
    mesh = om.MortarMesh(3, tuple(int(n) for n in np.random.default_rng(7).integers(2, 8, 27)))
    geo = om.build_geometry(mesh)
    m = om.mass(geo)
    assert m.shape == (mesh.n_dof,)
    assert math.isclose(m.sum() / 5.0, mesh.length ** 3, rel_tol=1e-13)
    assert max(np.ptp(el.jac) for el in geo.elems) > 1e-2          # not a uniform grid
