"""Pins of the oracle's GL-DGSEM residual against what the mathematics fixes.

Each check would fail for a plausible mistake in oracle/dgsem.py:
  * quadrature and differentiation exactness of the Gauss-Lobatto rule;
  * hand-evaluated Euler, viscous and Lax-Friedrichs fluxes, and the
    eigenvalues u - c, u, u, u, u + c of the Euler flux Jacobian;
  * free-stream preservation and discrete conservation on a periodic mesh;
  * spectral convergence of H / M to closed-form divergences (advected
    density wave, sinusoidal shear, heat conduction) and of the lifted
    gradient to the exact gradient;
  * piecewise-constant states, where H reduces to face fluxes alone;
  * the Jacobian blocks of the workload agree with central differences of
    the oracle's residual (the linear systems solved are linearizations of
    this residual, eq. NewtonLinSys1);
  * a planted sign error in the oracle fails at least one of these.
"""
import math

import numpy as np
import pytest

from oracle import dgsem as od

FLOW = od.Flow(mach=0.1, reynolds=1600.0)


def _coords(grid: od.Grid):
    x, _ = od.gl_rule(grid.order)
    k, h = grid.k_elem, grid.h
    line = np.arange(k)[:, None] * h + 0.5 * h * (x[None, :] + 1.0)      # [K, P]
    shp = (k, k, k, grid.p, grid.p, grid.p)
    xs = np.broadcast_to(line[None, None, :, None, None, :], shp)
    ys = np.broadcast_to(line[None, :, None, None, :, None], shp)
    zs = np.broadcast_to(line[:, None, None, :, None, None], shp)
    return xs, ys, zs


def _state(rho, u, v, w, p, gamma=1.4):
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack(np.broadcast_arrays(rho, rho * u, rho * v, rho * w, e), axis=-1).astype(float)


# ---------------------------------------------------------------- GL rule

@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_gl_rule_exactness(n):
    x, w = od.gl_rule(n)
    assert x[0] == -1.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    for deg in range(2 * n):          # exact up to degree 2N - 1
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-14
    # degree 2N is not integrated exactly by an (N+1)-point Lobatto rule
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6
    dm = od.lagrange_derivative(x)
    for deg in range(n + 1):
        want = deg * x ** (deg - 1) if deg else np.zeros_like(x)
        assert np.abs(dm @ x ** deg - want).max() < 1e-12


def test_gl_rule_closed_forms():
    x, w = od.gl_rule(2)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], rtol=0, atol=1e-15)
    x, w = od.gl_rule(3)
    np.testing.assert_allclose(x, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = od.gl_rule(4)
    np.testing.assert_allclose(x, [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], atol=1e-15)
    np.testing.assert_allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1], atol=1e-15)


def test_mass_sums_to_volume():
    g = od.Grid(3, 4, length=2.5)
    assert abs(od.mass(g).sum() - 2.5 ** 3) < 1e-12


# ---------------------------------------------------------------- fluxes

def test_euler_flux_hand_values():
    # rho = 1, v = (1, 0, 0), p = 1: rho E = 1 / 0.4 + 0.5 = 3
    q = np.array([1.0, 1.0, 0.0, 0.0, 3.0])
    np.testing.assert_allclose(od.euler_flux(q, 0, FLOW), [1.0, 2.0, 0.0, 0.0, 4.0], atol=1e-15)
    np.testing.assert_allclose(od.euler_flux(q, 1, FLOW), [0.0, 0.0, 1.0, 0.0, 0.0], atol=1e-15)
    # rho = 2, v = (0, 0, -0.5), p = 0.8: rho E = 2 + 0.25 = 2.25
    q = np.array([2.0, 0.0, 0.0, -1.0, 2.25])
    np.testing.assert_allclose(od.euler_flux(q, 2, FLOW), [-1.0, 0.0, 0.0, 0.5 + 0.8, -0.5 * (2.25 + 0.8)],
                               atol=1e-15)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_euler_jacobian_eigenvalues(d):
    rho, vel, p = 1.3, np.array([0.4, -0.7, 0.2]), 2.1
    q = _state(rho, *vel, p)
    jac = np.zeros((5, 5))
    for j in range(5):
        dq = np.zeros(5)
        dq[j] = 1e-6
        jac[:, j] = (od.euler_flux(q + dq, d, FLOW) - od.euler_flux(q - dq, d, FLOW)) / 2e-6
    c = math.sqrt(1.4 * p / rho)
    ev = np.sort(np.linalg.eigvals(jac).real)
    want = np.sort([vel[d] - c, vel[d], vel[d], vel[d], vel[d] + c])
    np.testing.assert_allclose(ev, want, atol=1e-6)


def test_viscous_flux_hand_values():
    flow = od.Flow(mach=0.2, reynolds=50.0)
    # rho = 1, v = (0.5, 0, 0), p with T = gamma Ma^2 p / rho = 1, so mu = 1
    p = 1.0 / (1.4 * 0.04)
    q = _state(1.0, 0.5, 0.0, 0.0, p)
    grad = np.zeros((3, 5))
    grad[1, 1] = 2.0          # d(rho u)/dy = 2 -> du/dy = 2
    grad[1, 4] = 1.0          # d(rho E)/dy = rho u du/dy at constant p, so de/dy = 0
    f_y = od.viscous_flux(q, grad, 1, flow)
    # tau_xy = mu du/dy = 2; energy flux u tau_xy = 1
    np.testing.assert_allclose(f_y, np.array([0.0, 2.0, 0.0, 0.0, 1.0]) / 50.0, atol=1e-15)
    f_x = od.viscous_flux(q, grad, 0, flow)
    np.testing.assert_allclose(f_x, np.array([0.0, 0.0, 2.0, 0.0, 0.0]) / 50.0, atol=1e-15)
    # dilatation: du/dx = 3 -> tau_xx = mu (2 * 3 - 2/3 * 3) = 4, tau_yy = -2
    grad = np.zeros((3, 5))
    grad[0, 1] = 3.0
    grad[0, 4] = 1.5          # rho u du/dx: again de/dx = 0
    np.testing.assert_allclose(od.viscous_flux(q, grad, 0, flow),
                               np.array([0.0, 4.0, 0.0, 0.0, 0.5 * 4.0]) / 50.0, atol=1e-14)
    np.testing.assert_allclose(od.viscous_flux(q, grad, 1, flow)[2], -2.0 / 50.0, atol=1e-15)
    # heat: v = 0, d(rho E)/dz = 1 with rho const -> de/dz = 1, flux mu gamma / Pr
    q = _state(1.0, 0.0, 0.0, 0.0, p)
    grad = np.zeros((3, 5))
    grad[2, 4] = 1.0
    np.testing.assert_allclose(od.viscous_flux(q, grad, 2, flow),
                               np.array([0.0, 0.0, 0.0, 0.0, 1.4 / 0.72]) / 50.0, atol=1e-14)


def test_sutherland_is_one_at_reference_temperature():
    assert abs(od.sutherland(np.array(1.0), FLOW) - 1.0) < 1e-15
    assert od.sutherland(np.array(2.0), FLOW) > 1.0


def test_lax_friedrichs_hand_values():
    ql = _state(1.0, 0.0, 0.0, 0.0, 1.0)
    qr = _state(0.5, 0.0, 0.0, 0.0, 1.0)
    lam = math.sqrt(1.4 * 1.0 / 0.5)
    f = od.lax_friedrichs(ql, qr, 0, FLOW)
    np.testing.assert_allclose(f, [0.25 * lam, 1.0, 0.0, 0.0, 0.0], atol=1e-15)
    # consistency: equal states give the physical flux
    q = _state(1.2, 0.3, -0.1, 0.2, 0.9)
    for d in range(3):
        np.testing.assert_allclose(od.lax_friedrichs(q, q, d, FLOW), od.euler_flux(q, d, FLOW), atol=1e-15)


# ---------------------------------------------------------------- operator

def test_free_stream_is_steady():
    g = od.Grid(2, 4)
    q = np.broadcast_to(_state(1.0, 0.3, -0.2, 0.1, 1.0 / (1.4 * 0.01)), (2, 2, 2, 5, 5, 5, 5)).copy()
    h = od.operator_h(q, g, FLOW)
    assert np.abs(h).max() < 1e-11
    assert np.abs(od.lifted_gradient(q, g)).max() < 1e-11


def test_conservation_on_discontinuous_state():
    g = od.Grid(2, 3)
    rng = np.random.default_rng(4)
    shp = (2, 2, 2, 4, 4, 4)
    q = _state(1.0 + 0.2 * rng.random(shp), 0.2 * rng.standard_normal(shp),
               0.2 * rng.standard_normal(shp), 0.2 * rng.standard_normal(shp), 50 + rng.random(shp))
    h = od.operator_h(q, g, FLOW)
    total = h.reshape(-1, 5).sum(axis=0)
    scale = np.abs(h).reshape(-1, 5).sum(axis=0)
    assert np.all(np.abs(total) <= 1e-13 * scale)


def _rel_err(h, grid, want):
    got = h / od.mass(grid)[..., None]
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


def test_advected_density_wave_converges():
    # inviscid limit: rho = 1 + 0.2 sin x, v = (U, 0, 0), p = P0
    flow = od.Flow(mach=0.5, reynolds=1e30)
    u0, p0 = 0.5, 1.0
    errs = []
    for n in (3, 5, 7):
        g = od.Grid(4, n)
        x, _, _ = _coords(g)
        rho = 1.0 + 0.2 * np.sin(x)
        q = _state(rho, u0, 0.0, 0.0, p0)
        drho = 0.2 * np.cos(x)
        want = np.stack([u0 * drho, u0 ** 2 * drho, 0 * x, 0 * x, 0.5 * u0 ** 3 * drho], axis=-1)
        errs.append(_rel_err(od.operator_h(q, g, flow), g, want))
    assert errs[0] < 0.05 and errs[1] < 5e-4 and errs[2] < 3e-6, errs
    assert errs[2] < errs[1] < errs[0]


def test_shear_flow_viscous_closed_form():
    # rho = 1, v = (U sin y, 0, 0), T const -> mu const; -div f^nu is closed form
    flow = od.Flow(mach=0.3, reynolds=1.0)
    u0 = 0.4
    p0 = 1.0 / (1.4 * 0.09)                 # T = 1, mu = 1
    errs = []
    for n in (3, 5, 7):
        g = od.Grid(4, n)
        _, y, _ = _coords(g)
        q = _state(1.0, u0 * np.sin(y), 0.0, 0.0, p0)
        want = np.stack([0 * y, u0 * np.sin(y), 0 * y, 0 * y, -u0 ** 2 * np.cos(2 * y)], axis=-1)
        errs.append(_rel_err(od.operator_h(q, g, flow), g, want))
    assert errs[0] < 0.25 and errs[1] < 8e-3 and errs[2] < 1e-4, errs
    assert errs[2] < errs[1] < errs[0]


def test_heat_conduction_closed_form():
    # rho = 1 + 0.1 sin z, v = 0, p = P0: only the heat flux acts
    flow = od.Flow(mach=0.3, reynolds=2.0)
    p0 = 1.0 / (1.4 * 0.09)

    def heat_flux(z):
        rho = 1.0 + 0.1 * np.sin(z)
        temp = 1.4 * 0.09 * p0 / rho
        mu = temp ** 1.5 * (1.0 + flow.sutherland) / (temp + flow.sutherland)
        de = -p0 * 0.1 * np.cos(z) / (0.4 * rho ** 2)
        return mu * 1.4 / 0.72 * de / flow.reynolds

    errs = []
    for n in (3, 5, 7):
        g = od.Grid(4, n)
        _, _, z = _coords(g)
        q = _state(1.0 + 0.1 * np.sin(z), 0.0, 0.0, 0.0, p0)
        eps = 1e-5
        dq = (heat_flux(z + eps) - heat_flux(z - eps)) / (2 * eps)
        want = np.stack([0 * z, 0 * z, 0 * z, 0 * z, -dq], axis=-1)
        errs.append(_rel_err(od.operator_h(q, g, flow), g, want))
    assert errs[0] < 0.25 and errs[1] < 8e-3 and errs[2] < 3e-4, errs


def test_lifted_gradient_converges():
    errs = []
    for n in (3, 5, 7):
        g = od.Grid(4, n)
        x, y, z = _coords(g)
        q = np.stack([np.sin(x), np.cos(y), np.sin(z + 0.3), np.sin(x) * np.cos(y), 2.0 + 0 * x],
                     axis=-1)
        grad = od.lifted_gradient(q, g)
        want = np.zeros(grad.shape)
        want[..., 0, 0] = np.cos(x)
        want[..., 1, 1] = -np.sin(y)
        want[..., 2, 2] = np.cos(z + 0.3)
        want[..., 0, 3] = np.cos(x) * np.cos(y)
        want[..., 1, 3] = -np.sin(x) * np.sin(y)
        errs.append(np.abs(grad - want).max())
    assert errs[0] < 0.06 and errs[1] < 6e-4 and errs[2] < 3e-6, errs


def test_piecewise_constant_state_reduces_to_face_fluxes():
    # elements constant, different along x; inviscid limit
    flow = od.Flow(mach=0.5, reynolds=1e30)
    g = od.Grid(2, 3)
    qa = _state(1.0, 0.2, 0.0, 0.0, 1.0)
    qb = _state(0.7, -0.1, 0.0, 0.0, 1.3)
    q = np.empty((2, 2, 2, 4, 4, 4, 5))
    q[:, :, 0] = qa
    q[:, :, 1] = qb
    h = od.operator_h(q, g, flow)
    _, w = od.gl_rule(3)
    jf = (g.h / 2) ** 2
    f_ab = od.lax_friedrichs(qa, qb, 0, flow)      # face between element 0 (left) and 1
    f_ba = od.lax_friedrichs(qb, qa, 0, flow)      # periodic face between 1 and 0
    for j in range(4):
        for k in range(4):
            wt = jf * w[j] * w[k]
            np.testing.assert_allclose(h[0, 0, 0, k, j, 3], wt * (f_ab - od.euler_flux(qa, 0, flow)) +
                                       0 * f_ab, atol=1e-12)
            np.testing.assert_allclose(h[0, 0, 0, k, j, 0], -wt * (f_ba - od.euler_flux(qa, 0, flow)),
                                       atol=1e-12)
            np.testing.assert_allclose(h[0, 0, 1, k, j, 3], wt * (f_ba - od.euler_flux(qb, 0, flow)),
                                       atol=1e-12)
    # interior nodes along x see no flux at all
    assert np.abs(h[:, :, :, :, :, 1:3]).max() < 1e-12


def test_jacobian_blocks_linearize_oracle_residual():
    from workload.cases import build_case, global_matrix_from_parts
    case = build_case(2, 3, reynolds=100.0, dt=1e-2, keep_parts=True)
    a = global_matrix_from_parts(case.parts)
    q = case.q_state.numpy().reshape(2, 2, 2, 4, 4, 4, 5)
    grid = od.Grid(2, 3)
    flow = od.Flow(mach=0.1, reynolds=100.0)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(q.shape)
    eps = 1e-6
    fd = (od.residual(q + eps * v, grid, flow, q, 1e-2) - od.residual(q - eps * v, grid, flow, q, 1e-2)) \
        / (2 * eps)
    av = a @ v.reshape(-1)
    assert np.abs(av - fd.reshape(-1)).max() <= 1e-6 * np.abs(av).max()
    # and B = -R(Q~) at Q~ = Q_s is the stored right-hand side
    np.testing.assert_allclose(case.rhs.numpy(), -od.residual(q, grid, flow).reshape(-1),
                               rtol=0, atol=1e-12 * np.abs(case.rhs.numpy()).max())


def test_planted_mistakes_are_caught(monkeypatch):
    """Plausible mistakes planted in the oracle each fail one of the pins above."""
    good_llf, good_visc, good_dm = od.lax_friedrichs, od.viscous_flux, od.lagrange_derivative

    # 1. dissipation with the wrong sign in the Rusanov flux
    def llf_flipped(qm, qp, d, flow):
        central = 0.5 * (od.euler_flux(qm, d, flow) + od.euler_flux(qp, d, flow))
        return 2.0 * central - good_llf(qm, qp, d, flow)

    monkeypatch.setattr(od, "lax_friedrichs", llf_flipped)
    with pytest.raises(AssertionError):
        test_lax_friedrichs_hand_values()
    monkeypatch.setattr(od, "lax_friedrichs", good_llf)

    # 2. the viscous flux off by a factor (half of it dropped)
    def visc_no_transpose(q, grad, d, flow):
        f = good_visc(q, grad, d, flow)
        g2 = grad.copy()
        return f + 0.5 * (good_visc(q, g2 * 0, d, flow) - f)

    monkeypatch.setattr(od, "viscous_flux", visc_no_transpose)
    with pytest.raises(AssertionError):
        test_viscous_flux_hand_values()
    with pytest.raises(AssertionError):
        test_shear_flow_viscous_closed_form()
    monkeypatch.setattr(od, "viscous_flux", good_visc)

    # 3. the derivative matrix transposed
    monkeypatch.setattr(od, "lagrange_derivative", lambda x: good_dm(x).T)
    with pytest.raises(AssertionError):
        test_advected_density_wave_converges()


# ---------------------------------------------------------------- curvilinear elements
# The perturbed map x = xi + A L s(xi) (1, 1, 1), s = sin xi_x sin xi_y sin xi_z
# (L = 2 pi), has d x / d xi_ref = (h/2) (I + 1 u^T) with u = A L grad s, so
#   J = (h/2)^3 (1 + sum u),   (J a^i)_n = (h/2)^2 ((1 + sum u) delta_in - u_n).

def _flow_params(reynolds):
    from workload.physics import FlowParams
    return FlowParams(mach=0.1, reynolds=reynolds)


def _curved(k, order, amplitude=0.05, kind="sine"):
    from workload.dgsem import Mesh, curved_node_coordinates, node_coordinates
    mesh = Mesh(k, order)
    return mesh, curved_node_coordinates(mesh, amplitude, kind), node_coordinates(mesh)


def _exact_metrics(xi, h, amplitude):
    L = 2.0 * math.pi
    s = [np.sin(xi[..., d]) for d in range(3)]
    c = [np.cos(xi[..., d]) for d in range(3)]
    u = amplitude * L * np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], axis=-1)
    su = u.sum(axis=-1)
    jac = (h / 2) ** 3 * (1 + su)
    ja = (h / 2) ** 2 * ((1 + su)[..., None, None] * np.eye(3) - u[..., None, :])
    return ja, jac


def test_curved_affine_map_reduces_to_cartesian():
    mesh, _, xi = _curved(2, 3)
    grid, flow = od.Grid(2, 3), od.Flow(0.1, 100.0)
    ja, jac = od.metric_terms(xi, grid)
    c = grid.h / 2
    np.testing.assert_allclose(ja, np.broadcast_to(c * c * np.eye(3), ja.shape), atol=1e-13 * c * c)
    np.testing.assert_allclose(jac, c ** 3, rtol=1e-13)
    from workload.dgsem import taylor_green_state
    q = taylor_green_state(mesh, _flow_params(100.0), seed=3)
    ref = od.operator_h(q, grid, flow)
    assert np.abs(od.operator_h_curved(q, grid, flow, ja, jac) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("order", [3, 4, 5, 7])
def test_curved_metrics_converge_to_the_map(order):
    _, xc, xi = _curved(3, order)
    grid = od.Grid(3, order)
    ja, jac = od.metric_terms(xc, grid)
    ja_x, jac_x = _exact_metrics(xi, grid.h, 0.05)
    assert jac.min() > 0
    # spectral convergence of the interpolated geometry; measured J: 3.6e-2,
    # 5.6e-3, 6.2e-4, 4.7e-6 and J a: 8.5e-2, 1.7e-2, 3.0e-3, 6.7e-5 (N = 3, 4, 5, 7)
    bound_j = {3: 5e-2, 4: 8e-3, 5: 1e-3, 7: 1e-5}[order]
    bound_ja = {3: 0.15, 4: 3e-2, 5: 6e-3, 7: 1.5e-4}[order]
    assert np.abs(jac - jac_x).max() <= bound_j * np.abs(jac_x).max()
    assert np.abs(ja - ja_x).max() <= bound_ja * np.abs(ja_x).max()


@pytest.mark.parametrize("kind", ["sine", "skew"])
def test_curved_metric_identities_hold_discretely(kind):
    _, xc, _ = _curved(3, 5, kind=kind)
    grid = od.Grid(3, 5)
    ja, _ = od.metric_terms(xc, grid)
    x, _ = od.gl_rule(5)
    dm = od.lagrange_derivative(x)
    div = sum(od._d_along(ja[..., i, :], 5 - i, dm) for i in range(3))
    assert np.abs(div).max() <= 1e-12 * np.abs(ja).max()
    # a rigid shift of the mesh changes nothing
    ja2, jac2 = od.metric_terms(xc + np.array([0.3, -1.7, 2.9]), grid)
    np.testing.assert_allclose(ja2, ja, rtol=0, atol=1e-12 * np.abs(ja).max())


@pytest.mark.parametrize("k,order,kind", [(2, 3, "sine"), (3, 4, "sine"), (3, 4, "skew")])
def test_curved_free_stream_is_preserved(k, order, kind):
    from workload.dgsem import uniform_state
    mesh, xc, _ = _curved(k, order, kind=kind)
    grid, flow = od.Grid(k, order), od.Flow(0.1, 100.0)
    ja, jac = od.metric_terms(xc, grid)
    q = uniform_state(mesh, _flow_params(100.0))
    h = od.operator_h_curved(q, grid, flow, ja, jac)
    p = 1.0 / (1.4 * 0.01)
    assert np.abs(h).max() <= 1e-12 * p * np.abs(ja).max()
    g = od.lifted_gradient_curved(q, grid, ja, jac)
    assert np.abs(g).max() <= 1e-12 * (np.abs(q).max() / grid.h)


def test_curved_residual_is_conservative():
    from workload.dgsem import taylor_green_state
    mesh, xc, _ = _curved(3, 4)
    grid, flow = od.Grid(3, 4), od.Flow(0.1, 1600.0)
    ja, jac = od.metric_terms(xc, grid)
    q = taylor_green_state(mesh, _flow_params(1600.0), seed=2, coords=xc)
    h = od.operator_h_curved(q, grid, flow, ja, jac).reshape(-1, 5)
    assert np.all(np.abs(h.sum(axis=0)) <= 1e-12 * np.abs(h).sum(axis=0))


def test_curved_planted_cross_product_metrics_break_the_free_stream(monkeypatch):
    good = od.metric_terms

    def cross_product(xyz, grid):
        ja, jac = good(xyz, grid)
        x, _ = od.gl_rule(grid.order)
        dm = od.lagrange_derivative(x)
        dX = np.stack([od._d_along(xyz, 5 - j, dm) for j in range(3)], axis=-2)
        for i in range(3):
            ja[..., i, :] = np.cross(dX[..., (i + 1) % 3, :], dX[..., (i + 2) % 3, :])
        return ja, jac

    monkeypatch.setattr(od, "metric_terms", cross_product)
    # on the "sine" map the cross products happen to satisfy the identities as
    # well (they are linear in grad s); the skew map tells the two forms apart
    with pytest.raises(AssertionError):
        test_curved_free_stream_is_preserved(3, 4, "skew")
