"""Sparsity claims of the paper (Section 3.1, Jacobian Sparsity Patterns) on its
1D mesh: seven periodic elements of order 9 and a scalar equation, with the
1D DGSEM of oracle.sparsity1d on Gauss-Lobatto and on Gauss nodes.

The operator itself is pinned first (a constant state is steady, the scheme
is conservative, and a smooth periodic state gives d_x(a q - nu d_x q) at the
nodes to spectral accuracy), so the sparsity checks look at a correct
discretization."""
import numpy as np
import pytest

from oracle import sparsity1d as sp

K, N = 7, 9
P = N + 1


def _nz(b, a):
    return np.abs(b) > 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("kind", ["gl", "gauss"])
@pytest.mark.parametrize("nu,visc", [(0.0, "br1"), (0.05, "br1"), (0.05, "compact")])
def test_operator_is_a_consistent_conservative_discretization(kind, nu, visc):
    length = 2.0
    x, w = sp.nodes_weights(kind, N)
    jac = length / K / 2.0
    pos = np.array([[e * 2 * jac + jac * (xi + 1.0) for xi in x] for e in range(K)])
    # constant state: steady
    h0 = sp.operator_h(np.full((K, P), 3.0), kind, N, length=length, nu=nu, viscous=visc)
    assert np.abs(h0).max() < 1e-12
    # conservation: the sum of H over all DOFs vanishes (face fluxes cancel)
    rng = np.random.default_rng(1)
    hr = sp.operator_h(rng.standard_normal((K, P)), kind, N, length=length, nu=nu, viscous=visc)
    assert abs(hr.sum()) < 1e-11 * np.abs(hr).max()
    # smooth periodic state: H_j / (J w_j) = d_x (a q - nu d_x q) at the nodes
    kw = 2.0 * np.pi / length
    q = np.sin(kw * pos)
    h = sp.operator_h(q, kind, N, length=length, a=1.0, nu=nu, viscous=visc)
    exact = kw * np.cos(kw * pos) + nu * kw ** 2 * np.sin(kw * pos)
    assert np.abs(h / (jac * w[None, :]) - exact).max() < 1e-6 * np.abs(exact).max()


def test_gl_advective_off_diagonal_blocks_hold_one_entry():
    a = sp.jacobian(K, N, "gl", nu=0.0)
    for e in range(K):
        right, left = sp.block(a, P, e, (e + 1) % K), sp.block(a, P, e, (e - 1) % K)
        assert _nz(right, a).sum() == 1 and _nz(right, a)[N, 0]      # last node <- neighbour's first
        assert _nz(left, a).sum() == 1 and _nz(left, a)[0, N]        # first node <- neighbour's last
        for f in range(K):
            if f not in (e, (e + 1) % K, (e - 1) % K):
                assert not _nz(sp.block(a, P, e, f), a).any()


def test_gauss_off_diagonal_blocks_are_dense():
    for nu, visc in ((0.0, "br1"), (0.05, "compact")):
        a = sp.jacobian(K, N, "gauss", nu=nu, viscous=visc)
        for e in range(K):
            assert _nz(sp.block(a, P, e, (e + 1) % K), a).all()
            assert _nz(sp.block(a, P, e, (e - 1) % K), a).all()


def test_gl_diffusive_blocks_fill_one_row_and_one_column():
    a = sp.jacobian(K, N, "gl", nu=0.05, viscous="compact")
    for e in range(K):
        nz = _nz(sp.block(a, P, e, (e + 1) % K), a)
        want = np.zeros((P, P), dtype=bool)
        want[N, :] = True          # the shared-face node of e sees every node of the neighbour
        want[:, 0] = True          # every node of e sees the neighbour's shared-face node
        assert (nz == want).all()
        nz = _nz(sp.block(a, P, e, (e - 1) % K), a)
        want = np.zeros((P, P), dtype=bool)
        want[0, :] = True
        want[:, N] = True
        assert (nz == want).all()


@pytest.mark.parametrize("nu,visc", [(0.0, "br1"), (0.05, "br1"), (0.05, "compact")])
def test_gl_interior_block_is_block_diagonal(nu, visc):
    """Reordered into boundary (first and last node) and interior DOFs, A_ii
    couples no two elements: static condensation applies."""
    a = sp.jacobian(K, N, "gl", nu=nu, viscous=visc)
    interior = [e * P + j for e in range(K) for j in range(1, N)]
    elem = np.repeat(np.arange(K), P)
    aii = a[np.ix_(interior, interior)]
    ei = elem[interior]
    assert not _nz(aii, a)[ei[:, None] != ei[None, :]].any()


def test_br1_reach_depends_on_the_nodes():
    """In 1D, BR1's lifted gradient at a Gauss-Lobatto face node involves only
    that face, so the scheme stays compact; on Gauss nodes every node's
    gradient involves both faces and the element two away is coupled densely."""
    gl = sp.jacobian(K, N, "gl", nu=0.05, viscous="br1")
    ga = sp.jacobian(K, N, "gauss", nu=0.05, viscous="br1")
    for e in range(K):
        assert not _nz(sp.block(gl, P, e, (e + 2) % K), gl).any()
        assert _nz(sp.block(ga, P, e, (e + 2) % K), ga).all()


def test_planted_mistakes_fail_the_operator_pins(monkeypatch):
    good = sp.lagrange_at
    # element ends swapped in the boundary interpolation
    monkeypatch.setattr(sp, "lagrange_at", lambda x, xi: good(x, -xi))
    with pytest.raises(AssertionError):
        test_operator_is_a_consistent_conservative_discretization("gl", 0.0, "br1")
    monkeypatch.setattr(sp, "lagrange_at", good)
    # the derivative matrix transposed in the volume terms
    good_d = sp.lagrange_derivative
    monkeypatch.setattr(sp, "lagrange_derivative", lambda x: good_d(x).T)
    with pytest.raises(AssertionError):
        test_operator_is_a_consistent_conservative_discretization("gauss", 0.05, "compact")
