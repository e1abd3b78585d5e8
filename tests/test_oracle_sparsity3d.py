"""3D sparsity claims of the paper (Section 3.1): with tensor-product bases
the diagonal and off-diagonal blocks are no longer dense; on Gauss-Lobatto
nodes only face DOFs couple across elements, so A_ii is block-diagonal after
the boundary/interior reordering, while on Gauss nodes every DOF of an
element couples to its neighbours.  Scalar advection-diffusion on a periodic
3^3 mesh of order 3 (27 elements, so the two x-neighbours are distinct),
Jacobian by brute force from oracle.sparsity1d.operator_h3."""
import numpy as np
import pytest

from oracle import sparsity1d as sp

K, N = 3, 3
P = N + 1
P3 = P ** 3


def _elem(ex, ey, ez):
    return (ex % K) + K * (ey % K) + K * K * (ez % K)


def _nz(b, a):
    return np.abs(b) > 1e-13 * np.abs(a).max()


def _block(a, e, f):
    return a[e * P3:(e + 1) * P3, f * P3:(f + 1) * P3]


def _node(i, j, k):
    return i + P * j + P * P * k


@pytest.fixture(scope="module")
def mats():
    out = {}
    for kind in ("gl", "gauss"):
        for nu, visc in ((0.0, "br1"), (0.05, "br1"), (0.05, "compact")):
            out[(kind, nu, visc)] = sp.jacobian3(K, N, kind, nu=nu, viscous=visc)
    return out


def _sine_error(kind, order, length=2.0):
    """max |H / (J w w w) - (a (d_x + d_y + d_z) q - nu lap q)| / max|...| for
    q = sin(kx) sin(ky) on the 3^3 mesh."""
    p = order + 1
    x, w = sp.nodes_weights(kind, order)
    jac = length / K / 2.0
    line = np.array([[e * 2 * jac + jac * (xi + 1.0) for xi in x] for e in range(K)])     # [K, P]
    X = line[None, None, :, None, None, :]
    Y = line[None, :, None, None, :, None]
    shape = (K, K, K, p, p, p)
    kw = 2 * np.pi / length
    q = np.broadcast_to(np.sin(kw * X) * np.sin(kw * Y), shape)
    h = sp.operator_h3(q, kind, order, length=length, nu=0.05)
    www = (w[:, None, None] * w[None, :, None] * w[None, None, :])[None, None, None]
    exact = np.broadcast_to(kw * np.cos(kw * X) * np.sin(kw * Y) + kw * np.sin(kw * X) * np.cos(kw * Y)
                            + 0.05 * 2 * kw ** 2 * np.sin(kw * X) * np.sin(kw * Y), shape)
    return np.abs(h / (jac ** 3 * www) - exact).max() / np.abs(exact).max()


@pytest.mark.parametrize("kind", ["gl", "gauss"])
def test_3d_operator_is_consistent(kind):
    shape = (K, K, K, P, P, P)
    # constant state steady; conservation
    assert np.abs(sp.operator_h3(np.full(shape, 2.0), kind, N, nu=0.05)).max() < 1e-12
    hr = sp.operator_h3(np.random.default_rng(2).standard_normal(shape), kind, N, nu=0.05)
    assert abs(hr.sum()) < 1e-11 * np.abs(hr).max()
    # a smooth state: spectral convergence with the order (one wavelength over three elements)
    e3, e6 = _sine_error(kind, 3), _sine_error(kind, 6)
    assert e6 < 1e-3 and e6 < e3 / 100.0, (e3, e6)


def test_blocks_are_not_dense(mats):
    """Tensor-product bases: a node couples to the nodes of its own lines."""
    for kind in ("gl", "gauss"):
        a = mats[(kind, 0.0, "br1")]
        diag = _nz(_block(a, 0, 0), a)
        assert diag.sum(axis=1).max() == 3 * P - 2          # its three lines, itself once
        off = _nz(_block(a, 0, _elem(1, 0, 0)), a)
        assert 0 < off.mean() < 1


def test_gl_advective_neighbour_blocks_couple_face_nodes_one_to_one(mats):
    a = mats[("gl", 0.0, "br1")]
    nz = _nz(_block(a, 0, _elem(1, 0, 0)), a)
    want = np.zeros((P3, P3), dtype=bool)
    for j in range(P):
        for k in range(P):
            want[_node(N, j, k), _node(0, j, k)] = True    # +x face of e <- -x face of e + x
    assert (nz == want).all()
    # no coupling with edge or corner neighbours
    for f in (_elem(1, 1, 0), _elem(1, 1, 1), _elem(2, 1, 0)):
        assert not _nz(_block(a, 0, f), a).any()


def test_gauss_advective_every_dof_couples_to_the_neighbour(mats):
    a = mats[("gauss", 0.0, "br1")]
    nz = _nz(_block(a, 0, _elem(1, 0, 0)), a)
    assert nz.any(axis=1).all()                            # every DOF of e
    assert nz.sum() == P ** 4                              # along its x-line only: P^2 lines x P^2 pairs


@pytest.mark.parametrize("nu,visc", [(0.0, "br1"), (0.05, "br1"), (0.05, "compact")])
def test_gl_interior_block_is_block_diagonal(mats, nu, visc):
    a = mats[("gl", nu, visc)]
    interior = [e * P3 + _node(i, j, k) for e in range(K ** 3)
                for k in range(1, N) for j in range(1, N) for i in range(1, N)]
    elem = np.repeat(np.arange(K ** 3), P3)
    aii = a[np.ix_(interior, interior)]
    ei = elem[interior]
    assert not _nz(aii, a)[ei[:, None] != ei[None, :]].any()


def test_gauss_interior_dofs_couple_across_elements(mats):
    a = mats[("gauss", 0.05, "compact")]
    nz = _nz(_block(a, 0, _elem(1, 0, 0)), a)
    centre = _node(1, 1, 1)                                # an interior node on GL, not special on Gauss
    assert nz[centre].any()
