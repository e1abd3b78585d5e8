"""Pins of the 1D Gauss-Lobatto operators (paper, Appendix C) against closed forms."""
import numpy as np
import pytest

from workload import gl


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_closed_form_nodes_weights(n):
    x, w = gl.gl_nodes_weights(n)
    xc, wc = gl.closed_form_nodes(n)
    np.testing.assert_allclose(x, xc, atol=1e-15)
    np.testing.assert_allclose(w, wc, atol=1e-15)


@pytest.mark.parametrize("n", range(1, 13))
def test_quadrature_exact_to_2n_minus_1(n):
    x, w = gl.gl_nodes_weights(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(0, 2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-13, (n, deg)
    # degree 2N is not integrated exactly (the Gauss-Lobatto limitation noted in the Introduction)
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-10


@pytest.mark.parametrize("n", range(1, 13))
def test_derivative_exact_and_sbp(n):
    x, w = gl.gl_nodes_weights(n)
    d = gl.derivative_matrix(n)
    for k in range(0, n + 1):
        deriv = k * x ** (k - 1) if k else np.zeros_like(x)
        np.testing.assert_allclose(d @ x ** k, deriv, atol=1e-11 * max(1, n ** 2))
    wd = np.diag(w) @ d
    np.testing.assert_allclose(wd + wd.T, gl.sbp_boundary(n), atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_discrete_orthogonality(n):
    x, _ = gl.gl_nodes_weights(n)
    np.testing.assert_allclose(gl.lagrange_eval(n, x), np.eye(n + 1), atol=1e-14)
    ends = gl.lagrange_eval(n, np.array([-1.0, 1.0]))
    # only one Lagrange polynomial is nonzero at each end point on GL nodes
    assert np.count_nonzero(np.abs(ends) > 1e-14, axis=1).tolist() == [1, 1]
