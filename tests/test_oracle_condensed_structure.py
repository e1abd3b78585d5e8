"""Structure of the condensed matrix (the paper's remarks on its Figure of the
condensation operations, Section 3.2): S keeps the diagonal dominance of A
with a denser structure, and with a viscous flux S couples elements two apart
(neighbours of neighbours) although A does not, which the purely advective
case does not show."""
import numpy as np
import pytest

import oracle
from oracle import linalg as ol
from oracle import sparsity1d as sp
from workload.cases import build_case


def _schur_1d(a, k, n):
    p = n + 1
    b = [e * p + j for e in range(k) for j in (0, n)]
    i = [e * p + j for e in range(k) for j in range(1, n)]
    return a[np.ix_(b, b)] - a[np.ix_(b, i)] @ np.linalg.solve(a[np.ix_(i, i)], a[np.ix_(i, b)])


def _element_reach(m, per_elem, k):
    """Largest periodic element distance between coupled rows and columns."""
    nz = np.abs(m) > 1e-12 * np.abs(m).max()
    r, c = np.nonzero(nz)
    d = np.abs(r // per_elem - c // per_elem)
    return int(np.minimum(d, k - d).max())


@pytest.mark.parametrize("nu,visc,reach_s", [(0.0, "br1", 1), (0.05, "compact", 2), (0.05, "br1", 2)])
def test_viscous_condensed_matrix_couples_neighbours_of_neighbours(nu, visc, reach_s):
    k, n = 7, 9
    a = sp.jacobian(k, n, "gl", nu=nu, viscous=visc)
    assert _element_reach(a, n + 1, k) == 1           # A couples direct neighbours only
    assert _element_reach(_schur_1d(a, k, n), 2, k) == reach_s


def test_condensed_ns_matrix_is_denser_and_keeps_diagonal_dominance():
    # a small step makes A strictly row diagonally dominant (the mass term leads;
    # at dt 1e-3 the energy rows are not yet, through the 1 / (gamma Ma^2) pressure)
    case = build_case(2, 3, 100.0, 1e-4, seed=0)
    aii, aib, abi, bbv = (x.numpy() for x in (case.aii, case.aib, case.abi, case.bb_val))
    a = oracle.assemble_global(case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib,
                               abi).toarray()
    s = ol.condensed_matrix_dense(case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, bbv, aii, aib, abi)
    dom = lambda m: np.abs(np.diag(m)) - (np.abs(m).sum(axis=1) - np.abs(np.diag(m)))
    assert dom(a).min() > 0
    assert dom(s).min() > 0
    abb = np.zeros_like(s)
    for g in range(case.n_bnodes):
        for t in range(case.bb_rowptr[g], case.bb_rowptr[g + 1]):
            h = case.bb_col[t]
            abb[5 * g:5 * g + 5, 5 * h:5 * h + 5] = bbv[t]
    dens = lambda m: np.mean(m != 0.0)          # structural: exact zeros where nothing couples
    assert dens(s) > 2.0 * dens(abb)
