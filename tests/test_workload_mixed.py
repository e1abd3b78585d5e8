"""CPU checks of the mixed-order (uneven polynomial order) structure generator:
coupling sets and A_bb pattern are well formed, every row of the global
matrix is strictly diagonally dominant (so the system is nonsingular and the
condensed solve is well defined), and the oracle's condensed solve equals its
uncondensed solve on it."""
import numpy as np

import oracle
from workload.mixed import mixed_order_case
from workload.partition import coupling_size


def test_mixed_structure_and_oracle_consistency():
    c = mixed_order_case(2, lo=2, hi=5, seed=1)
    assert len(set(c.order.tolist())) >= 3
    for e in range(c.n_elem):
        ce = c.c_node[c.c_ptr[e]:c.c_ptr[e + 1]]
        assert np.all(np.diff(ce) > 0) and ce.min() >= 0 and ce.max() < c.n_bnodes
    for g in range(c.n_bnodes):
        cols = c.bb_col[c.bb_rowptr[g]:c.bb_rowptr[g + 1]]
        assert np.all(np.diff(cols) > 0) and g in cols
    d = dict(order=c.order, c_ptr=c.c_ptr, c_node=c.c_node, bb_rowptr=c.bb_rowptr, bb_col=c.bb_col,
             **c.element_blocks())
    a = oracle.assemble_global(**d).tocsr()
    diag = np.abs(a.diagonal())
    off = np.asarray(abs(a).sum(axis=1)).ravel() - diag
    assert np.all(diag - off > 0.1)
    b = c.rhs.numpy()
    x = oracle.solve_sparse(a, b)
    xc = oracle.condensed_solve_dense(b=b, **d)
    assert np.abs(xc - x).max() <= 1e-12 * np.abs(x).max()


def test_uniform_orders_reduce_to_conforming_coupling_size():
    c = mixed_order_case(2, lo=4, hi=4, seed=2)
    assert np.all(np.diff(c.c_ptr) == coupling_size(4))
