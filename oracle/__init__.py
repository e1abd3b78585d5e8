"""CPU FP64 oracle for the statically condensed GL-DGSEM implicit solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (its index conventions are re-derived here with plain loops) and it
never consumes a value produced by the GPU path.

What it computes (each function cites the passage it follows):
  * the global backward-Euler Jacobian A assembled from the per-element blocks
    and the uncondensed solution of A dQ = B (eq. NewtonLinSys1) by LAPACK
    dense LU or SuperLU;
  * the Schur-complement quantities of eq. SC_step1 / SC_step2 written out as
    their definitions, per element, with numpy, and the paper's condensed CPU
    route at full size (LAPACK LU of every A_ii, element Schur blocks, GMRES
    with point Jacobi on S, back-substitution) for timing and large parity runs;
  * (module `oracle.dgsem`) the nonlinear residual R(Q) = M (Q - Q_s)/dt + H(Q)
    of the backward-Euler GL-DGSEM step, with H from the weak form of
    eq. DGSEMsystem evaluated as Gauss-Lobatto quadrature sums;
  * (module `oracle.mlp`) the learned-initial-guess network in FP64: forward,
    chain-rule backward, Adam, mean-squared loss, the feature maps and the
    condensed-residual loss of a predicted increment;
  * (module `oracle.sparsity1d`) the Jacobian of the 1D scalar DGSEM on
    Gauss and Gauss-Lobatto nodes, for the sparsity claims of Section 3.1;
  * (module `oracle.mortar`) the residual of elements of uneven order on
    displaced trilinear hexahedra, coupled through mortars on faces between
    different orders, and its Newton matrix by complex step.
"""
from .linalg import (  # noqa: F401
    NodeSets, node_sets, dof_maps, assemble_global, solve_dense, solve_sparse,
    element_inverse, element_schur, condensed_matrix_dense, condensed_rhs,
    back_substitute, full_residual, gmres_mgs, condensed_solve_dense, element_interior_residual,
    full_residual_blocks, CondensedCPU, condense_cpu, schur_matvec_cpu, condensed_gmres_solve,
    solve_gmres_element_jacobi, achievable_ratio,
)
