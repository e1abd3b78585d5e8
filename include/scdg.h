/*
 * scdg.h -- statically condensed GL-DGSEM implicit-step linear solve on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the Schur-complement solution of the Newton system of a
 * backward-Euler GL-DGSEM step, A dQ = B (paper, eq. NewtonLinSys1), after
 * reordering the unknowns into element-boundary DOFs Q_b and element-interior
 * DOFs Q_i (Section 3.1, eq. StaticDGSEM_QbQiSystem).  On Gauss-Lobatto nodes
 * the interior block A_ii is block-diagonal, one dense block per element
 * (Section 3.1, summary of the sparsity analysis), so
 *
 *     S   = A_bb - A_bi A_ii^-1 A_ib                         (eq. SC_step1)
 *     b_S = B_b  - A_bi A_ii^-1 B_i                          (eq. SC_step1)
 *     S Q_b = b_S,   Q_i = A_ii^-1 (B_i - A_ib Q_b)          (eq. SC_step2)
 *
 * SUBSCRIPTS ARE ROW-COLUMN: A_bi = A[b rows, i columns], A_ib = A[i rows,
 * b columns].  (The paper names the same blocks the other way round.)
 *
 * ------------------------------------------------------------------------
 * Data conventions
 * ------------------------------------------------------------------------
 * Element e has polynomial order N_e (2 <= N_e <= 7), P = N_e + 1 nodes per
 * direction, local node n = i + P j + P^2 k, and 5 conserved variables.
 *   - Natural vectors (B, dQ, r, x0): device, double, DOF index
 *     (sum_{e'<e} 5 P_{e'}^3) + 5 n + v.
 *   - Interior nodes of e: i, j, k all in [1, N_e-1], in increasing n;
 *     n_i(e) = 5 (N_e - 1)^3 DOFs.  With physical boundaries (phys_faces in
 *     scdg_structure) a node also counts as interior when every element face
 *     it lies on is physical: such DOFs couple to no other element, so they
 *     join Q_i (the achievable ratio of Section 3.2).
 *   - Boundary nodes of e: the other nodes in increasing n; the r-th one has
 *     global boundary id bnode_off[e] + r, bnode_off = exclusive prefix sum of
 *     (P^3 - (N_e-1)^3).  Boundary vectors (b_S, Q_b): device, double,
 *     index 5 g + v, length n1 = 5 n_bnodes.
 *   - Coupling set C_e: the global boundary nodes whose DOFs share a nonzero
 *     with an interior DOF of e, ascending; n_c(e) = 5 |C_e|.
 *   - Blocks, device, double, row-major, packed element after element:
 *       A_ii(e) [n_i x n_i], A_ib(e) [n_i x n_c], A_bi(e) [n_c x n_i];
 *     A_bb in BSR with 5x5 row-major blocks over global boundary nodes.
 *
 * Ownership and streams: the caller owns every buffer passed in.  Blocks given
 * to scdg_assemble are copied into plan-owned storage (SCDG_COPY) or
 * BORROWED until the next scdg_assemble or scdg_plan_destroy (SCDG_BORROW;
 * the FP64 originals are read again by the full-system residual).  The plan
 * owns its factors, Schur blocks and workspaces.  Every
 * call enqueues work on the plan's HIP stream; calls that return host data
 * (scdg_solve*, scdg_residual, scdg_factor_info) synchronize that stream.
 * A plan is not thread-safe; distinct plans are independent.
 *
 * Errors: every call returns scdg_status; nothing throws or aborts across the
 * ABI.  Argument and call-order errors return before any work is enqueued.
 * Call order: plan_create -> assemble -> factor -> condense -> (condense_rhs,
 * solve_condensed, backsolve | solve)*; assemble invalidates later stages.
 */
#ifndef SCDG_H
#define SCDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct scdg_plan scdg_plan;

typedef enum {
  SCDG_OK = 0,
  SCDG_ERR_ARG = -1,        /* bad pointer, size or option */
  SCDG_ERR_STATE = -2,      /* call out of order */
  SCDG_ERR_HIP = -3,        /* HIP runtime error (text in scdg_last_error) */
  SCDG_ERR_NOMEM = -4,      /* device allocation failed */
  SCDG_ERR_SINGULAR = -5,   /* zero / non-finite pivot in some A_ii(e) or S */
  SCDG_ERR_NOCONV = -6,     /* iteration budget exhausted; outputs hold the best iterate */
  SCDG_ERR_NONFINITE = -7,  /* NaN / Inf met in a right-hand side or residual */
  SCDG_ERR_UNSUPPORTED = -8 /* order or size outside what the library handles */
} scdg_status;

typedef enum { SCDG_FP64 = 0, SCDG_FP32 = 1 } scdg_precision;

/* Mesh structure; all pointers are HOST memory and are copied at create. */
typedef struct {
  int32_t n_elem;
  const int32_t *order;     /* [n_elem] polynomial order N_e, 2..7 */
  const int64_t *c_ptr;     /* [n_elem+1] offsets into c_node */
  const int32_t *c_node;    /* [c_ptr[n_elem]] C_e as ascending global boundary ids */
  const int64_t *bb_rowptr; /* [n_bnodes+1] BSR row pointer of A_bb */
  const int32_t *bb_col;    /* [bb_rowptr[n_bnodes]] BSR block columns of A_bb */
  const uint8_t *phys_faces; /* [n_elem] or NULL (no physical boundary): bit 2 d + s is set when the
                                element face of direction d (0: i, 1: j, 2: k) on side s (0: index 0,
                                1: index N_e) lies on a physical boundary (Section 2.1.1: its outer
                                state is a boundary condition, not a neighbour); bits 6, 7 must be 0 */
} scdg_structure;

typedef enum { SCDG_SOLVER_AUTO = 0, SCDG_SOLVER_DENSE = 1, SCDG_SOLVER_GMRES = 2 } scdg_solver;

/* Options of the condensed solve (zero-initialised fields take the defaults). */
typedef struct {
  int32_t solver;     /* scdg_solver; AUTO = dense LU of S when n1 <= 8192, else GMRES */
  int32_t restart;    /* GMRES restart length m (default 30) */
  int32_t max_iters;  /* total GMRES iterations (default 1000) */
  double tol;         /* GMRES stop: ||b_S - S x||_2 <= tol ||b_S||_2 (default 1e-10) */
  int32_t precond;    /* right preconditioner: 0 none, 1 point Jacobi on diag(S), 2 Jacobi on
                         the 5x5 diagonal node blocks of S (default: 1; -1 selects it) */
  int32_t ir_max;     /* iterative-refinement sweeps for FP32 factors (default 10) */
  double ir_tol;      /* refinement stop on ||B - A dQ||_2 / ||B||_2 (default 1e-8) */
} scdg_solve_opts;

typedef struct {
  int32_t iters;        /* GMRES iterations, all sweeps */
  int32_t restarts;     /* GMRES restart cycles, all sweeps */
  int32_t ir_sweeps;    /* condensed solves performed by scdg_solve */
  int32_t solver_used;  /* scdg_solver actually used */
  double rel_res_S;     /* last ||b_S - S x|| / ||b_S|| (GMRES estimate) */
  double rel_res_full;  /* ||B - A dQ||_2 / ||B||_2 in FP64, or -1 if not computed */
  int32_t guess_rejected; /* 1 if the initial guess was dropped: ||b_S - S x0|| > ||b_S|| */
  double rel_res_guess;   /* ||b_S - S x0|| / ||b_S|| of the first sweep's guess (1 without one) */
} scdg_solve_info;

/* Build the index maps of the partition (Section 3.2: permutation indexes from
 * the mesh connectivity), the Schur-apply maps and the work lists.  hip_stream
 * may be NULL (default stream) and must belong to the plan's device.  device:
 * -1 for the current HIP device, else a device index, which is made current
 * for the calling thread (SCDG_ERR_ARG if there is no such device).  Every
 * later call on the plan that enqueues work must be made with that device
 * current: SCDG_ERR_STATE otherwise. */
scdg_status scdg_plan_create(scdg_plan **out, const scdg_structure *s, void *hip_stream, int32_t device);
scdg_status scdg_plan_destroy(scdg_plan *p);
scdg_status scdg_set_stream(scdg_plan *p, void *hip_stream);
/* Sizes: natural DOFs, n1 = 5 n_bnodes (condensed size), n2 = sum n_i, n_bnodes. */
scdg_status scdg_plan_sizes(const scdg_plan *p, int64_t *n_dof, int64_t *n1, int64_t *n2,
                            int64_t *n_bnodes);

/* Number of A_bb node blocks folded into element Schur blocks and left in the
 * BSR remainder (see scdg_condense). */
scdg_status scdg_plan_fold_counts(const scdg_plan *p, int64_t *n_folded, int64_t *n_remainder);

/* Register the Jacobian blocks (device pointers, FP64) of A dQ = B
 * (eq. NewtonLinSys1) in the partition of Section 3.1.  flags:
 *   SCDG_COPY   (0)  the plan copies the four arrays into storage it owns
 *                    (allocated by the first copying call, freed by
 *                    scdg_plan_destroy) on its stream; the caller may reuse
 *                    its buffers as soon as the copy has run on that stream;
 *   SCDG_BORROW (1)  the plan keeps the caller's pointers until the next
 *                    scdg_assemble or scdg_plan_destroy (no copy; needed
 *                    where the blocks are large, 27 GB in FP64 at N = 7);
 *                    the caller must not change or free them meanwhile.
 * SCDG_ERR_ARG for NULL pointers or other flags; SCDG_ERR_NOMEM if the copy's
 * storage cannot be allocated. */
enum { SCDG_COPY = 0, SCDG_BORROW = 1 };
scdg_status scdg_assemble(scdg_plan *p, const double *aii, const double *aib,
                          const double *abi, const double *bb_val, int32_t flags);

/* Invert every A_ii(e) by Gauss-Jordan elimination with partial pivoting
 * (the paper inverts each interior block with LU routines, Section 3.2), in
 * FP64 or FP32.  A zero pivot is recorded per element (see scdg_factor_info)
 * and reported as SCDG_ERR_SINGULAR by scdg_condense. */
scdg_status scdg_factor(scdg_plan *p, scdg_precision prec);
/* Where the GMRES cycle runs (paper, Section 4 uses GMRES on the Newton
 * systems; this is an execution choice, same arithmetic):
 *   0  host-driven: one device-to-host transfer and wait per iteration for the
 *      Hessenberg column; Givens rotations on the host (default);
 *   1  device-resident: Hessenberg column, Givens rotations, stopping test and
 *      the next basis vector's scale stay on the device; every kernel of an
 *      Arnoldi step returns at once when a halt flag is set; the host waits once
 *      per restart cycle (true residual);
 *   2  as 1, with the m Arnoldi steps captured once into a HIP graph (on a
 *      plan-owned stream) and replayed per cycle on the plan's stream.  The
 *      graph is recaptured when the restart length, preconditioner, factor
 *      precision or the borrowed A_bb pointer change.  Phase timers do not see
 *      the kernels inside the graph. */
scdg_status scdg_set_krylov_mode(scdg_plan *p, int32_t mode);
/* Form of the Schur products S x inside the GMRES solve.  The paper assembles
 * S (Section 2.2, eq. SC_step1); applying it through its factors instead is
 * an execution choice with the same operator:
 *   0  assembled (default): scdg_condense forms the element blocks
 *      T_e = F_e - A_bi(e) X_e and every product streams them plus the A_bb
 *      remainder;
 *   1  matrix-free: scdg_condense forms X_e = A_ii(e)^-1 A_ib(e) only, plus the
 *      Jacobi blocks of S from the diagonal blocks of A_bb and of A_bi(e) X_e;
 *      every product is S x = A_bb x - sum_e P_e A_bi(e) (X_e x[C_e]), reading
 *      X_e, A_bi(e) and all of A_bb instead of T_e and the remainder;
 *   2  matrix-free and block-sparse: as 1, but every product is
 *      S x = A_bb x - sum_e P_e A_bi(e) (A_ii(e)^-1 (A_ib(e) x[C_e])) through
 *      the nonzero 5x5 blocks of A_ib and A_bi only (the paper notes the
 *      tensor-product sparsity of these blocks, Section 3.1).  scdg_condense
 *      finds the nonzero blocks from the values (zero blocks are skipped
 *      exactly), rebuilds its block lists when that pattern changed, and
 *      copies the nonzero blocks in the factor precision.
 * Changing the form sends a condensed plan back to the factored state (call
 * scdg_condense again).  The dense solve of S and scdg_export(SCDG_EXPORT_SCHUR)
 * need form 0: in forms 1 and 2 they return SCDG_ERR_STATE, and
 * SCDG_SOLVER_AUTO selects GMRES.  SCDG_ERR_ARG for a mode other than 0..2. */
scdg_status scdg_set_schur_mode(scdg_plan *p, int32_t mode);
scdg_status scdg_get_schur_mode(const scdg_plan *p, int32_t *mode);

/* Form of the batched inverse (Gauss-Jordan with partial pivoting, Section 3.2):
 * 0 automatic (form 3 up to n_i = 400, else form 2); 1 one workgroup per element for the whole elimination, 24- or
 * 32-column panels in LDS; 2 blocked: outer panels of 128 columns whose update
 * of the rest of the block is a batched matrix-core GEMM; 3 resident panel:
 * one workgroup per element holding an outer panel of 48 (FP64; 32 when some
 * n_i exceeds 320) or 64 (FP32) columns in LDS, so the rest of the block is
 * streamed once per outer panel (n_i <= 400, SCDG_ERR_UNSUPPORTED from
 * scdg_factor otherwise).  All
 * forms use the same pivot rule (largest |a| among unused rows, lowest row on
 * ties); rounding differs with the blocking, so near-ties may pick different
 * rows.  SCDG_ERR_ARG for a mode other than 0..3.  scdg_get_inverse_mode
 * reports the form used by the last scdg_factor (0 before). */
scdg_status scdg_set_inverse_mode(scdg_plan *p, int32_t mode);
scdg_status scdg_get_inverse_mode(const scdg_plan *p, int32_t *mode_used);
/* First singular element (or -1) and its LAPACK-style info (1-based step). */
scdg_status scdg_factor_info(scdg_plan *p, int64_t *first_bad_elem, int32_t *info);

/* X_e = A_ii(e)^-1 A_ib(e) and the element blocks of the condensed matrix
 * (eq. SC_step1).  S = A_bb - sum_e P_e A_bi(e) X_e P_e^T is stored as
 *     S = R + sum_e P_e T_e P_e^T,   T_e = F_e - A_bi(e) X_e,
 * where the A_bb block (g, h) is folded into F_e of the element e that owns
 * node g if both g and h lie in C_e, else of the lowest-numbered element whose
 * C_e holds both; blocks with no such element form the remainder R (BSR).
 * Uses the precision given to scdg_factor. */
scdg_status scdg_condense(scdg_plan *p);

/* b_S = B_b - sum_e P_e A_bi(e) A_ii(e)^-1 B_i(e) (eq. SC_step1).  b: natural
 * vector, bs: boundary vector (both device). */
scdg_status scdg_condense_rhs(scdg_plan *p, const double *b, double *bs);

/* Solve S Q_b = b_S: dense LU with partial pivoting of the assembled S, or
 * restarted GMRES(m) with right point-Jacobi and classical Gram-Schmidt with
 * reorthogonalisation (the paper's solvers: direct, and GMRES with a point-
 * Jacobi preconditioner, Section 4).  x0 (boundary vector) may be NULL. */
scdg_status scdg_solve_condensed(scdg_plan *p, const double *bs, double *qb, const double *x0,
                                 const scdg_solve_opts *o, scdg_solve_info *info);

/* Q_i(e) = A_ii(e)^-1 (B_i(e) - A_ib(e) Q_b[C_e]) (eq. SC_step2); writes the
 * whole natural vector dQ (boundary part copied from qb). */
scdg_status scdg_backsolve(scdg_plan *p, const double *b, const double *qb, double *dq);

/* Full solve of A dQ = B: condensed RHS, condensed solve, back-substitution.
 * With FP32 factors the FP64 full-system residual drives iterative
 * refinement until ||B - A dQ|| <= ir_tol ||B||.  x0 (natural vector) may be
 * NULL; its boundary part seeds the first condensed solve. */
scdg_status scdg_solve(scdg_plan *p, const double *b, double *dq, const double *x0,
                       const scdg_solve_opts *o, scdg_solve_info *info);

/* r = B - A dQ on the full FP64 system; rel2 (host, may be NULL) receives
 * ||r||_2 / ||B||_2.  r may be NULL when only rel2 is wanted. */
scdg_status scdg_residual(scdg_plan *p, const double *b, const double *dq, double *r,
                          double *rel2);

/* y = S x with the condensed operator as stored (boundary vectors, device). */
scdg_status scdg_schur_apply(scdg_plan *p, const double *x, double *y);
/* y = S^T x with the condensed operator as stored (eq. SC_step1: S^T =
 * A_bb^T - sum_e A_ib(e)^T A_ii(e)^-T A_bi(e)^T): the transposed element Schur
 * blocks and the transposed A_bb remainder, gathered and pulled exactly as
 * scdg_schur_apply does (for residual-weighted objectives, e.g. the gradient
 * S^T S e of ||S e||^2).  Boundary vectors of n1 doubles on the device; x and
 * y must differ.  Needs a condensed plan in the assembled form (schur mode
 * 0): SCDG_ERR_STATE otherwise.  Asynchronous on the plan's stream. */
scdg_status scdg_schur_apply_transpose(scdg_plan *p, const double *x, double *y);

/* Condensed-residual error of a predicted increment, for training the learned
 * initial guess (Section 3.2: the guess seeds GMRES on S Q_b = b_S, whose
 * starting residual is b_S - S x0_b = S (Q_b - x0_b)).  y and t are network
 * outputs and targets in the normalised natural order of scdg_guess_target
 * (n_dof floats each, device; either may be NULL for zero), stats the 25
 * device doubles of scdg_guess_stats whose entries 15..19 (rc) scale them back:
 *   e = P_b (rc (y - t)),  *loss = scale ||S e||_2^2 (one device double),
 *   dy = d loss / d y = 2 scale rc P_b^T S^T S e (n_dof floats, device; zero
 *   on interior DOFs; may be NULL to evaluate the loss only).
 * P_b restricts a natural vector to the plan's boundary vector.  Uses the
 * plan's boundary workspace (no other call may run on the plan meanwhile);
 * needs a condensed plan in the assembled form (schur mode 0), SCDG_ERR_STATE
 * otherwise; SCDG_ERR_ARG for scale < 0 or both y and t NULL.  Asynchronous
 * on the plan's stream. */
scdg_status scdg_guess_schur_loss(scdg_plan *p, const float *y, const float *t, const double *stats,
                                  double scale, float *dy, double *loss);

/* Copy internal arrays to caller device memory (for inspection and tests):
 * SCDG_EXPORT_AII_INV: sum n_i^2 values of A_ii(e)^-1; SCDG_EXPORT_SCHUR:
 * sum n_c^2 values of T_e; SCDG_EXPORT_X: sum n_i n_c values of X_e; all in the
 * factor precision (double or float). */
enum { SCDG_EXPORT_AII_INV = 1, SCDG_EXPORT_SCHUR = 2, SCDG_EXPORT_X = 3 };
scdg_status scdg_export(scdg_plan *p, int what, void *dst, size_t dst_bytes);

/* Device-time accounting per phase, measured with HIP events recorded on the
 * plan's stream around each launch (asynchronous; off by default). */
typedef enum {
  SCDG_PHASE_INVERSE = 0,     /* batched Gauss-Jordan inverse of A_ii */
  SCDG_PHASE_GEMM_X = 1,      /* X_e = A_ii^-1 A_ib */
  SCDG_PHASE_GEMM_S = 2,      /* element Schur blocks A_bi X_e */
  SCDG_PHASE_RHS = 3,         /* condensed right-hand side */
  SCDG_PHASE_SCHUR_APPLY = 4, /* one product with S (element blocks + A_bb) */
  SCDG_PHASE_CONDENSED = 5,   /* a whole condensed solve (GMRES or dense LU + solve) */
  SCDG_PHASE_BACKSOLVE = 6,   /* back-substitution */
  SCDG_PHASE_RESIDUAL = 7,    /* full-system FP64 residual */
  SCDG_PHASE_COUNT = 8
} scdg_phase;
scdg_status scdg_enable_timing(scdg_plan *p, int on);
/* Sum of event-measured milliseconds and launch counts per phase since the
 * previous call (then reset).  Synchronizes the stream.  ms and count are host
 * arrays of n entries (n <= SCDG_PHASE_COUNT). */
scdg_status scdg_phase_times(scdg_plan *p, double *ms, int32_t *count, int32_t n);

/* Tile autotuner for the two batched GEMMs of scdg_condense (X_e and the
 * element Schur blocks): every tile configuration is timed on the plan's own
 * problems (HIP events, best of two runs) and the fastest is kept.  Needs
 * scdg_factor; leaves the plan factored but not condensed.  ms_x / ms_s (host,
 * n entries, may be NULL) receive the time per configuration (-1 if skipped). */
scdg_status scdg_autotune(scdg_plan *p, double *ms_x, double *ms_s, int32_t n);
/* Select / query the tile configuration of the two GEMMs (0 .. 8). */
scdg_status scdg_set_gemm_config(scdg_plan *p, int32_t cfg_x, int32_t cfg_s);
scdg_status scdg_get_gemm_config(const scdg_plan *p, int32_t *cfg_x, int32_t *cfg_s);

/* ------------------------------------------------------------------------
 * Nonlinear residual of the implicit step (paper, eq. ImplicitDisc with
 * backward Euler, and eq. DiscretNS):
 *
 *     R(Q) = M (Q - Q_s) / dt + H(Q),
 *
 * H the GL-DGSEM operator of eq. DGSEMsystem for the compressible
 * Navier-Stokes equations (Appendix B fluxes, local Lax-Friedrichs advective
 * flux, Bassi-Rebay 1 or interior-penalty viscous flux and lifted gradient), M the diagonal mass
 * matrix J w_i w_j w_k, on a periodic Cartesian mesh of K^3 cubes of side
 * length / K with uniform order N.  B = -R(Q~) is the right-hand side of the
 * Newton system that scdg_solve solves (eq. NewtonLinSys1).
 *
 * Nondimensional state: p = (gamma - 1)(rho E - rho |v|^2 / 2), T = gamma
 * Ma^2 p / rho, Sutherland viscosity mu(T) = (1 + S) T^{3/2} / (T + S),
 * heat flux (mu gamma / Pr) grad e, Stokes stress with bulk term -2/3 mu div v,
 * viscous fluxes scaled by 1/Re.
 *
 * Vectors are device arrays of doubles in the natural DOF order of this
 * header: element e = ex + K ey + K^2 ez, node n = i + P j + P^2 k, DOF
 * 5 (e P^3 + n) + v.  The object owns its gradient workspace (15 doubles per
 * node); it is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct scdg_dg scdg_dg;
typedef struct {
  int32_t k_elem;           /* elements per direction K >= 2 */
  int32_t order;            /* N, 2 <= N <= 7 */
  double length;            /* side of the periodic box (> 0) */
  double mach, reynolds;    /* reference Mach and Reynolds numbers (> 0) */
  double gamma, prandtl;    /* <= 0 selects 1.4 / 0.72 */
  double sutherland_ratio;  /* T_suth / T_ref; <= 0 selects 110.4 / 288.15 */
  int32_t viscous_flux;     /* SCDG_VISCOUS_BR1 (0) or SCDG_VISCOUS_SIPG (1), see below */
  double sipg_eta;          /* interior-penalty factor eta (>= 0; 0 selects 1) */
} scdg_dg_params;
/* Face viscous flux.  BR1 (Bassi-Rebay 1): {{f^nu(q, g)}} with the lifted
 * gradients g of both sides.  SIPG (symmetric interior penalty, the paper's
 * choice for its example, Section 4; a compact flux, Section 3.1): the volume
 * term keeps the lifted gradient, whose surface value {{q}} supplies the
 * symmetric term, and the face flux is
 *     {{f^nu(q, grad q)}} + sigma f^nu({{q}}, [[q]] n),
 * with grad q each side's broken gradient (the derivative of its own
 * interpolant), [[q]] = q^- - q^+ taken as a gradient along the face normal n,
 * sigma = eta (N + 1)^2 / h.  SIPG needs Cartesian cubes (scdg_dg_set_geometry
 * returns SCDG_ERR_UNSUPPORTED) and keeps a second gradient workspace. */
enum { SCDG_VISCOUS_BR1 = 0, SCDG_VISCOUS_SIPG = 1 };
/* Create on the current device; HIP stream may be NULL (default stream).
 * SCDG_ERR_ARG for out-of-range parameters, SCDG_ERR_NOMEM on allocation. */
scdg_status scdg_dg_create(scdg_dg **out, const scdg_dg_params *prm, void *hip_stream);
scdg_status scdg_dg_destroy(scdg_dg *dg);
/* r = M (q - q_s) * inv_dt + H(q); q_s == NULL gives r = H(q).  q, q_s and r
 * hold 5 K^3 (N+1)^3 doubles; r must not alias q or q_s.  Asynchronous on the
 * object's stream. */
scdg_status scdg_dg_residual(scdg_dg *dg, const double *q, const double *q_s, double inv_dt,
                             double *r);
/* Curved hexahedra: xyz (host, 3 doubles per node, natural node order, the
 * physical position of every GL node, i.e. the element mapping sampled at its
 * nodes) replaces the Cartesian cubes.  The library forms the metric terms in
 * the conservative curl form, (J a^i)_n = - e_i . curl_xi(X_l grad_xi X_m) for
 * (n, m, l) cyclic (so a uniform state stays steady), and J = det(dx/dxi); H
 * then uses the contravariant fluxes sum_n (J a^i)_n f_n, face fluxes along
 * J a^i and the mass J w_i w_j w_k (the paper's eq. DGSEMsystem on mapped
 * elements).  The mesh must stay periodic with watertight faces (shared face
 * nodes at the same positions, up to a period).  xyz == NULL returns to the
 * Cartesian cubes.  Synchronizes the object's stream; SCDG_ERR_ARG if some J
 * is not positive and finite (the previous geometry is kept). */
scdg_status scdg_dg_set_geometry(scdg_dg *dg, const double *xyz);
/* Copy the lifted gradient of the last scdg_dg_residual call into g (device,
 * 15 doubles per node: g[(e P^3 + n) 15 + 5 d + v] = d q_v / d x_d). */
scdg_status scdg_dg_gradient(scdg_dg *dg, double *g);
/* The Newton matrix of the implicit step (eq. NewtonLinSys1: A = dR/dQ at q,
 * the same operator whose element blocks scdg_assemble takes) applied to v:
 *
 *     out = A v = M v * inv_dt + dH/dQ(q) v,
 *
 * exact to rounding, by forward-mode differentiation of the residual sums on
 * dual numbers (no difference step).  Where H is not differentiable the
 * derivative follows the branch the residual takes: |v . n| contributes
 * sign(v . n) at a nonzero argument and nothing at zero, and the larger
 * Lax-Friedrichs speed is the left state's at a tie.  Cartesian or curved, as
 * set by scdg_dg_set_geometry.  q, v and out hold 5 K^3 (N+1)^3 doubles
 * (device, natural DOF order); out must not alias q or v; inv_dt >= 0 (0 gives
 * dH/dQ v alone).  The first call allocates a second gradient workspace (15
 * doubles per node, freed by scdg_dg_destroy); the gradient workspace that
 * scdg_dg_gradient reads then holds the lifted gradient of q.  Asynchronous
 * on the object's stream.  SCDG_ERR_ARG for NULL pointers or a negative or
 * non-finite inv_dt, SCDG_ERR_NOMEM if the workspace cannot be allocated. */
scdg_status scdg_dg_jacobian_apply(scdg_dg *dg, const double *q, const double *v, double inv_dt, double *out);
/* Allocation-free form of scdg_dg_jacobian_apply, for callers that cannot
 * allocate device memory during the call: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same operator, same kernels,
 * same arguments and results; the lifted gradient of the direction v is kept
 * in a fixed device array of SCDG_NOALLOC_SCRATCH_BYTES compiled into the
 * library (one copy per GPU, resident until the process ends, its address
 * looked up once per device when a scdg_dg object is created) instead of a
 * workspace allocated on the first call.  The call allocates and frees
 * nothing.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams, or different host threads) race and give
 * undefined results; calls ordered on one stream are safe (the array needs no
 * clearing: each call writes all of the part it reads).
 * SCDG_ERR_UNSUPPORTED when the mesh needs more than the array holds
 * (15 * 8 bytes per node: at most 559 240 nodes, e.g. 16^3 elements of order 4)
 * or the object uses the interior-penalty flux (SCDG_VISCOUS_SIPG);
 * SCDG_ERR_ARG as for scdg_dg_jacobian_apply; SCDG_ERR_HIP if the array's
 * address could not be found on the object's device. */
#define SCDG_NOALLOC_SCRATCH_BYTES (64ll << 20)
scdg_status scdg_dg_jacobian_apply_noalloc(scdg_dg *dg, const double *q, const double *v, double inv_dt,
                                           double *out);

/* Element blocks of the backward-Euler Newton matrix A = M inv_dt + dH/dQ(q)
 * (eq. NewtonLinSys1), formed on the device from the state q by the chain
 * rule: the linearised Lax-Friedrichs advective flux (Section 2.1.1) and the
 * linearised Bassi-Rebay 1 viscous flux through the lifted gradient
 * (Section 2.1.2, eq. GradDGImp).  Pointwise 5x5 flux Jacobians are taken on
 * dual numbers (the same branches as scdg_dg_jacobian_apply at the kinks of
 * |u| and of the larger face speed); every node block of A is their linear
 * combination with coefficients of the mesh (Gauss-Lobatto weights, the
 * derivative matrix, the element size), built once per order on the host.
 * The blocks are written in the plan's format (interior / element-boundary
 * partition of Section 3.1, the layout scdg_assemble takes):
 *   aii [n_elem n_i^2], aib [n_elem n_i n_c], abi [n_elem n_c n_i]
 *   (row-major, node-major with the 5 variables fastest), and
 *   bb_val [nnzb * 25] over the plan's A_bb pattern;
 * every entry of the four arrays is overwritten (device pointers).  q holds
 * 5 K^3 (N+1)^3 doubles in the DG object's layout.  Requirements: the DG
 * object describes Cartesian cubes (no scdg_dg_set_geometry) with the
 * Bassi-Rebay 1 flux, and the plan is its periodic K^3 mesh of the same
 * uniform order with no physical faces; otherwise SCDG_ERR_UNSUPPORTED.
 * SCDG_ERR_ARG for NULL pointers, a negative or non-finite inv_dt, or a
 * nonzero block outside the plan's coupling sets or A_bb pattern (the
 * outputs are then incomplete).  Runs on the DG object's stream.  A call
 * with a plan other than the previous call's checks (one synchronisation)
 * that the plan's coupling sets and A_bb pattern hold a place for every block
 * the template can fill; when they do, this call and the following ones with
 * the same plan return without waiting for the stream.  Otherwise every call
 * returns after the stream, having checked that no block without a place is
 * nonzero.  Workspaces (the term template
 * and about 3.4 KB of pointwise Jacobians per node) are allocated on the
 * first call and freed by scdg_dg_destroy. */
scdg_status scdg_dg_jacobian_blocks(scdg_dg *dg, scdg_plan *plan, const double *q, double inv_dt, double *aii,
                                    double *aib, double *abi, double *bb_val);

/* ------------------------------------------------------------------------
 * Newton iterations of one backward-Euler step replayed from captured HIP
 * graphs (the Newton linearization of eq. NewtonLinSys1 solved by static
 * condensation, eq. SC_step1 and SC_step2):
 *
 *     B = -R(Q);  b_S = condense(B);  S x = b_S by GMRES(m);
 *     dQ = backsolve(B, x);  Q += dQ;  R(Q) and ||R(Q)||
 *
 * with R from the scdg_dg object and A, S from the plan: the plan must be
 * condensed (scdg_condense) for a Jacobian supplied by the caller, usually at
 * Q_s, and that Jacobian is kept for every iteration of the step (a chord
 * iteration; with FP32 factors the FP64 nonlinear residual drives the
 * refinement).  An iteration is three graphs: the condensed right-hand side
 * and GMRES set-up; one GMRES restart cycle, replayed until a flag in device
 * memory reports the solve finished (the host reads it after each cycle; at
 * most `cycles` cycles, after which the iteration goes on with the partial
 * solution); and back-substitution, update and residual.  Within a cycle the
 * kernels of the steps after convergence return at once.  The host reads
 * ||R(Q)|| after each iteration and stops when ||R(Q)|| <= newton_tol ||R(Q_s)||.  The GMRES tolerance of an iteration is
 * clip(forcing * newton_tol * ||R(Q_s)|| / ||R(Q)||, lin_tol, eta_max)
 * (inexact Newton; forcing = 0 gives lin_tol).  GMRES starts from zero; a
 * guess enters as the starting state Q.
 *
 * q_s (device, read only) is the state at the previous time level; q (device,
 * in: starting state, e.g. a copy of q_s or q_s plus a predicted increment;
 * out: the new state) must not alias q_s.  Both hold n_dof doubles in the
 * natural DOF order, which must match the dg object's size.  If the starting
 * state has a larger residual than Q_s it is replaced by Q_s
 * (info.start_rejected).  The graphs are captured on the first call and reused
 * while q, q_s, dg, inv_dt, the options, the plan's buffers and the dg
 * object's geometry (any scdg_dg_set_geometry call forces a new capture) stay the same;
 * keep them fixed across steps to avoid a new capture.  The call synchronizes
 * the plan's stream.  Errors: SCDG_ERR_STATE before scdg_condense,
 * SCDG_ERR_ARG for sizes that differ or restart > 63, SCDG_ERR_NONFINITE when
 * a residual norm is not finite, SCDG_ERR_NOCONV when max_newton iterations
 * end above the tolerance (q then holds the last iterate).
 * ------------------------------------------------------------------------ */
typedef struct {
  double newton_tol;   /* relative to ||R(Q_s)||; <= 0 selects 1e-8 */
  double lin_tol;      /* floor of the GMRES tolerance; <= 0 selects 1e-10 */
  double forcing;      /* < 0 selects 0.5; 0 disables the forcing term */
  double eta_max;      /* cap of the GMRES tolerance; <= 0 selects 0.1 */
  int32_t restart;     /* GMRES(m), <= 0 selects 30, at most 63 */
  int32_t cycles;      /* restart cycles per Newton iteration at most, <= 0 selects 8, at most 64 */
  int32_t precond;     /* 0 none, 1 point Jacobi, 2 5x5 node-block Jacobi; < 0 selects 1 */
  int32_t max_newton;  /* <= 0 selects 10 */
} scdg_newton_opts;
typedef struct {
  int32_t newton;          /* Newton iterations (graph replays) */
  int32_t gmres;           /* GMRES iterations, all Newton iterations */
  int32_t first_gmres;     /* GMRES iterations of the first Newton iteration */
  int32_t lin_unconverged; /* iterations whose GMRES ended at the cycle budget above its tolerance */
  int32_t start_rejected;  /* the starting state was replaced by Q_s */
  int32_t converged;       /* ||R(Q)|| <= newton_tol ||R(Q_s)|| on return */
  double r0;               /* ||R(Q_s)|| */
  double rel_res;          /* ||R(Q)|| / ||R(Q_s)|| on return */
} scdg_newton_info;
scdg_status scdg_newton_step(scdg_plan *p, scdg_dg *dg, const double *q_s, double inv_dt, double *q,
                             const scdg_newton_opts *o, scdg_newton_info *info);

/* ------------------------------------------------------------------------
 * Learned initial guess.  A per-element multilayer perceptron maps an
 * element's state and its previous Newton increment to a prediction of the
 * next increment; its boundary part serves as the initial guess x0 of the
 * condensed GMRES solve (scdg_solve; the guess is dropped for the zero vector
 * when ||b_S - S x0|| > ||b_S||, so the solve always converges to the same
 * tolerance as without it).  The paper has no learned component: this is an
 * addition to its Newton-Krylov loop (Section 2.2).
 *
 * Network (FP32 storage, FP32 matrix-core arithmetic):
 *   a_0 = x;  a_l = tanh(W_l^T a_{l-1} + b_l), l = 1..n_layers;
 *   y = W_out^T a_{n_layers} + b_out (linear output).
 * Parameters: one flat device float vector, layer after layer, each W_l
 * [fan_in x fan_out] row-major followed by b_l [fan_out]; the caller owns it
 * and its Adam moments.  Batches are row-major [batch x width].
 * Features for element e of a DG vector (natural DOF order, d = 5 P^3 DOFs
 * per element, n_out = d, n_in = 2 d or 3 d):
 *   x_e = [ (Q_e - mean_v) / std_v , dQprev_e / rp_v ( , R_e / rr_v ) ],
 *   target t_e = (dQ_e - dQprev_e) / rc_v,  prediction dQ_e = dQprev_e + rc_v y_e,
 * with per-variable mean and standard deviation of Q, root mean square rp of
 * dQprev, rc of dQ - dQprev and rr of R over the whole field (stats: 25 device
 * doubles mean[5], std[5], rp[5], rc[5], rr[5]; a zero spread is replaced by
 * 1).  R is the nonlinear residual at the start of the step, R(Q_s) = H(Q_s),
 * the right-hand side the step's increment answers; the third block is used
 * when n_in = 3 d.  The network thus predicts a correction to the previous
 * increment.
 * The object owns the hidden activations of its last forward call (for
 * scdg_mlp_backward), scratch for the backward pass and reduction partials.
 * All calls are asynchronous on the object's stream and bitwise repeatable.
 * ------------------------------------------------------------------------ */
typedef struct scdg_mlp scdg_mlp;
typedef struct {
  int32_t n_in, n_hidden, n_layers, n_out;  /* n_layers hidden layers (0..16; 0: one linear map) */
  int32_t max_batch;                        /* largest batch of any call */
} scdg_mlp_shape;
scdg_status scdg_mlp_create(scdg_mlp **out, const scdg_mlp_shape *s, void *hip_stream);
scdg_status scdg_mlp_destroy(scdg_mlp *m);
/* number of floats of the flat parameter vector (and of its gradient) */
scdg_status scdg_mlp_param_count(const scdg_mlp *m, int64_t *n);
/* Arithmetic of the matrix products of forward and backward:
 * SCDG_MLP_FP32 (default) multiplies FP32 operands; SCDG_MLP_BF16 rounds both
 * operands of every product (weights, activations, gradients) to the nearest
 * bfloat16, ties to even, and multiplies them on the bf16 matrix cores; both
 * accumulate in FP32, and parameters, biases, activations, gradients and Adam
 * stay FP32.  SCDG_ERR_ARG for another mode. */
enum { SCDG_MLP_FP32 = 0, SCDG_MLP_BF16 = 1 };
scdg_status scdg_mlp_set_compute(scdg_mlp *m, int32_t mode);
/* y [batch x n_out] = network(x [batch x n_in]); keeps the activations */
scdg_status scdg_mlp_forward(scdg_mlp *m, const float *w, const float *x, int32_t batch, float *y);
/* Gradients of a loss with respect to the parameters (dw, overwritten) and,
 * if dx != NULL, to the input, given dy = dLoss/dy for the batch of the last
 * scdg_mlp_forward call (same x and batch; SCDG_ERR_STATE otherwise). */
scdg_status scdg_mlp_backward(scdg_mlp *m, const float *w, const float *x, const float *dy, int32_t batch,
                              float *dw, float *dx);
/* One Adam step (Kingma and Ba): m1 = b1 m1 + (1-b1) g, m2 = b2 m2 + (1-b2) g^2,
 * w -= lr (m1 / (1 - b1^step)) / (sqrt(m2 / (1 - b2^step)) + eps); step >= 1. */
scdg_status scdg_mlp_adam(scdg_mlp *m, float *w, const float *dw, float *m1, float *m2, float lr, float beta1,
                          float beta2, float eps, int32_t step);
/* Mean squared error over n values: *loss (device double) = mean((y - t)^2);
 * dy (may be NULL) = 2 (y - t) / n. */
scdg_status scdg_mlp_mse(scdg_mlp *m, const float *y, const float *t, int64_t n, float *dy, double *loss);
/* dst[r] = src[idx[r]] for rows of width floats (idx: device int32, count rows) */
scdg_status scdg_mlp_gather(scdg_mlp *m, const float *src, int32_t width, const int32_t *idx, int32_t count,
                            float *dst);
/* Field statistics of the features (n_dof = 5 * nodes, natural order; stats:
 * 25 device doubles); dq (the increment that followed dq_prev) may be NULL,
 * then rc = rp; r (the residual R(Q_s)) may be NULL, then rr = 1. */
scdg_status scdg_guess_stats(scdg_mlp *m, const double *q, const double *dq_prev, const double *dq,
                             const double *r, int64_t n_dof, double *stats);
/* x [n_elem x n_in] from Q, dQprev and, when n_in == 3 n_out, R (r may be NULL
 * when n_in == 2 n_out; n_out % 5 == 0; SCDG_ERR_ARG otherwise) */
scdg_status scdg_guess_features(scdg_mlp *m, const double *q, const double *dq_prev, const double *r,
                                const double *stats, int32_t n_elem, float *x);
/* t [n_elem x n_out] = (dQ - dQprev) / rc */
scdg_status scdg_guess_target(scdg_mlp *m, const double *dq, const double *dq_prev, const double *stats,
                              int32_t n_elem, float *t);
/* dQ = dQprev + rc * y (natural order, n_elem * n_out doubles) */
scdg_status scdg_guess_apply(scdg_mlp *m, const double *dq_prev, const float *y, const double *stats,
                             int32_t n_elem, double *dq);

/* ---- Measured ceilings (measurement utilities, no part of the solve) ----
 * The rooflines of the contraction and streaming kernels are quoted against
 * the vendor peaks; these probes measure what a kernel reaches on the part at
 * hand, for context beside them.  Both run on hip_stream (NULL: the null
 * stream), allocate and free their own device buffers, and synchronize.
 *
 * scdg_probe_mfma: back-to-back 16x16x4 MFMAs on register operands (FP64 when
 * precision == 0, FP32 when 1), 8 workgroups of 4 waves per compute unit, four
 * independent accumulators per wave, `iters` rounds (1..2^20) per wave; writes
 * the dense TFLOP/s (2*16*16*4 flops per MFMA), best of three launches.
 * scdg_probe_hbm_read: fills a buffer of `bytes` (64 MiB..16 GiB, a multiple
 * of 16) and reads it with 16-byte nontemporal loads; writes the read GB/s
 * (1e9 bytes/s), best of five launches.
 * SCDG_ERR_ARG for arguments outside those ranges or a NULL output,
 * SCDG_ERR_NOMEM when the buffers cannot be allocated, SCDG_ERR_HIP on a
 * runtime error. */
scdg_status scdg_probe_mfma(int32_t precision, int32_t iters, void *hip_stream, double *tflops);
scdg_status scdg_probe_hbm_read(int64_t bytes, void *hip_stream, double *gbs);

const char *scdg_status_string(scdg_status s);
/* Last error text of a plan (or of plan creation when p is NULL). */
scdg_status scdg_last_error(const scdg_plan *p, char *buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* SCDG_H */
