// Internal declarations of the scdg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/scdg.h"

namespace scdg {

constexpr int kNvar = 5;
constexpr int kMaxOrder = 7;
constexpr int kGjOuter = 128;        // outer panel width of the blocked Gauss-Jordan inverse
constexpr int kGjAutoBlocked = 320;  // automatic choice: blocked form above this n_i

// One GEMM problem of a batched launch: C = alpha A B + beta C, row-major with
// leading dimensions; offsets are element offsets into the three base arrays.
struct GemmDesc {
  int64_t a_off, b_off, c_off;
  int32_t m, n, k, lda, ldb, ldc;
  // fold map of this problem's C (m/5 x n/5 node blocks: index into the folded
  // blocks' values, -1 for none), added in the epilogue; -1: no fold
  int64_t f_off = -1;
};

// One tile of a batched GEMV: rows [row0, row0 + rows) of problem `prob`.
struct RowTile {
  int32_t prob, row0;
};

// One matrix-vector product y = M x for element e in a batched GEMV.
struct GemvDesc {
  int64_t m_off;   // offset of the row-major matrix
  int32_t rows, cols;
  int32_t x_off;   // offset into the x index map (or into x when no map)
  int32_t y_off;   // offset into the y / y0 index space
};

// What a captured GMRES cycle depends on; a different key means recapture.
// Everything a captured Newton iteration depends on: scalars baked into kernel
// arguments and every device pointer its kernels read or write.
struct NewtonKey {
  int m = 0, cycles = 0, pmode = -1, smode = 0;
  uint64_t sp_gen = 0, dg_gen = 0;
  bool fp32 = false;
  double inv_dt = 0, eta_c = 0, lin_tol = 0, eta_max = 0;
  const void *q = nullptr, *q_s = nullptr, *dg = nullptr;
  const void *dg_g = nullptr, *dg_met = nullptr, *dg_params = nullptr;
  const void *ptr[23] = {};
  bool operator==(const NewtonKey &o) const {
    if (m != o.m || cycles != o.cycles || pmode != o.pmode || smode != o.smode || sp_gen != o.sp_gen ||
        dg_gen != o.dg_gen || dg_g != o.dg_g || dg_met != o.dg_met || dg_params != o.dg_params ||
        fp32 != o.fp32 ||
        inv_dt != o.inv_dt ||
        eta_c != o.eta_c || lin_tol != o.lin_tol || eta_max != o.eta_max || q != o.q || q_s != o.q_s ||
        dg != o.dg)
      return false;
    for (int i = 0; i < 23; ++i)
      if (ptr[i] != o.ptr[i]) return false;
    return true;
  }
};

struct KrylovKey {
  int m = 0, pmode = -1, smode = 0;
  uint64_t sp_gen = 0;
  bool fp32 = false;
  const void *sloc = nullptr, *bb_val = nullptr, *gm_v = nullptr;
  // the matrix-free forms' operands: block-sparse lists, work vector, and the
  // caller's A_ib / A_bi (their addresses can change with every assemble)
  const void *sp[7] = {};
  bool operator==(const KrylovKey &o) const {
    for (int i = 0; i < 7; ++i)
      if (sp[i] != o.sp[i]) return false;
    return m == o.m && pmode == o.pmode && smode == o.smode && sp_gen == o.sp_gen && fp32 == o.fp32 &&
           sloc == o.sloc &&
           bb_val == o.bb_val && gm_v == o.gm_v;
  }
};

// A block-sparse element operator (rows of 5x5 blocks): the nonzero blocks of
// A_ib (block rows = interior nodes, x = boundary vector) or of A_bi (block
// rows = coupling-set nodes, x = interior vector), found from the values.
struct SparseOp {
  int64_t n_rows = 0, n_blocks = 0;
  int64_t *d_rowptr = nullptr;   // [n_rows + 1]
  int32_t *d_xnode = nullptr;    // [n_blocks] node of x the block multiplies (x index 5 xnode + w)
  int64_t *d_ybase = nullptr;    // [n_rows] first y index of the block row
  int64_t *d_src = nullptr;      // [n_blocks] offset of the block's entry (0, 0) in the dense blocks
  int32_t *d_ld = nullptr;       // [n_blocks] row length of the dense element matrix
  void *val = nullptr;           // [n_blocks * 25] compacted values in the factor precision
  size_t cap_val = 0;
  uint8_t *d_mask_ref = nullptr; // block mask the lists were built from
};

// GEMM tile configurations (rows x columns of C per workgroup)
enum { kGemm64x64 = 0, kGemm64x128 = 1, kGemm128x128 = 2, kGemm128x128w8 = 3, kGemmConfigs = 9 };

template <typename T>
struct DevBuf {
  T *ptr = nullptr;
  size_t count = 0;
};

struct Plan {
  hipStream_t stream = nullptr;
  int device = 0;
  uint64_t uid = 0;   // distinct for every plan the process creates (never reused)
  std::string last_error;
  int state = 0;  // 0 created, 1 assembled, 2 factored, 3 condensed
  // Schur products: 0 through the element blocks T_e and the A_bb remainder
  // (S assembled), 1 matrix-free through X_e, A_bi and the full A_bb
  int schur_mode = 0;
  double *mf_dblk = nullptr;  // [sum |C_e| * 25] diagonal 5x5 blocks of A_bi(e) X_e per slot (modes 1, 2)
  // mode 2: products through the nonzero blocks of A_ib and A_bi and A_ii^-1
  SparseOp sp_ib, sp_bi;
  uint64_t sp_gen = 0;              // count of block-list rebuilds (part of the graph keys)
  // FP32 copies of A_bb (matrix-free forms) and of its remainder (assembled form)
  // used inside the Schur products when the factors are FP32
  float *bb_lo = nullptr, *rem_lo = nullptr;
  uint8_t *d_mask = nullptr;        // [sum (n_i / 5)(n_c / 5)] block mask (one matrix at a time)
  int32_t *d_mask_flag = nullptr;   // [1] masks differ
  int64_t *d_e_offib = nullptr, *d_e_maskoff = nullptr;  // [n_elem] A_ib / A_bi offset, mask offset
  int32_t *d_e_ri = nullptr, *d_e_rc = nullptr;          // [n_elem] n_i / 5, n_c / 5
  double *w_z2 = nullptr;           // [n2]
  scdg_precision prec = SCDG_FP64;

  // structure
  int32_t n_elem = 0;
  std::vector<int32_t> order;
  int64_t n_dof = 0, n1 = 0, n2 = 0, n_bnodes = 0, nnzb = 0;
  std::vector<int32_t> ni, nc;          // DOF counts per element
  std::vector<int64_t> h_c_ptr;         // host copy of the coupling sets
  std::vector<int32_t> h_c_node;
  std::vector<int64_t> off_q, off_ii, off_ib, off_cc, off_i, off_c, bnode_off;
  int32_t max_ni = 0, max_nc = 0;

  // device index maps
  int32_t *d_imap = nullptr;      // [n2] natural DOF of each interior slot
  int32_t *d_bmap = nullptr;      // [n1] natural DOF of each boundary slot
  int32_t *d_cmap = nullptr;      // [sum n_c] boundary-vector index of each C slot
  int32_t *d_pull_ptr = nullptr;  // [n_bnodes+1] C-slot lists per boundary node
  int32_t *d_pull_idx = nullptr;  // C node-slot indices (sum |C_e| entries)
  int64_t *d_slot_soff = nullptr; // [sum |C_e|] S_loc offset of the slot's element
  int32_t *d_slot_nc = nullptr;   // [sum |C_e|] n_c of the slot's element
  int32_t *d_slot_pos = nullptr;  // [sum |C_e|] position of the slot within C_e
  int64_t *d_slot_ib = nullptr;   // [sum |C_e|] A_bi / X offset of the slot's element
  int32_t *d_slot_ni = nullptr;   // [sum |C_e|] n_i of the slot's element
  int64_t *d_bb_rowptr = nullptr; // [n_bnodes+1]
  int32_t *d_bb_col = nullptr;    // [nnzb]
  // A_bb blocks folded into the element Schur blocks T_e, and the remainder
  int64_t n_fold = 0, n_rem = 0;
  // [sum |C_e|^2] per element, the A_bb block folded into each node block of
  // T_e (index into bb_val) or -1; the Schur GEMM adds them in its epilogue
  int32_t *d_fold_map = nullptr;
  int64_t *d_rem_rowptr = nullptr;  // [n_bnodes+1]
  int32_t *d_rem_col = nullptr;     // [n_rem]
  int32_t *d_rem_src = nullptr;     // [n_rem] block index into bb_val
  // the remainder transposed (rows = its columns), for S^T x: source index into rem_val
  int64_t *d_remt_rowptr = nullptr; // [n_bnodes+1]
  int32_t *d_remt_col = nullptr;    // [n_rem]
  int32_t *d_remt_src = nullptr;    // [n_rem] remainder-order index of the block (read transposed)
  RowTile *d_ct_s = nullptr;        // 256-column tiles of the element Schur blocks (S^T x)
  int32_t n_ct_s = 0;
  int32_t *d_inv_n = nullptr;     // [n_elem] n_i per element
  int64_t *d_inv_off = nullptr;   // [n_elem] offset of A_ii(e)
  int32_t *d_inv_order = nullptr; // [n_elem] elements by decreasing n_i (stable)
  int32_t *d_info = nullptr;      // [n_elem] factor info
  int32_t *d_jac_cnode = nullptr; // [sum |C_e|] device copy of the coupling sets (device Jacobian blocks)

  // batched GEMM descriptors and tile lists (X = Ainv A_ib, S_loc = A_bi X)
  GemmDesc *d_gx = nullptr, *d_gs = nullptr;
  int32_t *d_tiles_x = nullptr, *d_tiles_s = nullptr;
  int32_t n_tiles_x = 0, n_tiles_s = 0;
  int gemm_cfg_x = kGemm64x128, gemm_cfg_s = kGemm128x128;
  std::vector<GemmDesc> gx_host, gs_host;   // kept to rebuild tile lists

  // batched GEMV descriptors
  GemvDesc *d_gv_inv = nullptr;  // Ainv (n_i x n_i), x: interior slots
  GemvDesc *d_gv_abi = nullptr;  // A_bi (n_c x n_i)
  GemvDesc *d_gv_aib = nullptr;  // A_ib / X (n_i x n_c)
  GemvDesc *d_gv_s = nullptr;    // S_loc (n_c x n_c)
  RowTile *d_rt_inv = nullptr, *d_rt_abi = nullptr, *d_rt_aib = nullptr, *d_rt_s = nullptr;
  int32_t n_rt_inv = 0, n_rt_abi = 0, n_rt_aib = 0, n_rt_s = 0;

  // FP64 blocks: the caller's (SCDG_BORROW) or the plan's copies (SCDG_COPY)
  const double *aii = nullptr, *aib = nullptr, *abi = nullptr, *bb_val = nullptr;
  double *own_aii = nullptr, *own_aib = nullptr, *own_abi = nullptr, *own_bb = nullptr;

  // factors and Schur blocks (precision = prec)
  void *ainv = nullptr;   // sum n_i^2
  void *ainv_work = nullptr;  // sum n_i^2 (Gauss-Jordan work space)
  void *xmat = nullptr;   // sum n_i n_c
  void *sloc = nullptr;   // sum n_c^2
  void *aib_lo = nullptr, *abi_lo = nullptr;  // FP32 shadows (FP32 mode)
  double *diag_s = nullptr;  // [n1] 1 / diag(S) (point Jacobi)
  double *pc_blk = nullptr;  // [n_bnodes * 25] inverse 5x5 diagonal blocks of S
  double *rem_val = nullptr; // [n_rem * 25] A_bb remainder blocks in remainder order
  size_t cap_ainv = 0, cap_x = 0, cap_s = 0;  // bytes allocated

  // blocked Gauss-Jordan inverse (outer panels of kGjOuter columns)
  int inverse_mode = 0;            // 0 automatic, 1 one kernel per element, 2 blocked, 3 resident panel
  int inverse_used = 0;            // form used by the last scdg_factor (1, 2 or 3)
  int64_t sum_ni = 0;
  int64_t *d_gj_voff = nullptr;    // [n_elem] exclusive prefix of n_i
  int32_t *d_gj_piv = nullptr;     // [sum n_i] pivot row of each column
  unsigned char *d_gj_flag = nullptr;  // [sum n_i] row already used as a pivot
  void *gj_pbuf = nullptr, *gj_rbuf = nullptr;  // [sum n_i * kGjOuter] each
  size_t cap_gj = 0;
  GemmDesc *d_gj_desc = nullptr;   // per outer panel, the update GEMMs W += P R
  int32_t *d_gj_tiles = nullptr;
  std::vector<int64_t> gj_desc_off, gj_tile_off;
  std::vector<int32_t> gj_ntiles;
  int gj_cfg = -1;                 // tile configuration the lists were built for

  // dense S path
  double *s_dense = nullptr;
  int32_t *s_piv = nullptr;
  int32_t *d_dense_info = nullptr;
  bool dense_factored = false;

  // work vectors (doubles)
  double *w_z = nullptr;      // [n2]
  double *w_t = nullptr;      // [sum n_c]
  double *w_bs = nullptr;     // [n1]
  double *w_qb = nullptr;     // [n1]
  double *w_r = nullptr;      // [n_dof]
  double *w_rx = nullptr;     // [n1] A_bb remainder product of the assembled Schur product
  double *w_dq = nullptr;     // [n_dof]
  double *w_vec = nullptr;    // [n_dof] scratch
  double *gm_v = nullptr;     // [(m+1) * n1] Krylov basis
  double *gm_w = nullptr;     // [n1]
  double *gm_z = nullptr;     // [n1]
  double *gm_part = nullptr;  // reduction partials
  double *gm_h = nullptr;     // [m+2] device h column
  double *h_pinned = nullptr; // host pinned staging
  int32_t gm_m = 0;

  // device-resident GMRES cycles (krylov_mode 1) and their graph (mode 2)
  int krylov_mode = 0;            // 0 host Givens, 1 device, 2 device + graph replay
  const int32_t *halt = nullptr;  // set while enqueueing Arnoldi steps: kernels return when *halt
  bool capturing = false;
  double *kr_H = nullptr, *kr_cs = nullptr, *kr_sn = nullptr, *kr_g = nullptr, *kr_dev = nullptr;
  int32_t *kr_st = nullptr;
  int kr_m = 0;
  hipStream_t cap_stream = nullptr;   // plan-owned stream for graph capture
  hipGraph_t kr_graph = nullptr;
  hipGraphExec_t kr_exec = nullptr;
  KrylovKey kr_key{};

  // one Newton iteration of a backward-Euler step as a graph (scdg_newton_step)
  double *nw_r = nullptr;      // [n_dof] nonlinear residual R(Q)
  double *nw_dq = nullptr;     // [n_dof] minus the Newton increment
  double *nw_stat = nullptr;   // [8] norms, see newton_gmres_setup_kernel
  hipGraph_t nw_graph[3] = {};        // 0: right-hand side and GMRES set-up, 1: one restart
  hipGraphExec_t nw_exec[3] = {};     //    cycle, 2: back-substitution, update and residual
  NewtonKey nw_key{};
  int32_t red_blocks = 0;

  // phase timing (events recorded asynchronously, summed on query)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
};

// ---- kernel launchers (implemented in the .hip files) ----
hipError_t launch_gj_inverse(Plan &p, void *work, void *out, bool fp32);
hipError_t launch_gj_inverse_blocked(Plan &p, void *work, void *out, bool fp32);
bool gj_supported(int max_n, bool fp32);
hipError_t launch_gj_inverse_resident(Plan &p, void *work, void *out, bool fp32);
bool gj_resident_supported(int max_n, bool fp32);
hipError_t launch_cast_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, size_t n, hipStream_t s);
void gemm_tile_shape(int cfg, int *bm, int *bn);
// C = alpha A B + beta C per problem, plus the folded A_bb blocks of
// fold_val (FP64) where fold_map (and the problem's f_off) names them
hipError_t launch_gemm_batched(int cfg, const GemmDesc *d_desc, const int32_t *d_tiles,
                               int32_t n_tiles, const void *a, const void *b, void *c, double alpha,
                               double beta, bool fp32, hipStream_t s, const int32_t *fold_map = nullptr,
                               const double *fold_val = nullptr);

// y[omap?omap[y_off+r]:y_off+r] = alpha * sum_c M[r,c] x[xmap?xmap[x_off+c]:x_off+c]
//                                 + beta * y0[y_off + r]
hipError_t launch_gemv_batched(const GemvDesc *d_desc, const RowTile *d_tiles, int32_t n_tiles,
                               int32_t max_cols, const void *mat, bool fp32, const double *x,
                               const int32_t *xmap, double *y, const int32_t *omap, double alpha,
                               double beta, const double *y0, hipStream_t s,
                               const int32_t *halt = nullptr);

// out[j] = c0 * src0[map0 ? map0[j] : j] + c1 * (B x)[j] + c2 * sum_{s in pull(j/5)} t[5 s + j%5]
// with B = A_bb (full = true) or the remainder of A_bb not folded into T_e.
// Assembled Schur product, first launch: t = T_e x[C_e] per slot and rx = R x.
hipError_t launch_schur_apply_t(const Plan &p, const double *x, double *z, double *y, bool lo);
hipError_t launch_schur_gemv_rem(const Plan &p, const double *x, double *t, double *rx, bool lo);
hipError_t launch_bsr_pull(const Plan &p, bool full, double c0, const double *src0,
                           const int32_t *map0, double c1, const double *x, double c2,
                           const double *t, double *out, bool lo = false);
// T[dst + v nc + w] += A_bb[src][v][w] for the folded blocks
// 5x5 diagonal blocks of S (remainder + element blocks), inverted; point inverse too
// Matrix-free mode: diagonal 5x5 blocks of A_bi(e) X_e per slot, and the
// Jacobi preconditioners from diag(A_bb) minus their pulled sums.
hipError_t launch_mf_diag_blocks(const Plan &p, const void *abi, bool fp32);
hipError_t launch_precond_setup_mf(const Plan &p);
// Block-sparse element products (Schur form 2)
hipError_t launch_block_mask(const double *mat, const int64_t *m_off, const int32_t *rb_n, const int32_t *cb_n,
                             const int64_t *mask_off, uint8_t *mask, int n_elem, hipStream_t s);
hipError_t launch_gather_blocks_ld(const void *src, const int64_t *src_off, const int32_t *ld, int64_t n, void *dst,
                                   bool fp32, hipStream_t s);
hipError_t launch_mask_diff(const uint8_t *a, const uint8_t *b, int64_t n, int32_t *flag, hipStream_t s);
hipError_t launch_bsr5_rows(int64_t n_rows, const int64_t *rowptr, const int32_t *xnode, const void *val,
                            bool fp32, const double *x, const int64_t *ybase, double *y, hipStream_t s,
                            const int32_t *halt);
hipError_t launch_precond_setup(const Plan &p, const void *t, bool fp32);
// y = a M^-1 x with M = I (mode 0), diag(S) (1) or the 5x5 node blocks of S (2)
hipError_t launch_precond_apply(const Plan &p, int mode, const double *x, double *y, double a);

hipError_t launch_gather(const double *src, const int32_t *map, double *dst, int64_t n, hipStream_t s);
// dst[b * 25 + k] = src[idx[b] * 25 + k]  (5x5 blocks)
hipError_t launch_gather_blocks(const double *src, const int32_t *idx, double *dst, int64_t nblocks,
                                hipStream_t s);
hipError_t launch_scatter(const double *src, const int32_t *map, double *dst, int64_t n, hipStream_t s);
hipError_t launch_guess_err_gather(const float *y, const float *t, const double *stats, const int32_t *map,
                                   int64_t n, double *e, hipStream_t s);
hipError_t launch_guess_grad_scatter(const double *g, const double *stats, const int32_t *map, int64_t n,
                                     int64_t n_dof, double a, float *dy, hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s,
                        const int32_t *halt = nullptr);
hipError_t launch_fill(double *y, int64_t n, double v, hipStream_t s, const int32_t *halt = nullptr);
hipError_t launch_scatter_axpby(int64_t n, double a, const double *x, double b, const double *yin,
                                const int32_t *map, double *dst, hipStream_t s);

// multi-dot: out[k] = sum_i V[k*ld + i] w[i], k < nv (deterministic two-stage)
hipError_t launch_multidot(const double *v, int64_t ld, int32_t nv, const double *w, int64_t n,
                           double *partials, int32_t nblocks, double *out, hipStream_t s,
                           const int32_t *halt = nullptr);
// w -= sum_k V[k*ld+i] h[k]
hipError_t launch_multi_axpy(const double *v, int64_t ld, int32_t nv, const double *h, double *w,
                             int64_t n, hipStream_t s,
                             const int32_t *nv_dev = nullptr, const int32_t *halt = nullptr);
// y = x * dinv (elementwise); dinv may be null (copy)
hipError_t launch_diag_scale(const double *x, const double *dinv, double *y, int64_t n, double a,
                             hipStream_t s,
                             const double *a_dev = nullptr, const int32_t *halt = nullptr);
hipError_t launch_reciprocal(double *x, int64_t n, hipStream_t s);
hipError_t launch_krylov_start(double beta, double target, int limit, double *g, int32_t *st, double *dev,
                               hipStream_t s);
hipError_t launch_krylov_givens(int j, int m, const double *hc, double *H, double *cs, double *sn, double *g,
                                int32_t *st, double *dev, hipStream_t s);
hipError_t launch_krylov_solve(int m, const double *H, const double *g, const int32_t *st, double *yneg,
                               hipStream_t s, const int32_t *halt = nullptr);
hipError_t launch_newton_gmres_setup(const double *stat, double eta_c, double lin_tol, double eta_max, int m,
                                     double *g, int32_t *st, double *dev, hipStream_t s);
hipError_t launch_newton_gmres_restart(const double *stat, int m, double *g, int32_t *st, double *dev,
                                       hipStream_t s);

// device residual R(Q) of a scdg_dg object (k_dgsem.hip), enqueued on stream s
hipError_t dg_residual_on(scdg_dg *dg, const double *q, const double *q_s, double inv_dt, double *r,
                          hipStream_t s);
int64_t dg_dof_count(const scdg_dg *dg);
void dg_graph_state(const scdg_dg *dg, uint64_t *gen, const void **g, const void **met, const void **params);
// device Jacobian blocks (k_dgsem.hip): the plan's structure as the assembly sees it
struct JacPlanView {
  uint64_t plan_uid;             // the plan's uid: its coupling sets and A_bb pattern never change
  int ni, nc, ncn, nb;           // n_i, n_c (DOFs), |C_e| (nodes), boundary nodes per element
  int64_t nnzb;
  const int32_t *c_node;         // [n_elem * ncn] device copy of the coupling sets
  const int64_t *bb_rowptr;
  const int32_t *bb_col;
};
bool dg_jacobian_shape(const scdg_dg *dg, int *k_elem, int *order, bool *cartesian_br1);
std::string dg_last_error(const scdg_dg *dg);
scdg_status dg_jacobian_blocks_on(scdg_dg *dg, const JacPlanView &v, const double *q, double inv_dt, double *aii,
                                  double *aib, double *abi, double *bb_val);

// dense path
hipError_t launch_dense_assemble(const Plan &p, double *s_dense);
hipError_t launch_dense_lu(Plan &p, double *a, int32_t n, int32_t *piv, int32_t *info);
hipError_t launch_dense_solve(const double *lu, int32_t n, const int32_t *piv, double *x,
                              hipStream_t s);

}  // namespace scdg
