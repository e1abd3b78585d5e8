// C ABI of the scdg library: plan construction (index maps of the interior /
// boundary partition), state machine, and the orchestration of the kernels
// for factor / condense / condensed RHS / condensed solve / back-substitution
// / full residual and iterative refinement.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace scdg;

struct scdg_plan {
  Plan p;
};

namespace {

std::string g_create_error;

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      p.last_error = std::string(#expr) + ": " + hipGetErrorString(e_);           \
      return SCDG_ERR_HIP;                                                         \
    }                                                                              \
  } while (0)

#define ST_TRY(expr)                   \
  do {                                 \
    scdg_status s_ = (expr);           \
    if (s_ != SCDG_OK) return s_;      \
  } while (0)

template <typename T>
scdg_status dalloc(Plan &p, T **ptr, size_t count) {
  if (*ptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(ptr), sizeof(T) * count);
  if (e != hipSuccess) {
    *ptr = nullptr;
    p.last_error = std::string("hipMalloc of ") + std::to_string(sizeof(T) * count) +
                   " bytes: " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SCDG_ERR_NOMEM : SCDG_ERR_HIP;
  }
  return SCDG_OK;
}

// work may be enqueued only with the plan's device current
scdg_status on_device(Plan &p) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p.device) {
    p.last_error = "call with the plan's HIP device (" + std::to_string(p.device) + ") current";
    return SCDG_ERR_STATE;
  }
  return SCDG_OK;
}

template <typename T>
scdg_status upload(Plan &p, T **ptr, const std::vector<T> &host) {
  ST_TRY(dalloc(p, ptr, host.size()));
  if (!host.empty()) HIP_TRY(hipMemcpy(*ptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
  return SCDG_OK;
}

template <typename T>
void dfree(T *&ptr) {
  if (ptr) (void)hipFree(const_cast<void *>(reinterpret_cast<const void *>(ptr)));
  ptr = nullptr;
}

// Interior / boundary nodes of an element of the given order.  A node is interior
// when, in every direction, its index is strictly inside or sits on a face that
// `phys` marks physical (bit 2 d for index 0, bit 2 d + 1 for index N).
void local_node_sets(int order, int phys, std::vector<int> &interior, std::vector<int> &boundary) {
  const int p = order + 1;
  interior.clear();
  boundary.clear();
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i) {
        const int n = i + p * j + p * p * k;
        const int idx[3] = {i, j, k};
        bool in = true;
        for (int d = 0; d < 3; ++d) {
          if (idx[d] == 0 && !((phys >> (2 * d)) & 1)) in = false;
          if (idx[d] == order && !((phys >> (2 * d + 1)) & 1)) in = false;
        }
        (in ? interior : boundary).push_back(n);
      }
}

// Tile list ordered so that the workgroups of one problem share an XCD: block b
// runs on XCD b % 8, so block b takes tile (b % 8) * per + b / 8 of the
// problem-major list.
// Tile list of a batched GEMM for the 8 XCDs (a workgroup runs on XCD
// blockIdx % 8 and XCDs take their workgroups in blockIdx order): every
// problem's tiles stay on one XCD (its operands stay in that XCD's L2), problems
// go to XCDs by longest-processing-time-first (largest remaining cost to the
// least-loaded XCD; cost = tiles x K), and each XCD runs its largest problems
// first.  Slots past the end of a shorter XCD list hold -1 (no work).
std::vector<int32_t> xcd_tile_list(const std::vector<GemmDesc> &descs, int cfg) {
  int bm, bn;
  gemm_tile_shape(cfg, &bm, &bn);
  const size_t nq = descs.size();
  std::vector<double> cost(nq);
  std::vector<size_t> order(nq);
  for (size_t q = 0; q < nq; ++q) {
    const double tm = (descs[q].m + bm - 1) / bm, tn = (descs[q].n + bn - 1) / bn;
    cost[q] = tm * tn * std::max(1, descs[q].k);
    order[q] = q;
  }
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int32_t>> lists(8);
  std::vector<double> load(8, 0.0);
  for (size_t q : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    const int tm = (descs[q].m + bm - 1) / bm, tn = (descs[q].n + bn - 1) / bn;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        lists[x].push_back((int32_t)q);
        lists[x].push_back(a);
        lists[x].push_back(b);
      }
    load[x] += cost[q];
  }
  size_t longest = 0;
  for (auto &l : lists) longest = std::max(longest, l.size() / 3);
  std::vector<int32_t> out(3 * 8 * longest, -1);
  for (size_t pos = 0; pos < longest; ++pos)
    for (int x = 0; x < 8; ++x)
      if (pos < lists[x].size() / 3) std::memcpy(&out[3 * (pos * 8 + x)], &lists[x][3 * pos], 3 * sizeof(int32_t));
  return out;
}

std::vector<RowTile> row_tiles(const std::vector<GemvDesc> &descs) {
  std::vector<RowTile> t;
  for (size_t q = 0; q < descs.size(); ++q)
    for (int r = 0; r < descs[q].rows; r += 64) t.push_back(RowTile{(int32_t)q, r});
  return t;
}

// Event pair around a stretch of stream work when timing is on.
struct PhaseTimer {
  Plan &p;
  int phase;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  PhaseTimer(Plan &pl, int ph) : p(pl), phase(ph) {
    if (!p.timing || p.capturing) return;
    if (p.ev_pool.empty()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      p.ev_pool.emplace_back(a, b);
    }
    ev = p.ev_pool.back();
    p.ev_pool.pop_back();
    (void)hipEventRecord(ev.first, p.stream);
  }
  ~PhaseTimer() {
    if (!ev.first) return;
    (void)hipEventRecord(ev.second, p.stream);
    p.ev_used.emplace_back(phase, ev);
  }
};

bool fp32(const Plan &p) { return p.prec == SCDG_FP32; }
size_t esize(const Plan &p) { return fp32(p) ? sizeof(float) : sizeof(double); }

scdg_status sync(Plan &p) {
  HIP_TRY(hipStreamSynchronize(p.stream));
  return SCDG_OK;
}

// ||x||_2^2 of a device vector, result on host (synchronizes)
scdg_status norm2sq(Plan &p, const double *x, int64_t n, double *out) {
  HIP_TRY(launch_multidot(x, 0, 1, x, n, p.gm_part, p.red_blocks, p.gm_h, p.stream));
  HIP_TRY(hipMemcpyAsync(p.h_pinned, p.gm_h, sizeof(double), hipMemcpyDeviceToHost, p.stream));
  ST_TRY(sync(p));
  *out = p.h_pinned[0];
  return SCDG_OK;
}

// ---- stage helpers (all enqueue on p.stream) ----

// z = A_ii^-1 B_i for every element (B natural)
scdg_status apply_inverse(Plan &p, const double *b_nat, double *z) {
  HIP_TRY(launch_gemv_batched(p.d_gv_inv, p.d_rt_inv, p.n_rt_inv, p.max_ni, p.ainv, fp32(p), b_nat,
                              p.d_imap, z, nullptr, 1.0, 0.0, nullptr, p.stream));
  return SCDG_OK;
}

scdg_status condense_rhs_impl(Plan &p, const double *b, double *bs) {
  PhaseTimer tm(p, SCDG_PHASE_RHS);
  ST_TRY(apply_inverse(p, b, p.w_z));
  const void *abi = fp32(p) ? p.abi_lo : static_cast<const void *>(p.abi);
  HIP_TRY(launch_gemv_batched(p.d_gv_abi, p.d_rt_abi, p.n_rt_abi, p.max_ni, abi, fp32(p), p.w_z,
                              nullptr, p.w_t, nullptr, 1.0, 0.0, nullptr, p.stream));
  HIP_TRY(launch_bsr_pull(p, false, 1.0, b, p.d_bmap, 0.0, nullptr, -1.0, p.w_t, bs));
  return SCDG_OK;
}

void drop_krylov_graph(Plan &p);
void drop_newton_graph(Plan &p);

// Block-sparse copy of A_ib (which == 0) or A_bi (which == 1) for the sparse
// matrix-free form.  The block mask comes from the FP64 values on the device;
// the block lists are rebuilt on the host only when the mask changed (new
// lists mean new device arrays, which the graph keys see); the values are
// compacted in the factor precision at every condense.
scdg_status sparse_op_update(Plan &p, int which, const void *vals) {
  SparseOp &op = which == 0 ? p.sp_ib : p.sp_bi;
  const int E = p.n_elem;
  int64_t mask_n = 0;
  for (int e = 0; e < E; ++e) mask_n += (int64_t)(p.ni[e] / kNvar) * (p.nc[e] / kNvar);
  if (!p.d_mask) ST_TRY(dalloc(p, &p.d_mask, (size_t)std::max<int64_t>(mask_n, 1)));
  // A_ib(e) is n_i x n_c (block rows n_i / 5); A_bi(e) is n_c x n_i
  HIP_TRY(launch_block_mask(which == 0 ? p.aib : p.abi, p.d_e_offib, which == 0 ? p.d_e_ri : p.d_e_rc,
                            which == 0 ? p.d_e_rc : p.d_e_ri, p.d_e_maskoff, p.d_mask, E, p.stream));
  bool rebuild = op.d_mask_ref == nullptr;
  if (!rebuild) {
    // compare with the mask the lists were built from on the device: only a flag comes back
    if (!p.d_mask_flag) ST_TRY(dalloc(p, &p.d_mask_flag, 1));
    HIP_TRY(hipMemsetAsync(p.d_mask_flag, 0, sizeof(int32_t), p.stream));
    HIP_TRY(launch_mask_diff(p.d_mask, op.d_mask_ref, mask_n, p.d_mask_flag, p.stream));
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, p.d_mask_flag, sizeof(int32_t), hipMemcpyDeviceToHost, p.stream));
    HIP_TRY(hipStreamSynchronize(p.stream));
    rebuild = flag != 0;
  }
  if (rebuild) {
    // the captured GMRES cycle and Newton pieces hold the old list pointers as
    // kernel arguments: drop them (the next use recaptures), and count the
    // rebuild in the graph keys, since a new list may reuse a freed address
    HIP_TRY(hipStreamSynchronize(p.stream));
    drop_krylov_graph(p);
    drop_newton_graph(p);
    ++p.sp_gen;
    std::vector<uint8_t> mask((size_t)mask_n);
    HIP_TRY(hipMemcpyAsync(mask.data(), p.d_mask, (size_t)mask_n, hipMemcpyDeviceToHost, p.stream));
    HIP_TRY(hipStreamSynchronize(p.stream));
    std::vector<int64_t> rowptr(1, 0), ybase, src;
    std::vector<int32_t> xnode, ld;
    int64_t mo = 0;
    for (int e = 0; e < E; ++e) {
      const int ri = p.ni[e] / kNvar, rc = p.nc[e] / kNvar;
      const int rows = which == 0 ? ri : rc, cols = which == 0 ? rc : ri;
      for (int rb = 0; rb < rows; ++rb) {
        ybase.push_back(which == 0 ? p.off_i[e] + kNvar * rb : p.off_c[e] + kNvar * rb);
        for (int cb = 0; cb < cols; ++cb) {
          if (!mask[(size_t)(mo + (int64_t)rb * cols + cb)]) continue;
          xnode.push_back(which == 0 ? p.h_c_node[(size_t)(p.h_c_ptr[e] + cb)]
                                     : (int32_t)(p.off_i[e] / kNvar + cb));
          src.push_back(p.off_ib[e] + (int64_t)(kNvar * rb) * (kNvar * cols) + kNvar * cb);
          ld.push_back(kNvar * cols);
        }
        rowptr.push_back((int64_t)xnode.size());
      }
      mo += (int64_t)rows * cols;
    }
    dfree(op.d_rowptr); dfree(op.d_xnode); dfree(op.d_ybase); dfree(op.d_src); dfree(op.d_ld);
    op.n_rows = (int64_t)ybase.size();
    op.n_blocks = (int64_t)xnode.size();
    ST_TRY(upload(p, &op.d_rowptr, rowptr));
    ST_TRY(upload(p, &op.d_ybase, ybase));
    if (op.n_blocks > 0) {
      ST_TRY(upload(p, &op.d_xnode, xnode));
      ST_TRY(upload(p, &op.d_src, src));
      ST_TRY(upload(p, &op.d_ld, ld));
    }
    if (!op.d_mask_ref) ST_TRY(dalloc(p, &op.d_mask_ref, (size_t)std::max<int64_t>(mask_n, 1)));
    HIP_TRY(hipMemcpyAsync(op.d_mask_ref, p.d_mask, (size_t)mask_n, hipMemcpyDeviceToDevice, p.stream));
  }
  const size_t need = esize(p) * (size_t)std::max<int64_t>(op.n_blocks, 1) * 25;
  if (need > op.cap_val) {
    dfree(op.val);
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&op.val), need));
    op.cap_val = need;
  }
  HIP_TRY(launch_gather_blocks_ld(vals, op.d_src, op.d_ld, op.n_blocks, op.val, fp32(p), p.stream));
  return SCDG_OK;
}

scdg_status schur_apply_impl(Plan &p, const double *x, double *y) {
  PhaseTimer tm(p, SCDG_PHASE_SCHUR_APPLY);
  if (p.schur_mode == 2) {
    // S x = A_bb x - sum_e P_e A_bi(e) (A_ii(e)^-1 (A_ib(e) x[C_e])) through the nonzero blocks
    HIP_TRY(launch_bsr5_rows(p.sp_ib.n_rows, p.sp_ib.d_rowptr, p.sp_ib.d_xnode, p.sp_ib.val, fp32(p), x,
                             p.sp_ib.d_ybase, p.w_z, p.stream, p.halt));
    HIP_TRY(launch_gemv_batched(p.d_gv_inv, p.d_rt_inv, p.n_rt_inv, p.max_ni, p.ainv, fp32(p), p.w_z, nullptr,
                                p.w_z2, nullptr, 1.0, 0.0, nullptr, p.stream, p.halt));
    HIP_TRY(launch_bsr5_rows(p.sp_bi.n_rows, p.sp_bi.d_rowptr, p.sp_bi.d_xnode, p.sp_bi.val, fp32(p), p.w_z2,
                             p.sp_bi.d_ybase, p.w_t, p.stream, p.halt));
    HIP_TRY(launch_bsr_pull(p, true, 0.0, nullptr, nullptr, 1.0, x, -1.0, p.w_t, y, fp32(p)));
    return SCDG_OK;
  }
  if (p.schur_mode == 1) {
    // S x = A_bb x - sum_e P_e A_bi(e) (X_e x[C_e]), S never formed
    const void *abi = fp32(p) ? p.abi_lo : static_cast<const void *>(p.abi);
    HIP_TRY(launch_gemv_batched(p.d_gv_aib, p.d_rt_aib, p.n_rt_aib, p.max_nc, p.xmat, fp32(p), x, p.d_cmap,
                                p.w_z, nullptr, 1.0, 0.0, nullptr, p.stream, p.halt));
    HIP_TRY(launch_gemv_batched(p.d_gv_abi, p.d_rt_abi, p.n_rt_abi, p.max_ni, abi, fp32(p), p.w_z, nullptr,
                                p.w_t, nullptr, 1.0, 0.0, nullptr, p.stream, p.halt));
    HIP_TRY(launch_bsr_pull(p, true, 0.0, nullptr, nullptr, 1.0, x, -1.0, p.w_t, y, fp32(p)));
    return SCDG_OK;
  }
  // S x = A_bb,rem x + sum_e P_e T_e x[C_e],  T_e = folded A_bb blocks - A_bi(e) X_e:
  // the element GEMVs and the remainder rows in one launch, then the pull
  HIP_TRY(launch_schur_gemv_rem(p, x, p.w_t, p.w_rx, fp32(p)));
  HIP_TRY(launch_bsr_pull(p, false, 1.0, p.w_rx, nullptr, 0.0, x, 1.0, p.w_t, y, fp32(p)));
  return SCDG_OK;
}

scdg_status backsolve_impl(Plan &p, const double *b, const double *qb, double *dq) {
  PhaseTimer tm(p, SCDG_PHASE_BACKSOLVE);
  ST_TRY(apply_inverse(p, b, p.w_z));
  HIP_TRY(launch_gemv_batched(p.d_gv_aib, p.d_rt_aib, p.n_rt_aib, p.max_nc, p.xmat, fp32(p), qb,
                              p.d_cmap, dq, p.d_imap, -1.0, 1.0, p.w_z, p.stream));
  HIP_TRY(launch_scatter(qb, p.d_bmap, dq, p.n1, p.stream));
  return SCDG_OK;
}

// r = B - A dQ on the full FP64 system (r, B, dQ natural vectors)
scdg_status residual_impl(Plan &p, const double *b, const double *dq, double *r) {
  PhaseTimer tm(p, SCDG_PHASE_RESIDUAL);
  // interior rows: u = A_ii dQ_i + A_ib dQ_b[C_e]
  HIP_TRY(launch_gather(dq, p.d_bmap, p.w_qb, p.n1, p.stream));
  HIP_TRY(launch_gemv_batched(p.d_gv_inv, p.d_rt_inv, p.n_rt_inv, p.max_ni, p.aii, false, dq,
                              p.d_imap, p.w_z, nullptr, 1.0, 0.0, nullptr, p.stream));
  HIP_TRY(launch_gemv_batched(p.d_gv_aib, p.d_rt_aib, p.n_rt_aib, p.max_nc, p.aib, false, p.w_qb,
                              p.d_cmap, p.w_z, nullptr, 1.0, 1.0, p.w_z, p.stream));
  HIP_TRY(launch_scatter_axpby(p.n2, 1.0, b, -1.0, p.w_z, p.d_imap, r, p.stream));
  // boundary rows: B_b - A_bb dQ_b - pull(A_bi dQ_i)
  HIP_TRY(launch_gemv_batched(p.d_gv_abi, p.d_rt_abi, p.n_rt_abi, p.max_ni, p.abi, false, dq,
                              p.d_imap, p.w_t, nullptr, 1.0, 0.0, nullptr, p.stream));
  HIP_TRY(launch_bsr_pull(p, true, 1.0, b, p.d_bmap, -1.0, p.w_qb, -1.0, p.w_t, p.w_bs));
  HIP_TRY(launch_scatter(p.w_bs, p.d_bmap, r, p.n1, p.stream));
  return SCDG_OK;
}

scdg_status ensure_gmres(Plan &p, int m) {
  if (p.gm_v && p.gm_m >= m) return SCDG_OK;
  ST_TRY(dalloc(p, &p.gm_v, (size_t)(m + 1) * p.n1));
  p.gm_m = m;
  return SCDG_OK;
}

// One Arnoldi step j of the device-resident cycle: every kernel first reads the
// halt flag (p.halt) and returns at once after convergence, so the fixed
// sequence of m steps can be replayed from a graph.
scdg_status krylov_step(Plan &p, int j, int m, int pmode) {
  const int64_t n = p.n1;
  double *vj = p.gm_v + (int64_t)j * n;
  double *w = p.gm_w;
  HIP_TRY(launch_precond_apply(p, pmode, vj, p.gm_z, 1.0));
  ST_TRY(schur_apply_impl(p, p.gm_z, w));
  HIP_TRY(launch_multidot(p.gm_v, n, j + 1, w, n, p.gm_part, p.red_blocks, p.gm_h, p.stream, p.halt));
  HIP_TRY(launch_multi_axpy(p.gm_v, n, j + 1, p.gm_h, w, n, p.stream, nullptr, p.halt));
  HIP_TRY(launch_multidot(p.gm_v, n, j + 1, w, n, p.gm_part, p.red_blocks, p.gm_h + (m + 1), p.stream, p.halt));
  HIP_TRY(launch_multi_axpy(p.gm_v, n, j + 1, p.gm_h + (m + 1), w, n, p.stream, nullptr, p.halt));
  HIP_TRY(launch_multidot(w, 0, 1, w, n, p.gm_part, p.red_blocks, p.gm_h + 2 * (m + 1), p.stream, p.halt));
  HIP_TRY(launch_krylov_givens(j, m, p.gm_h, p.kr_H, p.kr_cs, p.kr_sn, p.kr_g, p.kr_st, p.kr_dev, p.stream));
  HIP_TRY(launch_diag_scale(w, nullptr, p.gm_v + (int64_t)(j + 1) * n, n, 1.0, p.stream, p.kr_dev, p.halt));
  return SCDG_OK;
}

void drop_krylov_graph(Plan &p) {
  if (p.kr_exec) (void)hipGraphExecDestroy(p.kr_exec);
  if (p.kr_graph) (void)hipGraphDestroy(p.kr_graph);
  p.kr_exec = nullptr;
  p.kr_graph = nullptr;
}

// The m Arnoldi steps of a cycle as a graph (captured once per configuration).
scdg_status krylov_graph(Plan &p, int m, int pmode) {
  KrylovKey key;
  key.m = m;
  key.pmode = pmode;
  key.fp32 = fp32(p);
  key.sloc = p.sloc;
  key.bb_val = p.bb_val;
  key.gm_v = p.gm_v;
  key.smode = p.schur_mode;
  const void *sp[7] = {p.sp_ib.val, p.sp_ib.d_rowptr, p.sp_bi.val, p.sp_bi.d_rowptr, p.w_z2, p.aib, p.abi};
  for (int i = 0; i < 7; ++i) key.sp[i] = sp[i];
  key.sp_gen = p.sp_gen;
  if (p.kr_exec && p.kr_key == key) return SCDG_OK;
  drop_krylov_graph(p);
  if (!p.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  // capture on the plan's own stream (the caller's may be the null stream,
  // which cannot be captured); the graph is launched on the caller's stream
  hipStream_t user = p.stream;
  p.stream = p.cap_stream;
  HIP_TRY(hipStreamBeginCapture(p.stream, hipStreamCaptureModeRelaxed));
  p.capturing = true;
  scdg_status st = SCDG_OK;
  for (int j = 0; j < m && st == SCDG_OK; ++j) st = krylov_step(p, j, m, pmode);
  p.capturing = false;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p.stream, &g);
  p.stream = user;
  if (st != SCDG_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    p.last_error = "capture of the GMRES cycle failed";
    return st != SCDG_OK ? st : SCDG_ERR_HIP;
  }
  if (hipGraphInstantiate(&p.kr_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    p.kr_exec = nullptr;
    p.last_error = "instantiation of the GMRES cycle graph failed";
    return SCDG_ERR_HIP;
  }
  p.kr_graph = g;
  p.kr_key = key;
  return SCDG_OK;
}

scdg_status ensure_krylov_state(Plan &p, int m) {
  if (p.kr_H && p.kr_m >= m) return SCDG_OK;
  dfree(p.kr_H); dfree(p.kr_cs); dfree(p.kr_sn); dfree(p.kr_g); dfree(p.kr_st); dfree(p.kr_dev);
  ST_TRY(dalloc(p, &p.kr_H, (size_t)(m + 1) * m));
  ST_TRY(dalloc(p, &p.kr_cs, (size_t)m));
  ST_TRY(dalloc(p, &p.kr_sn, (size_t)m));
  ST_TRY(dalloc(p, &p.kr_g, (size_t)m + 1));
  ST_TRY(dalloc(p, &p.kr_st, (size_t)8));
  ST_TRY(dalloc(p, &p.kr_dev, (size_t)4));
  p.kr_m = m;
  return SCDG_OK;
}

// Restart cycles with the Hessenberg column, the Givens rotations and the stopping
// test on the device; the host waits once per cycle (true residual).  r holds
// bs - S x on entry, beta its norm.
scdg_status gmres_device_cycles(Plan &p, const double *bs, double *x, double *r, double bnorm, double beta,
                                const scdg_solve_opts &o, scdg_solve_info &info) {
  const int64_t n = p.n1;
  const int m = o.restart;
  const int pmode = o.precond;
  const double target = o.tol * bnorm;
  ST_TRY(ensure_krylov_state(p, m));
  const bool use_graph = p.krylov_mode == 2;
  if (use_graph) {
    p.halt = p.kr_st;
    scdg_status st = krylov_graph(p, m, pmode);
    p.halt = nullptr;
    if (st != SCDG_OK) return st;
  }
  int it = 0;
  while (it < o.max_iters && beta > target) {
    if (!std::isfinite(beta)) {
      p.last_error = "non-finite GMRES residual";
      return SCDG_ERR_NONFINITE;
    }
    ++info.restarts;
    const int limit = std::min(m, o.max_iters - it);
    HIP_TRY(launch_diag_scale(r, nullptr, p.gm_v, n, 1.0 / beta, p.stream));
    HIP_TRY(launch_krylov_start(beta, target, limit, p.kr_g, p.kr_st, p.kr_dev, p.stream));
    if (use_graph) {
      HIP_TRY(hipGraphLaunch(p.kr_exec, p.stream));
    } else {
      p.halt = p.kr_st;
      scdg_status st = SCDG_OK;
      for (int j = 0; j < limit && st == SCDG_OK; ++j) st = krylov_step(p, j, m, pmode);
      p.halt = nullptr;
      if (st != SCDG_OK) return st;
    }
    // x += Dinv (V y)
    HIP_TRY(launch_krylov_solve(m, p.kr_H, p.kr_g, p.kr_st, p.gm_h, p.stream));
    HIP_TRY(hipMemsetAsync(p.gm_z, 0, sizeof(double) * n, p.stream));
    HIP_TRY(launch_multi_axpy(p.gm_v, n, m, p.gm_h, p.gm_z, n, p.stream, p.kr_st + 1, nullptr));
    HIP_TRY(launch_precond_apply(p, pmode, p.gm_z, p.gm_w, 1.0));
    HIP_TRY(launch_axpby(n, 1.0, p.gm_w, 1.0, x, p.stream));
    HIP_TRY(hipMemcpyAsync(p.h_pinned + 8, p.kr_st, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, p.stream));
    // true residual
    ST_TRY(schur_apply_impl(p, x, r));
    HIP_TRY(launch_axpby(n, 1.0, bs, -1.0, r, p.stream));
    double beta2;
    ST_TRY(norm2sq(p, r, n, &beta2));
    int32_t done[2];
    std::memcpy(done, p.h_pinned + 8, sizeof(done));
    it += done[1];
    beta = std::sqrt(beta2);
    info.rel_res_S = beta / bnorm;
    if (done[1] == 0) break;   // no progress possible (breakdown at the first step)
  }
  info.iters += it;
  if (beta > target) {
    p.last_error = "GMRES did not reach the tolerance";
    return SCDG_ERR_NOCONV;
  }
  return SCDG_OK;
}

scdg_status gmres(Plan &p, const double *bs, double *x, const double *x0, const scdg_solve_opts &o,
                  scdg_solve_info &info) {
  const int64_t n = p.n1;
  const int m = o.restart;
  ST_TRY(ensure_gmres(p, m));
  const int pmode = o.precond;  // 0 none, 1 point Jacobi, 2 5x5 node-block Jacobi
  double bnorm2;
  ST_TRY(norm2sq(p, bs, n, &bnorm2));
  if (!std::isfinite(bnorm2)) {
    p.last_error = "non-finite condensed right-hand side";
    return SCDG_ERR_NONFINITE;
  }
  const double bnorm = std::sqrt(bnorm2);
  if (bnorm == 0.0) {
    HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, p.stream));
    info.rel_res_S = 0.0;
    return SCDG_OK;
  }
  double *r = p.gm_w;
  if (x0) {
    if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, p.stream));
    ST_TRY(schur_apply_impl(p, x, r));
    HIP_TRY(launch_axpby(n, 1.0, bs, -1.0, r, p.stream));  // r = bs - S x
  } else {
    HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, p.stream));
    HIP_TRY(hipMemcpyAsync(r, bs, sizeof(double) * n, hipMemcpyDeviceToDevice, p.stream));
  }
  double beta2;
  ST_TRY(norm2sq(p, r, n, &beta2));
  double beta = std::sqrt(beta2);
  if (info.rel_res_guess < 0) info.rel_res_guess = x0 ? beta / bnorm : 1.0;
  if (x0 && !(beta <= bnorm)) {
    // the guess is worse than none (or not finite): start from zero instead
    info.guess_rejected = 1;
    HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, p.stream));
    HIP_TRY(hipMemcpyAsync(r, bs, sizeof(double) * n, hipMemcpyDeviceToDevice, p.stream));
    beta = bnorm;
  }
  if (p.krylov_mode != 0) return gmres_device_cycles(p, bs, x, r, bnorm, beta, o, info);
  std::vector<double> h((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  int it = 0;
  const double target = o.tol * bnorm;
  while (it < o.max_iters && beta > target) {
    if (!std::isfinite(beta)) {
      p.last_error = "non-finite GMRES residual";
      return SCDG_ERR_NONFINITE;
    }
    ++info.restarts;
    HIP_TRY(launch_diag_scale(r, nullptr, p.gm_v, n, 1.0 / beta, p.stream));
    std::fill(h.begin(), h.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jused = 0;
    for (int j = 0; j < m && it < o.max_iters; ++j) {
      double *vj = p.gm_v + (int64_t)j * n;
      double *w = p.gm_w;
      HIP_TRY(launch_precond_apply(p, pmode, vj, p.gm_z, 1.0));
      ST_TRY(schur_apply_impl(p, p.gm_z, w));
      // classical Gram-Schmidt, twice (FP64)
      HIP_TRY(launch_multidot(p.gm_v, n, j + 1, w, n, p.gm_part, p.red_blocks, p.gm_h, p.stream));
      HIP_TRY(launch_multi_axpy(p.gm_v, n, j + 1, p.gm_h, w, n, p.stream));
      HIP_TRY(launch_multidot(p.gm_v, n, j + 1, w, n, p.gm_part, p.red_blocks, p.gm_h + (m + 1),
                              p.stream));
      HIP_TRY(launch_multi_axpy(p.gm_v, n, j + 1, p.gm_h + (m + 1), w, n, p.stream));
      HIP_TRY(launch_multidot(w, 0, 1, w, n, p.gm_part, p.red_blocks, p.gm_h + 2 * (m + 1), p.stream));
      HIP_TRY(hipMemcpyAsync(p.h_pinned, p.gm_h, sizeof(double) * 3 * (m + 1), hipMemcpyDeviceToHost,
                             p.stream));
      ST_TRY(sync(p));
      for (int i = 0; i <= j; ++i) h[(size_t)i * m + j] = p.h_pinned[i] + p.h_pinned[(m + 1) + i];
      const double hn = std::sqrt(std::max(0.0, p.h_pinned[2 * (m + 1)]));
      h[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0)
        HIP_TRY(launch_diag_scale(w, nullptr, p.gm_v + (int64_t)(j + 1) * n, n, 1.0 / hn, p.stream));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[(size_t)i * m + j] + sn[i] * h[(size_t)(i + 1) * m + j];
        h[(size_t)(i + 1) * m + j] = -sn[i] * h[(size_t)i * m + j] + cs[i] * h[(size_t)(i + 1) * m + j];
        h[(size_t)i * m + j] = t;
      }
      const double den = std::hypot(h[(size_t)j * m + j], hn);
      cs[j] = den > 0 ? h[(size_t)j * m + j] / den : 1.0;
      sn[j] = den > 0 ? hn / den : 0.0;
      h[(size_t)j * m + j] = den;
      h[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jused = j + 1;
      info.rel_res_S = std::fabs(g[j + 1]) / bnorm;
      if (std::fabs(g[j + 1]) <= target || hn == 0.0) break;
    }
    for (int i = jused - 1; i >= 0; --i) {
      double v = g[i];
      for (int q = i + 1; q < jused; ++q) v -= h[(size_t)i * m + q] * y[q];
      y[i] = v / h[(size_t)i * m + i];
    }
    // x += Dinv (V y): accumulate V y into z with negated coefficients
    for (int i = 0; i < jused; ++i) p.h_pinned[i] = -y[i];
    HIP_TRY(hipMemcpyAsync(p.gm_h, p.h_pinned, sizeof(double) * jused, hipMemcpyHostToDevice, p.stream));
    HIP_TRY(hipMemsetAsync(p.gm_z, 0, sizeof(double) * n, p.stream));
    HIP_TRY(launch_multi_axpy(p.gm_v, n, jused, p.gm_h, p.gm_z, n, p.stream));
    HIP_TRY(launch_precond_apply(p, pmode, p.gm_z, p.gm_w, 1.0));
    HIP_TRY(launch_axpby(n, 1.0, p.gm_w, 1.0, x, p.stream));
    // true residual
    ST_TRY(schur_apply_impl(p, x, r));
    HIP_TRY(launch_axpby(n, 1.0, bs, -1.0, r, p.stream));
    ST_TRY(norm2sq(p, r, n, &beta2));
    beta = std::sqrt(beta2);
    info.rel_res_S = beta / bnorm;
  }
  info.iters += it;
  if (beta > target) {
    p.last_error = "GMRES did not reach the tolerance";
    return SCDG_ERR_NOCONV;
  }
  return SCDG_OK;
}

// ---- one Newton iteration of the implicit step, captured as a graph ----

void drop_newton_graph(Plan &p) {
  for (int i = 0; i < 3; ++i) {
    if (p.nw_exec[i]) (void)hipGraphExecDestroy(p.nw_exec[i]);
    if (p.nw_graph[i]) (void)hipGraphDestroy(p.nw_graph[i]);
    p.nw_exec[i] = nullptr;
    p.nw_graph[i] = nullptr;
  }
}

struct NewtonSetup {
  int m, cycles, pmode;
  double eta_c, lin_tol, eta_max, inv_dt;
};

NewtonKey newton_key(const Plan &p, scdg_dg *dg, const double *q_s, const double *q, const NewtonSetup &ns) {
  NewtonKey k;
  k.m = ns.m;
  k.cycles = 0;   // the cycle budget is a host loop bound, not part of any graph
  k.pmode = ns.pmode;
  k.smode = p.schur_mode;
  k.sp_gen = p.sp_gen;
  k.fp32 = fp32(p);
  k.inv_dt = ns.inv_dt;
  k.eta_c = ns.eta_c;
  k.lin_tol = ns.lin_tol;
  k.eta_max = ns.eta_max;
  k.q = q;
  k.q_s = q_s;
  k.dg = dg;
  dg_graph_state(dg, &k.dg_gen, &k.dg_g, &k.dg_met, &k.dg_params);
  const void *ptrs[23] = {p.ainv, p.xmat, p.sloc,  p.abi,  p.abi_lo, p.bb_val, p.rem_val, p.gm_v,
                          p.nw_r, p.nw_dq, p.diag_s, p.pc_blk, p.kr_H, p.kr_cs, p.kr_sn,  p.kr_g,
                          p.kr_st, p.kr_dev, p.sp_ib.val, p.sp_ib.d_rowptr, p.sp_bi.val, p.sp_bi.d_rowptr,
                          p.w_z2};
  for (int i = 0; i < 23; ++i) k.ptr[i] = ptrs[i];
  return k;
}

// One Newton iteration is enqueued as three pieces, each captured as a graph.
// The linear system is solved for the right-hand side R (not -R):
// x = S^-1 condense(R), nw_dq = backsolve(R, x) = -dQ.
// Piece 0: on entry nw_r holds R(Q), nw_stat[0] its squared norm and
// nw_stat[2] = ||R(Q_s)||; condensed right-hand side, x = 0, GMRES set-up.
scdg_status newton_piece_setup(Plan &p, const NewtonSetup &ns) {
  const int64_t n = p.n1;
  p.halt = nullptr;
  ST_TRY(condense_rhs_impl(p, p.nw_r, p.w_bs));
  HIP_TRY(launch_multidot(p.w_bs, 0, 1, p.w_bs, n, p.gm_part, p.red_blocks, p.nw_stat + 1, p.stream));
  HIP_TRY(launch_fill(p.w_qb, n, 0.0, p.stream));
  HIP_TRY(launch_newton_gmres_setup(p.nw_stat, ns.eta_c, ns.lin_tol, ns.eta_max, ns.m, p.kr_g, p.kr_st,
                                    p.kr_dev, p.stream));
  HIP_TRY(launch_diag_scale(p.w_bs, nullptr, p.gm_v, n, 1.0, p.stream, p.kr_dev, p.kr_st + 3));
  return SCDG_OK;
}

// Piece 1: one restart cycle (m Arnoldi steps that stop on the device flag),
// x += Dinv V y, the true residual, and the set-up of the next cycle; every
// kernel returns at once once the solve has finished (kr_st[3]).
scdg_status newton_piece_cycle(Plan &p, const NewtonSetup &ns) {
  const int64_t n = p.n1;
  const int m = ns.m;
  int32_t *st = p.kr_st;
  const int32_t *done = p.kr_st + 3;
  double *rg = p.gm_w;
  p.halt = st;
  scdg_status s1 = SCDG_OK;
  for (int j = 0; j < m && s1 == SCDG_OK; ++j) s1 = krylov_step(p, j, m, ns.pmode);
  p.halt = done;
  if (s1 == SCDG_OK) {
    HIP_TRY(launch_krylov_solve(m, p.kr_H, p.kr_g, st, p.gm_h, p.stream, done));
    HIP_TRY(launch_fill(p.gm_z, n, 0.0, p.stream, done));
    HIP_TRY(launch_multi_axpy(p.gm_v, n, m, p.gm_h, p.gm_z, n, p.stream, st + 1, done));
    HIP_TRY(launch_precond_apply(p, ns.pmode, p.gm_z, rg, 1.0));
    HIP_TRY(launch_axpby(n, 1.0, rg, 1.0, p.w_qb, p.stream, done));
    s1 = schur_apply_impl(p, p.w_qb, rg);
  }
  if (s1 == SCDG_OK) {
    HIP_TRY(launch_axpby(n, 1.0, p.w_bs, -1.0, rg, p.stream, done));
    HIP_TRY(launch_multidot(rg, 0, 1, rg, n, p.gm_part, p.red_blocks, p.nw_stat + 3, p.stream, done));
    HIP_TRY(launch_newton_gmres_restart(p.nw_stat, m, p.kr_g, st, p.kr_dev, p.stream));
    HIP_TRY(launch_diag_scale(rg, nullptr, p.gm_v, n, 1.0, p.stream, p.kr_dev, done));
  }
  p.halt = nullptr;
  return s1;
}

// Piece 2: back-substitution, Q += dQ, R(Q) and its squared norm.
scdg_status newton_piece_update(Plan &p, scdg_dg *dg, const double *q_s, double *q, const NewtonSetup &ns) {
  p.halt = nullptr;
  ST_TRY(backsolve_impl(p, p.nw_r, p.w_qb, p.nw_dq));
  HIP_TRY(launch_axpby(p.n_dof, -1.0, p.nw_dq, 1.0, q, p.stream));
  HIP_TRY(dg_residual_on(dg, q, q_s, ns.inv_dt, p.nw_r, p.stream));
  HIP_TRY(launch_multidot(p.nw_r, 0, 1, p.nw_r, p.n_dof, p.gm_part, p.red_blocks, p.nw_stat, p.stream));
  return SCDG_OK;
}

scdg_status newton_graphs(Plan &p, scdg_dg *dg, const double *q_s, double *q, const NewtonSetup &ns) {
  const NewtonKey key = newton_key(p, dg, q_s, q, ns);
  if (p.nw_exec[0] && p.nw_key == key) return SCDG_OK;
  drop_newton_graph(p);
  if (!p.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  for (int piece = 0; piece < 3; ++piece) {
    hipStream_t user = p.stream;
    p.stream = p.cap_stream;
    HIP_TRY(hipStreamBeginCapture(p.stream, hipStreamCaptureModeRelaxed));
    p.capturing = true;
    const scdg_status st = piece == 0   ? newton_piece_setup(p, ns)
                           : piece == 1 ? newton_piece_cycle(p, ns)
                                        : newton_piece_update(p, dg, q_s, q, ns);
    p.capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p.stream, &g);
    p.stream = user;
    if (st != SCDG_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      drop_newton_graph(p);
      p.last_error = "capture of the Newton iteration failed";
      return st != SCDG_OK ? st : SCDG_ERR_HIP;
    }
    if (hipGraphInstantiate(&p.nw_exec[piece], g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      p.nw_exec[piece] = nullptr;
      drop_newton_graph(p);
      p.last_error = "instantiation of the Newton iteration graph failed";
      return SCDG_ERR_HIP;
    }
    p.nw_graph[piece] = g;
  }
  p.nw_key = key;
  return SCDG_OK;
}

scdg_status dense_solve(Plan &p, const double *bs, double *x) {
  if (!p.dense_factored) {
    ST_TRY(dalloc(p, &p.s_dense, (size_t)p.n1 * p.n1));
    ST_TRY(dalloc(p, &p.s_piv, (size_t)p.n1));
    ST_TRY(dalloc(p, &p.d_dense_info, 1));
    HIP_TRY(launch_dense_assemble(p, p.s_dense));
    HIP_TRY(launch_dense_lu(p, p.s_dense, (int32_t)p.n1, p.s_piv, p.d_dense_info));
    int32_t info = 0;
    HIP_TRY(hipMemcpy(&info, p.d_dense_info, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (info != 0) {
      p.last_error = "zero pivot in the dense LU of S at step " + std::to_string(info);
      return SCDG_ERR_SINGULAR;
    }
    p.dense_factored = true;
  }
  if (x != bs) HIP_TRY(hipMemcpyAsync(x, bs, sizeof(double) * p.n1, hipMemcpyDeviceToDevice, p.stream));
  HIP_TRY(launch_dense_solve(p.s_dense, (int32_t)p.n1, p.s_piv, x, p.stream));
  return SCDG_OK;
}

// a solve that never looked at a guess reports a guess residual of 1
scdg_solve_info finish_info(scdg_solve_info inf) {
  if (inf.rel_res_guess < 0) inf.rel_res_guess = 1.0;
  return inf;
}

void defaults(scdg_solve_opts &o) {
  if (o.restart <= 0) o.restart = 30;
  if (o.max_iters <= 0) o.max_iters = 1000;
  if (o.tol <= 0) o.tol = 1e-10;
  if (o.precond < 0) o.precond = 1;
  if (o.precond > 2) o.precond = 2;
  if (o.ir_max <= 0) o.ir_max = 10;
  if (o.ir_tol <= 0) o.ir_tol = 1e-8;
}

scdg_status solve_condensed_impl(Plan &p, const double *bs, double *qb, const double *x0,
                                 const scdg_solve_opts &o, scdg_solve_info &info) {
  PhaseTimer tm(p, SCDG_PHASE_CONDENSED);
  int solver = o.solver;
  if (solver == SCDG_SOLVER_AUTO)
    solver = p.n1 <= 8192 && p.schur_mode == 0 ? SCDG_SOLVER_DENSE : SCDG_SOLVER_GMRES;
  info.solver_used = solver;
  if (solver == SCDG_SOLVER_DENSE && p.schur_mode != 0) {
    p.last_error = "the dense solve needs the assembled S (scdg_set_schur_mode 0)";
    return SCDG_ERR_STATE;
  }
  if (solver == SCDG_SOLVER_DENSE) {
    if (p.n1 > 40000) {
      p.last_error = "dense solve of S limited to n1 <= 40000";
      return SCDG_ERR_UNSUPPORTED;
    }
    info.rel_res_S = 0.0;
    return dense_solve(p, bs, qb);
  }
  if (solver != SCDG_SOLVER_GMRES) {
    p.last_error = "unknown solver";
    return SCDG_ERR_ARG;
  }
  return gmres(p, bs, qb, x0, o, info);
}

}  // namespace

// =====================================================================
extern "C" {

const char *scdg_status_string(scdg_status s) {
  switch (s) {
    case SCDG_OK: return "ok";
    case SCDG_ERR_ARG: return "invalid argument";
    case SCDG_ERR_STATE: return "call out of order";
    case SCDG_ERR_HIP: return "HIP runtime error";
    case SCDG_ERR_NOMEM: return "out of device memory";
    case SCDG_ERR_SINGULAR: return "singular pivot";
    case SCDG_ERR_NOCONV: return "no convergence";
    case SCDG_ERR_NONFINITE: return "non-finite value";
    case SCDG_ERR_UNSUPPORTED: return "unsupported size or order";
  }
  return "unknown status";
}

scdg_status scdg_last_error(const scdg_plan *pl, char *buf, size_t n) {
  if (!buf || n == 0) return SCDG_ERR_ARG;
  const std::string &s = pl ? pl->p.last_error : g_create_error;
  std::snprintf(buf, n, "%s", s.c_str());
  return SCDG_OK;
}

scdg_status scdg_plan_destroy(scdg_plan *pl) {
  if (!pl) return SCDG_OK;
  Plan &p = pl->p;
  (void)hipStreamSynchronize(p.stream);
  dfree(p.d_imap); dfree(p.d_bmap); dfree(p.d_cmap); dfree(p.d_pull_ptr); dfree(p.d_pull_idx);
  dfree(p.d_slot_soff); dfree(p.d_slot_nc); dfree(p.d_slot_pos); dfree(p.d_slot_ib); dfree(p.d_slot_ni);
  dfree(p.mf_dblk);
  for (SparseOp *op : {&p.sp_ib, &p.sp_bi}) {
    dfree(op->d_rowptr); dfree(op->d_xnode); dfree(op->d_ybase); dfree(op->d_src); dfree(op->d_ld);
    dfree(op->val); dfree(op->d_mask_ref);
  }
  dfree(p.d_mask_flag); dfree(p.bb_lo); dfree(p.rem_lo);
  dfree(p.d_mask); dfree(p.d_e_offib); dfree(p.d_e_maskoff); dfree(p.d_e_ri); dfree(p.d_e_rc); dfree(p.w_z2);
  dfree(p.d_fold_map);
  dfree(p.d_rem_rowptr); dfree(p.d_rem_col); dfree(p.d_rem_src); dfree(p.pc_blk); dfree(p.rem_val);
  dfree(p.d_remt_rowptr); dfree(p.d_remt_col); dfree(p.d_remt_src); dfree(p.d_ct_s);
  dfree(p.d_bb_rowptr); dfree(p.d_bb_col); dfree(p.d_inv_n); dfree(p.d_inv_off); dfree(p.d_inv_order); dfree(p.d_info);
  dfree(p.d_jac_cnode);
  dfree(p.own_aii); dfree(p.own_aib); dfree(p.own_abi); dfree(p.own_bb);
  dfree(p.d_gx); dfree(p.d_gs); dfree(p.d_tiles_x); dfree(p.d_tiles_s);
  dfree(p.d_gv_inv); dfree(p.d_gv_abi); dfree(p.d_gv_aib); dfree(p.d_gv_s);
  dfree(p.d_rt_inv); dfree(p.d_rt_abi); dfree(p.d_rt_aib); dfree(p.d_rt_s);
  drop_krylov_graph(p);
  if (p.cap_stream) (void)hipStreamDestroy(p.cap_stream);
  dfree(p.kr_H); dfree(p.kr_cs); dfree(p.kr_sn); dfree(p.kr_g); dfree(p.kr_st); dfree(p.kr_dev);
  drop_newton_graph(p);
  dfree(p.nw_r); dfree(p.nw_dq); dfree(p.nw_stat);
  dfree(p.d_gj_voff); dfree(p.d_gj_piv); dfree(p.d_gj_flag); dfree(p.gj_pbuf); dfree(p.gj_rbuf);
  dfree(p.d_gj_desc); dfree(p.d_gj_tiles);
  dfree(p.ainv); dfree(p.ainv_work); dfree(p.xmat); dfree(p.sloc); dfree(p.aib_lo); dfree(p.abi_lo); dfree(p.diag_s);
  dfree(p.s_dense); dfree(p.s_piv); dfree(p.d_dense_info);
  dfree(p.w_z); dfree(p.w_t); dfree(p.w_bs); dfree(p.w_qb); dfree(p.w_r); dfree(p.w_rx); dfree(p.w_dq); dfree(p.w_vec);
  dfree(p.gm_v); dfree(p.gm_w); dfree(p.gm_z); dfree(p.gm_part); dfree(p.gm_h);
  if (p.h_pinned) (void)hipHostFree(p.h_pinned);
  for (auto &u : p.ev_used) p.ev_pool.push_back(u.second);
  for (auto &e : p.ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete pl;
  return SCDG_OK;
}

scdg_status scdg_plan_create(scdg_plan **out, const scdg_structure *s, void *hip_stream, int32_t device) {
  if (!out || !s || !s->order || !s->c_ptr || !s->c_node || !s->bb_rowptr || s->n_elem <= 0) {
    g_create_error = "null pointer or empty mesh in scdg_structure";
    return SCDG_ERR_ARG;
  }
  *out = nullptr;
  if (device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
      g_create_error = "no HIP device " + std::to_string(device);
      return SCDG_ERR_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) {
      g_create_error = "hipSetDevice failed";
      return SCDG_ERR_HIP;
    }
  } else if (device != -1) {
    g_create_error = "device must be -1 or a device index";
    return SCDG_ERR_ARG;
  }
  scdg_plan *pl = new (std::nothrow) scdg_plan();
  if (!pl) return SCDG_ERR_NOMEM;
  Plan &p = pl->p;
  static std::atomic<uint64_t> next_uid{1};
  p.uid = next_uid.fetch_add(1);
  p.stream = static_cast<hipStream_t>(hip_stream);
  (void)hipGetDevice(&p.device);
  const int E = s->n_elem;
  p.n_elem = E;
  p.order.assign(s->order, s->order + E);
  p.ni.resize(E); p.nc.resize(E);
  p.off_q.resize(E + 1); p.off_ii.resize(E + 1); p.off_ib.resize(E + 1); p.off_cc.resize(E + 1);
  p.off_i.resize(E + 1); p.off_c.resize(E + 1); p.bnode_off.resize(E + 1);
  p.off_q[0] = p.off_ii[0] = p.off_ib[0] = p.off_cc[0] = p.off_i[0] = p.off_c[0] = p.bnode_off[0] = 0;
  for (int e = 0; e < E; ++e) {
    const int N = p.order[e];
    if (N < 2 || N > kMaxOrder) {
      g_create_error = "element order outside 2..7";
      delete pl;
      return SCDG_ERR_UNSUPPORTED;
    }
    const int64_t cnt = s->c_ptr[e + 1] - s->c_ptr[e];
    if (cnt <= 0 || s->c_ptr[e] < 0) {
      g_create_error = "c_ptr must be increasing with non-empty coupling sets";
      delete pl;
      return SCDG_ERR_ARG;
    }
    const int P = N + 1;
    const int phys = s->phys_faces ? s->phys_faces[e] : 0;
    if (phys & 0xC0) {
      g_create_error = "phys_faces: bits 6 and 7 must be zero";
      delete pl;
      return SCDG_ERR_ARG;
    }
    std::vector<int> in_n, b_n;
    local_node_sets(N, phys, in_n, b_n);
    p.ni[e] = kNvar * (int32_t)in_n.size();
    p.nc[e] = (int32_t)(kNvar * cnt);
    p.off_q[e + 1] = p.off_q[e] + (int64_t)kNvar * P * P * P;
    p.off_ii[e + 1] = p.off_ii[e] + (int64_t)p.ni[e] * p.ni[e];
    p.off_ib[e + 1] = p.off_ib[e] + (int64_t)p.ni[e] * p.nc[e];
    p.off_cc[e + 1] = p.off_cc[e] + (int64_t)p.nc[e] * p.nc[e];
    p.off_i[e + 1] = p.off_i[e] + p.ni[e];
    p.off_c[e + 1] = p.off_c[e] + p.nc[e];
    p.bnode_off[e + 1] = p.bnode_off[e] + (int64_t)b_n.size();
    p.max_ni = std::max(p.max_ni, p.ni[e]);
    p.max_nc = std::max(p.max_nc, p.nc[e]);
  }
  p.n_dof = p.off_q[E];
  p.n2 = p.off_i[E];
  p.n_bnodes = p.bnode_off[E];
  p.n1 = kNvar * p.n_bnodes;
  if (p.n_dof >= (int64_t)INT32_MAX || p.off_c[E] >= (int64_t)INT32_MAX) {
    g_create_error = "problem too large for 32-bit DOF indices";
    delete pl;
    return SCDG_ERR_UNSUPPORTED;
  }
  p.nnzb = s->bb_rowptr[p.n_bnodes];
  if (p.nnzb < 0 || (p.nnzb > 0 && !s->bb_col)) {
    g_create_error = "bad A_bb pattern";
    delete pl;
    return SCDG_ERR_ARG;
  }
  for (int64_t g = 0; g < p.n_bnodes; ++g)
    if (s->bb_rowptr[g + 1] < s->bb_rowptr[g]) {
      g_create_error = "bb_rowptr not monotone";
      delete pl;
      return SCDG_ERR_ARG;
    }
  for (int64_t t = 0; t < p.nnzb; ++t)
    if (s->bb_col[t] < 0 || s->bb_col[t] >= p.n_bnodes) {
      g_create_error = "bb_col out of range";
      delete pl;
      return SCDG_ERR_ARG;
    }

  // ---- index maps (a1) ----
  std::vector<int32_t> imap(p.n2), bmap(p.n1), cmap(p.off_c[E]);
  std::vector<int> in_nodes, b_nodes;
  std::vector<int32_t> pull_cnt(p.n_bnodes + 1, 0);
  int cur_order = -1, cur_phys = -1;
  for (int e = 0; e < E; ++e) {
    const int phys = s->phys_faces ? s->phys_faces[e] : 0;
    if (p.order[e] != cur_order || phys != cur_phys) {
      local_node_sets(p.order[e], phys, in_nodes, b_nodes);
      cur_order = p.order[e];
      cur_phys = phys;
    }
    for (size_t t = 0; t < in_nodes.size(); ++t)
      for (int v = 0; v < kNvar; ++v)
        imap[p.off_i[e] + kNvar * t + v] = (int32_t)(p.off_q[e] + kNvar * in_nodes[t] + v);
    for (size_t r = 0; r < b_nodes.size(); ++r)
      for (int v = 0; v < kNvar; ++v)
        bmap[kNvar * (p.bnode_off[e] + r) + v] = (int32_t)(p.off_q[e] + kNvar * b_nodes[r] + v);
    const int64_t c0 = s->c_ptr[e], c1 = s->c_ptr[e + 1];
    for (int64_t q = c0; q < c1; ++q) {
      const int32_t g = s->c_node[q];
      if (g < 0 || g >= p.n_bnodes || (q > c0 && s->c_node[q - 1] >= g)) {
        g_create_error = "c_node entries must be ascending boundary ids within range";
        delete pl;
        return SCDG_ERR_ARG;
      }
      for (int v = 0; v < kNvar; ++v) cmap[p.off_c[e] + kNvar * (q - c0) + v] = kNvar * g + v;
      pull_cnt[g + 1]++;
    }
  }
  const int64_t n_slots = p.off_c[E] / kNvar;
  p.h_c_ptr.assign(s->c_ptr, s->c_ptr + E + 1);
  p.h_c_node.assign(s->c_node, s->c_node + s->c_ptr[E]);
  std::vector<int32_t> pull_ptr(p.n_bnodes + 1, 0), pull_idx(n_slots);
  for (int64_t g = 0; g < p.n_bnodes; ++g) pull_ptr[g + 1] = pull_ptr[g] + pull_cnt[g + 1];
  std::vector<int32_t> fill(pull_ptr.begin(), pull_ptr.end() - 1);
  std::vector<int64_t> slot_soff(n_slots), slot_ib(n_slots);
  std::vector<int32_t> slot_nc(n_slots), slot_pos(n_slots), slot_ni(n_slots);
  for (int e = 0; e < E; ++e) {
    const int64_t c0 = s->c_ptr[e];
    for (int64_t q = c0; q < s->c_ptr[e + 1]; ++q) {
      const int64_t slot = p.off_c[e] / kNvar + (q - c0);
      pull_idx[fill[s->c_node[q]]++] = (int32_t)slot;
      slot_soff[slot] = p.off_cc[e];
      slot_nc[slot] = p.nc[e];
      slot_pos[slot] = (int32_t)(q - c0);
      slot_ib[slot] = p.off_ib[e];
      slot_ni[slot] = p.ni[e];
    }
  }
  // ---- A_bb fold: block (g, h) goes to the element that owns node g when both
  // g and h lie in its coupling set, else to the lowest-numbered element whose
  // coupling set holds both; blocks with no such element form the remainder.
  std::vector<int32_t> slot_elem(n_slots);
  for (int e = 0; e < E; ++e)
    for (int64_t q = s->c_ptr[e]; q < s->c_ptr[e + 1]; ++q)
      slot_elem[p.off_c[e] / kNvar + (q - s->c_ptr[e])] = e;
  // per element, the A_bb block folded into each node block of T_e (|C_e|^2
  // entries, -1 for none)
  std::vector<int64_t> fm_off(E + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int64_t ncn = p.nc[e] / kNvar;
    fm_off[e + 1] = fm_off[e] + ncn * ncn;
  }
  std::vector<int32_t> fold_map((size_t)std::max<int64_t>(fm_off[E], 1), -1);
  std::vector<int32_t> rem_col, rem_src;
  std::vector<int64_t> rem_rowptr(p.n_bnodes + 1, 0);
  int64_t n_fold = 0;
  {
    std::vector<std::pair<int, int>> cand;
    for (int64_t g = 0; g < p.n_bnodes; ++g) {
      const int owner = (int)(std::upper_bound(p.bnode_off.begin(), p.bnode_off.end(), g) -
                              p.bnode_off.begin()) - 1;
      cand.clear();
      for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q)
        cand.emplace_back(slot_elem[pull_idx[q]], slot_pos[pull_idx[q]]);
      std::sort(cand.begin(), cand.end(), [owner](const std::pair<int, int> &a, const std::pair<int, int> &b) {
        const bool ao = a.first == owner, bo = b.first == owner;
        if (ao != bo) return ao;
        return a.first < b.first;
      });
      for (int64_t t = s->bb_rowptr[g]; t < s->bb_rowptr[g + 1]; ++t) {
        const int32_t h = s->bb_col[t];
        bool done = false;
        for (const auto &cp : cand) {
          const int e = cp.first;
          const int32_t *cb = s->c_node + s->c_ptr[e], *ce = s->c_node + s->c_ptr[e + 1];
          const int32_t *it = std::lower_bound(cb, ce, h);
          if (it != ce && *it == h) {
            const int64_t pos_h = it - cb;
            fold_map[fm_off[e] + (int64_t)cp.second * (p.nc[e] / kNvar) + pos_h] = (int32_t)t;
            ++n_fold;
            done = true;
            break;
          }
        }
        if (!done) {
          rem_col.push_back(h);
          rem_src.push_back((int32_t)t);
        }
      }
      rem_rowptr[g + 1] = (int64_t)rem_col.size();
    }
  }
  p.n_fold = n_fold;
  p.n_rem = (int64_t)rem_col.size();
  std::vector<int64_t> bb_rowptr(s->bb_rowptr, s->bb_rowptr + p.n_bnodes + 1);
  std::vector<int32_t> bb_col(s->bb_col, s->bb_col + p.nnzb);
  std::vector<int32_t> inv_n(p.ni.begin(), p.ni.end());
  std::vector<int64_t> inv_off(p.off_ii.begin(), p.off_ii.end() - 1);

  // ---- GEMM / GEMV work lists ----
  std::vector<GemmDesc> gx(E), gs(E);
  std::vector<GemvDesc> gv_inv(E), gv_abi(E), gv_aib(E), gv_s(E);
  for (int e = 0; e < E; ++e) {
    const int ni = p.ni[e], nc = p.nc[e];
    gx[e] = GemmDesc{p.off_ii[e], p.off_ib[e], p.off_ib[e], ni, nc, ni, ni, nc, nc};
    gs[e] = GemmDesc{p.off_ib[e], p.off_ib[e], p.off_cc[e], nc, nc, ni, ni, nc, nc, fm_off[e]};
    gv_inv[e] = GemvDesc{p.off_ii[e], ni, ni, (int32_t)p.off_i[e], (int32_t)p.off_i[e]};
    gv_abi[e] = GemvDesc{p.off_ib[e], nc, ni, (int32_t)p.off_i[e], (int32_t)p.off_c[e]};
    gv_aib[e] = GemvDesc{p.off_ib[e], ni, nc, (int32_t)p.off_c[e], (int32_t)p.off_i[e]};
    gv_s[e] = GemvDesc{p.off_cc[e], nc, nc, (int32_t)p.off_c[e], (int32_t)p.off_c[e]};
  }
  // X_e is n_i x n_c (n_i = 5 (N-1)^3 is a multiple of 64 only for some N): 64-row tiles;
  // the element Schur blocks are n_c x n_c: 128 x 128 tiles
  p.gemm_cfg_x = kGemm64x128;
  p.gemm_cfg_s = kGemm64x64;
  p.gx_host = gx;
  p.gs_host = gs;
  std::vector<int32_t> tiles_x = xcd_tile_list(gx, p.gemm_cfg_x);
  std::vector<int32_t> tiles_s = xcd_tile_list(gs, p.gemm_cfg_s);
  p.n_tiles_x = (int32_t)(tiles_x.size() / 3);
  p.n_tiles_s = (int32_t)(tiles_s.size() / 3);
  std::vector<RowTile> rt_inv = row_tiles(gv_inv), rt_abi = row_tiles(gv_abi),
                       rt_aib = row_tiles(gv_aib), rt_s = row_tiles(gv_s);
  p.n_rt_inv = (int32_t)rt_inv.size();
  p.n_rt_abi = (int32_t)rt_abi.size();
  p.n_rt_aib = (int32_t)rt_aib.size();
  p.n_rt_s = (int32_t)rt_s.size();

  scdg_status st = SCDG_OK;
  auto chk = [&](scdg_status x) { if (st == SCDG_OK) st = x; };
  chk(upload(p, &p.d_imap, imap));
  chk(upload(p, &p.d_bmap, bmap));
  chk(upload(p, &p.d_cmap, cmap));
  chk(upload(p, &p.d_pull_ptr, pull_ptr));
  chk(upload(p, &p.d_pull_idx, pull_idx));
  chk(upload(p, &p.d_slot_soff, slot_soff));
  chk(upload(p, &p.d_slot_nc, slot_nc));
  chk(upload(p, &p.d_slot_pos, slot_pos));
  chk(upload(p, &p.d_slot_ib, slot_ib));
  chk(upload(p, &p.d_slot_ni, slot_ni));
  chk(upload(p, &p.d_bb_rowptr, bb_rowptr));
  chk(upload(p, &p.d_fold_map, fold_map));
  chk(upload(p, &p.d_rem_rowptr, rem_rowptr));
  chk(upload(p, &p.d_rem_col, rem_col));
  chk(upload(p, &p.d_rem_src, rem_src));
  {
    // transposed remainder: entry k = (row g, column h) becomes (row h, column g)
    std::vector<int64_t> rt_ptr(p.n_bnodes + 1, 0);
    for (int32_t h : rem_col) ++rt_ptr[h + 1];
    for (int64_t g = 0; g < p.n_bnodes; ++g) rt_ptr[g + 1] += rt_ptr[g];
    std::vector<int32_t> rt_col(rem_col.size()), rt_src(rem_col.size());
    std::vector<int64_t> fill(rt_ptr.begin(), rt_ptr.end() - 1);
    for (int64_t g = 0; g < p.n_bnodes; ++g)
      for (int64_t k = rem_rowptr[g]; k < rem_rowptr[g + 1]; ++k) {
        const int64_t at = fill[rem_col[k]]++;
        rt_col[at] = (int32_t)g;
        rt_src[at] = (int32_t)k;
      }
    chk(upload(p, &p.d_remt_rowptr, rt_ptr));
    chk(upload(p, &p.d_remt_col, rt_col));
    chk(upload(p, &p.d_remt_src, rt_src));
    std::vector<RowTile> ct;
    for (int e = 0; e < E; ++e)
      for (int j0 = 0; j0 < p.nc[e]; j0 += 256) ct.push_back(RowTile{e, j0});
    p.n_ct_s = (int32_t)ct.size();
    chk(upload(p, &p.d_ct_s, ct));
  }
  chk(dalloc(p, &p.pc_blk, (size_t)p.n_bnodes * 25));
  chk(upload(p, &p.d_bb_col, bb_col));
  chk(upload(p, &p.d_inv_n, inv_n));
  chk(upload(p, &p.d_inv_off, inv_off));
  {
    // per-element sizes for the block masks of the sparse matrix-free form
    std::vector<int64_t> offib(E), maskoff(E);
    std::vector<int32_t> ri(E), rc(E);
    int64_t mo = 0;
    for (int e = 0; e < E; ++e) {
      offib[e] = p.off_ib[e];
      ri[e] = p.ni[e] / kNvar;
      rc[e] = p.nc[e] / kNvar;
      maskoff[e] = mo;
      mo += (int64_t)ri[e] * rc[e];
    }
    chk(upload(p, &p.d_e_offib, offib));
    chk(upload(p, &p.d_e_maskoff, maskoff));
    chk(upload(p, &p.d_e_ri, ri));
    chk(upload(p, &p.d_e_rc, rc));
  }
  {
    std::vector<int32_t> ord(p.n_elem);
    for (int e = 0; e < p.n_elem; ++e) ord[e] = e;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return p.ni[a] > p.ni[b]; });
    chk(upload(p, &p.d_inv_order, ord));
  }
  chk(dalloc(p, &p.d_info, (size_t)E));
  chk(upload(p, &p.d_gx, gx));
  chk(upload(p, &p.d_gs, gs));
  chk(upload(p, &p.d_tiles_x, tiles_x));
  chk(upload(p, &p.d_tiles_s, tiles_s));
  chk(upload(p, &p.d_gv_inv, gv_inv));
  chk(upload(p, &p.d_gv_abi, gv_abi));
  chk(upload(p, &p.d_gv_aib, gv_aib));
  chk(upload(p, &p.d_gv_s, gv_s));
  chk(upload(p, &p.d_rt_inv, rt_inv));
  chk(upload(p, &p.d_rt_abi, rt_abi));
  chk(upload(p, &p.d_rt_aib, rt_aib));
  chk(upload(p, &p.d_rt_s, rt_s));
  chk(dalloc(p, &p.w_z, (size_t)p.n2));
  chk(dalloc(p, &p.w_t, (size_t)p.off_c[E]));
  chk(dalloc(p, &p.w_bs, (size_t)p.n1));
  chk(dalloc(p, &p.w_qb, (size_t)p.n1));
  chk(dalloc(p, &p.w_r, (size_t)p.n_dof));
  chk(dalloc(p, &p.w_rx, (size_t)p.n1));
  chk(dalloc(p, &p.w_dq, (size_t)p.n_dof));
  chk(dalloc(p, &p.w_vec, (size_t)p.n_dof));
  chk(dalloc(p, &p.gm_w, (size_t)p.n1));
  chk(dalloc(p, &p.gm_z, (size_t)p.n1));
  chk(dalloc(p, &p.diag_s, (size_t)p.n1));
  p.red_blocks = 512;
  chk(dalloc(p, &p.gm_part, (size_t)p.red_blocks * 64));
  chk(dalloc(p, &p.gm_h, (size_t)3 * 64));
  if (st == SCDG_OK) {
    if (hipHostMalloc(reinterpret_cast<void **>(&p.h_pinned), sizeof(double) * 3 * 64) != hipSuccess) {
      p.last_error = "pinned host allocation failed";
      st = SCDG_ERR_NOMEM;
    }
  }
  if (st != SCDG_OK) {
    g_create_error = p.last_error;
    scdg_plan_destroy(pl);
    return st;
  }
  *out = pl;
  return SCDG_OK;
}

scdg_status scdg_set_stream(scdg_plan *pl, void *hip_stream) {
  if (!pl) return SCDG_ERR_ARG;
  pl->p.stream = static_cast<hipStream_t>(hip_stream);
  return SCDG_OK;
}

scdg_status scdg_plan_sizes(const scdg_plan *pl, int64_t *n_dof, int64_t *n1, int64_t *n2,
                            int64_t *n_bnodes) {
  if (!pl) return SCDG_ERR_ARG;
  if (n_dof) *n_dof = pl->p.n_dof;
  if (n1) *n1 = pl->p.n1;
  if (n2) *n2 = pl->p.n2;
  if (n_bnodes) *n_bnodes = pl->p.n_bnodes;
  return SCDG_OK;
}

scdg_status scdg_plan_fold_counts(const scdg_plan *pl, int64_t *n_folded, int64_t *n_remainder) {
  if (!pl) return SCDG_ERR_ARG;
  if (n_folded) *n_folded = pl->p.n_fold;
  if (n_remainder) *n_remainder = pl->p.n_rem;
  return SCDG_OK;
}

scdg_status scdg_assemble(scdg_plan *pl, const double *aii, const double *aib, const double *abi,
                          const double *bb_val, int32_t flags) {
  if (!pl || !aii || !aib || !abi || (pl->p.nnzb > 0 && !bb_val) || (flags != SCDG_COPY && flags != SCDG_BORROW))
    return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (flags == SCDG_COPY) {
    const size_t n_ii = (size_t)p.off_ii[p.n_elem], n_ib = (size_t)p.off_ib[p.n_elem], n_bb = 25 * (size_t)p.nnzb;
    if (!p.own_aii) {
      ST_TRY(dalloc(p, &p.own_aii, std::max<size_t>(1, n_ii)));
      ST_TRY(dalloc(p, &p.own_aib, std::max<size_t>(1, n_ib)));
      ST_TRY(dalloc(p, &p.own_abi, std::max<size_t>(1, n_ib)));
      ST_TRY(dalloc(p, &p.own_bb, std::max<size_t>(1, n_bb)));
    }
    HIP_TRY(hipMemcpyAsync(p.own_aii, aii, sizeof(double) * n_ii, hipMemcpyDeviceToDevice, p.stream));
    HIP_TRY(hipMemcpyAsync(p.own_aib, aib, sizeof(double) * n_ib, hipMemcpyDeviceToDevice, p.stream));
    HIP_TRY(hipMemcpyAsync(p.own_abi, abi, sizeof(double) * n_ib, hipMemcpyDeviceToDevice, p.stream));
    if (n_bb) HIP_TRY(hipMemcpyAsync(p.own_bb, bb_val, sizeof(double) * n_bb, hipMemcpyDeviceToDevice, p.stream));
    aii = p.own_aii;
    aib = p.own_aib;
    abi = p.own_abi;
    bb_val = p.own_bb;
  }
  p.aii = aii;
  p.aib = aib;
  p.abi = abi;
  p.bb_val = bb_val;
  p.state = 1;
  p.dense_factored = false;
  return SCDG_OK;
}

// Work lists and buffers of the blocked inverse: for every outer panel, one
// GEMM W += P R per element whose block has columns outside that panel.
scdg_status prepare_blocked_inverse(Plan &p) {
  const int cfg = kGemm128x128w8;
  if (!p.d_gj_voff) {
    std::vector<int64_t> voff(p.n_elem);
    int64_t acc = 0;
    for (int e = 0; e < p.n_elem; ++e) {
      voff[e] = acc;
      acc += p.ni[e];
    }
    p.sum_ni = acc;
    ST_TRY(upload(p, &p.d_gj_voff, voff));
    ST_TRY(dalloc(p, &p.d_gj_piv, (size_t)std::max<int64_t>(1, acc)));
    ST_TRY(dalloc(p, &p.d_gj_flag, (size_t)std::max<int64_t>(1, acc)));
  }
  const size_t need = sizeof(double) * (size_t)std::max<int64_t>(1, p.sum_ni) * kGjOuter;
  if (need > p.cap_gj) {
    dfree(p.gj_pbuf);
    dfree(p.gj_rbuf);
    p.cap_gj = 0;
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.gj_pbuf), need));
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.gj_rbuf), need));
    p.cap_gj = need;
  }
  if (p.gj_cfg == cfg) return SCDG_OK;
  std::vector<GemmDesc> all;
  std::vector<int32_t> tiles;
  p.gj_desc_off.clear();
  p.gj_tile_off.clear();
  p.gj_ntiles.clear();
  int64_t voff = 0;
  std::vector<int64_t> vo(p.n_elem);
  for (int e = 0; e < p.n_elem; ++e) {
    vo[e] = voff;
    voff += p.ni[e];
  }
  for (int ko = 0; ko < p.max_ni; ko += kGjOuter) {
    std::vector<GemmDesc> step;
    for (int e = 0; e < p.n_elem; ++e) {
      const int n = p.ni[e];
      if (n <= kGjOuter || ko >= n) continue;   // nothing outside the outer panel
      GemmDesc d{};
      d.a_off = vo[e] * kGjOuter;
      d.b_off = vo[e] * kGjOuter;
      d.c_off = p.off_ii[e];
      d.m = n;
      d.n = n;
      d.k = std::min(kGjOuter, n - ko);
      d.lda = kGjOuter;
      d.ldb = n;
      d.ldc = n;
      step.push_back(d);
    }
    std::vector<int32_t> t = xcd_tile_list(step, cfg);
    p.gj_desc_off.push_back((int64_t)all.size());
    p.gj_tile_off.push_back((int64_t)tiles.size() / 3);
    p.gj_ntiles.push_back(step.empty() ? 0 : (int32_t)(t.size() / 3));
    all.insert(all.end(), step.begin(), step.end());
    if (!step.empty()) tiles.insert(tiles.end(), t.begin(), t.end());
  }
  dfree(p.d_gj_desc);
  dfree(p.d_gj_tiles);
  if (all.empty()) all.push_back(GemmDesc{});
  if (tiles.empty()) tiles.assign(3, -1);
  ST_TRY(upload(p, &p.d_gj_desc, all));
  ST_TRY(upload(p, &p.d_gj_tiles, tiles));
  p.gj_cfg = cfg;
  return SCDG_OK;
}

scdg_status scdg_factor(scdg_plan *pl, scdg_precision prec) {
  if (!pl) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 1) {
    p.last_error = "scdg_factor before scdg_assemble";
    return SCDG_ERR_STATE;
  }
  if (prec != SCDG_FP64 && prec != SCDG_FP32) return SCDG_ERR_ARG;
  p.prec = prec;
  if (!gj_supported(p.max_ni, fp32(p))) {
    p.last_error = "interior block too large for the batched inverse";
    return SCDG_ERR_UNSUPPORTED;
  }
  const size_t need = esize(p) * (size_t)p.off_ii[p.n_elem];
  if (need > p.cap_ainv) {
    dfree(p.ainv);
    dfree(p.ainv_work);
    p.cap_ainv = 0;
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.ainv), need));
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.ainv_work), need));
    p.cap_ainv = need;
  }
  const bool res_ok = gj_resident_supported(p.max_ni, fp32(p));
  if (p.inverse_mode == 3 && !res_ok) {
    p.last_error = "interior block too large for the resident-panel inverse";
    return SCDG_ERR_UNSUPPORTED;
  }
  int form = p.inverse_mode;
  if (form == 0) form = res_ok ? 3 : (p.max_ni > kGjAutoBlocked ? 2 : 1);
  if (form == 2) ST_TRY(prepare_blocked_inverse(p));
  {
    PhaseTimer tm(p, SCDG_PHASE_INVERSE);
    if (form == 2)
      HIP_TRY(launch_gj_inverse_blocked(p, p.ainv_work, p.ainv, fp32(p)));
    else if (form == 3)
      HIP_TRY(launch_gj_inverse_resident(p, p.ainv_work, p.ainv, fp32(p)));
    else
      HIP_TRY(launch_gj_inverse(p, p.ainv_work, p.ainv, fp32(p)));
  }
  p.inverse_used = form;
  p.state = 2;
  p.dense_factored = false;
  return SCDG_OK;
}

scdg_status scdg_set_krylov_mode(scdg_plan *pl, int32_t mode) {
  if (!pl || mode < 0 || mode > 2) return SCDG_ERR_ARG;
  pl->p.krylov_mode = mode;
  return SCDG_OK;
}

scdg_status scdg_set_schur_mode(scdg_plan *pl, int32_t mode) {
  if (!pl || mode < 0 || mode > 2) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  if (mode != p.schur_mode) {
    p.schur_mode = mode;
    if (p.state > 2) p.state = 2;   // condense again in the new form
    p.dense_factored = false;
  }
  return SCDG_OK;
}

scdg_status scdg_get_schur_mode(const scdg_plan *pl, int32_t *mode) {
  if (!pl || !mode) return SCDG_ERR_ARG;
  *mode = pl->p.schur_mode;
  return SCDG_OK;
}

scdg_status scdg_set_inverse_mode(scdg_plan *pl, int32_t mode) {
  if (!pl || mode < 0 || mode > 3) return SCDG_ERR_ARG;
  pl->p.inverse_mode = mode;
  return SCDG_OK;
}

scdg_status scdg_get_inverse_mode(const scdg_plan *pl, int32_t *mode_used) {
  if (!pl || !mode_used) return SCDG_ERR_ARG;
  *mode_used = pl->p.inverse_used;
  return SCDG_OK;
}

scdg_status scdg_factor_info(scdg_plan *pl, int64_t *first_bad_elem, int32_t *info) {
  if (!pl) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  if (p.state < 2) return SCDG_ERR_STATE;
  std::vector<int32_t> h(p.n_elem);
  HIP_TRY(hipMemcpyAsync(h.data(), p.d_info, sizeof(int32_t) * p.n_elem, hipMemcpyDeviceToHost, p.stream));
  ST_TRY(sync(p));
  int64_t bad = -1;
  int32_t val = 0;
  for (int e = 0; e < p.n_elem; ++e)
    if (h[e] != 0) {
      bad = e;
      val = h[e];
      break;
    }
  if (first_bad_elem) *first_bad_elem = bad;
  if (info) *info = val;
  return SCDG_OK;
}

scdg_status scdg_condense(scdg_plan *pl) {
  if (!pl) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 2) {
    p.last_error = "scdg_condense before scdg_factor";
    return SCDG_ERR_STATE;
  }
  int64_t bad = -1;
  int32_t info = 0;
  ST_TRY(scdg_factor_info(pl, &bad, &info));
  if (bad >= 0) {
    p.last_error = "singular interior block in element " + std::to_string(bad) + " at step " +
                   std::to_string(info);
    return SCDG_ERR_SINGULAR;
  }
  const int E = p.n_elem;
  const size_t nx = esize(p) * (size_t)p.off_ib[E], ns = esize(p) * (size_t)p.off_cc[E];
  if (nx > p.cap_x) {
    dfree(p.xmat);
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.xmat), nx));
    p.cap_x = nx;
  }
  if (p.schur_mode == 0 && ns > p.cap_s) {   // the matrix-free forms never store T_e
    dfree(p.sloc);
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.sloc), ns));
    p.cap_s = ns;
  }
  const void *aib = p.aib, *abi = p.abi;
  if (fp32(p)) {
    if (!p.aib_lo) ST_TRY(dalloc(p, reinterpret_cast<float **>(&p.aib_lo), (size_t)p.off_ib[E]));
    if (!p.abi_lo) ST_TRY(dalloc(p, reinterpret_cast<float **>(&p.abi_lo), (size_t)p.off_ib[E]));
    HIP_TRY(launch_cast_f64_to_f32(p.aib, static_cast<float *>(p.aib_lo), p.off_ib[E], p.stream));
    HIP_TRY(launch_cast_f64_to_f32(p.abi, static_cast<float *>(p.abi_lo), p.off_ib[E], p.stream));
    aib = p.aib_lo;
    abi = p.abi_lo;
  }
  {
    PhaseTimer tm(p, SCDG_PHASE_GEMM_X);
    HIP_TRY(launch_gemm_batched(p.gemm_cfg_x, p.d_gx, p.d_tiles_x, p.n_tiles_x, p.ainv, aib, p.xmat,
                                1.0, 0.0, fp32(p), p.stream));
  }
  if (p.schur_mode != 0) {
    // matrix-free Schur products: only the Jacobi blocks of S are formed, from
    // diag(A_bb) and the diagonal 5x5 blocks of A_bi(e) X_e
    if (!p.mf_dblk) ST_TRY(dalloc(p, &p.mf_dblk, (size_t)p.off_c[E] / kNvar * 25));
    HIP_TRY(launch_mf_diag_blocks(p, abi, fp32(p)));
    HIP_TRY(launch_precond_setup_mf(p));
    if (fp32(p) && p.nnzb > 0) {
      if (!p.bb_lo) ST_TRY(dalloc(p, &p.bb_lo, (size_t)p.nnzb * 25));
      HIP_TRY(launch_cast_f64_to_f32(p.bb_val, p.bb_lo, (size_t)p.nnzb * 25, p.stream));
    }
    if (p.schur_mode == 2) {
      if (!p.w_z2) ST_TRY(dalloc(p, &p.w_z2, (size_t)std::max<int64_t>(p.n2, 1)));
      ST_TRY(sparse_op_update(p, 0, aib));
      ST_TRY(sparse_op_update(p, 1, abi));
    }
    p.state = 3;
    p.dense_factored = false;
    ST_TRY(sync(p));
    return SCDG_OK;
  }
  {
    PhaseTimer tm(p, SCDG_PHASE_GEMM_S);
    // T_e = F_e - A_bi X_e: the folded A_bb blocks F_e are added in the epilogue
    HIP_TRY(launch_gemm_batched(p.gemm_cfg_s, p.d_gs, p.d_tiles_s, p.n_tiles_s, abi, p.xmat, p.sloc,
                                -1.0, 0.0, fp32(p), p.stream, p.d_fold_map, p.bb_val));
  }
  // the A_bb remainder blocks, copied contiguously in remainder order: every
  // Schur product then streams them instead of gathering from A_bb
  if (p.n_rem > 0) {
    if (!p.rem_val) ST_TRY(dalloc(p, &p.rem_val, (size_t)p.n_rem * 25));
    HIP_TRY(launch_gather_blocks(p.bb_val, p.d_rem_src, p.rem_val, p.n_rem, p.stream));
    if (fp32(p)) {
      if (!p.rem_lo) ST_TRY(dalloc(p, &p.rem_lo, (size_t)p.n_rem * 25));
      HIP_TRY(launch_cast_f64_to_f32(p.rem_val, p.rem_lo, (size_t)p.n_rem * 25, p.stream));
    }
  }
  HIP_TRY(launch_precond_setup(p, p.sloc, fp32(p)));
  p.state = 3;
  p.dense_factored = false;
  ST_TRY(sync(p));
  return SCDG_OK;
}

scdg_status scdg_condense_rhs(scdg_plan *pl, const double *b, double *bs) {
  if (!pl || !b || !bs) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) return SCDG_ERR_STATE;
  return condense_rhs_impl(p, b, bs);
}

scdg_status scdg_schur_apply(scdg_plan *pl, const double *x, double *y) {
  if (!pl || !x || !y) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) return SCDG_ERR_STATE;
  return schur_apply_impl(p, x, y);
}

scdg_status scdg_schur_apply_transpose(scdg_plan *pl, const double *x, double *y) {
  if (!pl || !x || !y || x == y) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3 || p.schur_mode != 0) {
    p.last_error = "scdg_schur_apply_transpose: needs the condensed plan in the assembled form (mode 0)";
    return SCDG_ERR_STATE;
  }
  HIP_TRY(launch_schur_apply_t(p, x, p.w_t, y, fp32(p)));
  return SCDG_OK;
}

scdg_status scdg_guess_schur_loss(scdg_plan *pl, const float *y, const float *t, const double *stats,
                                  double scale, float *dy, double *loss) {
  if (!pl || (!y && !t) || !stats || !loss || !(scale >= 0.0) || !std::isfinite(scale)) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3 || p.schur_mode != 0) {
    p.last_error = "scdg_guess_schur_loss: needs the condensed plan in the assembled form (mode 0)";
    return SCDG_ERR_STATE;
  }
  // e = P_b (rc (y - t)), s = S e, loss = scale s.s; dy = 2 scale rc P_b^T S^T s
  double *e = p.w_bs, *sv = p.w_qb;
  HIP_TRY(launch_guess_err_gather(y, t, stats, p.d_bmap, p.n1, e, p.stream));
  ST_TRY(schur_apply_impl(p, e, sv));
  HIP_TRY(launch_multidot(sv, 0, 1, sv, p.n1, p.gm_part, p.red_blocks, p.gm_h, p.stream));
  HIP_TRY(launch_axpby(1, scale, p.gm_h, 0.0, loss, p.stream));
  if (dy) {
    HIP_TRY(launch_schur_apply_t(p, sv, p.w_t, e, fp32(p)));
    HIP_TRY(launch_guess_grad_scatter(e, stats, p.d_bmap, p.n1, p.n_dof, 2.0 * scale, dy, p.stream));
  }
  return SCDG_OK;
}

scdg_status scdg_solve_condensed(scdg_plan *pl, const double *bs, double *qb, const double *x0,
                                 const scdg_solve_opts *o, scdg_solve_info *info) {
  if (!pl || !bs || !qb) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) return SCDG_ERR_STATE;
  scdg_solve_opts opts{};
  if (o) opts = *o;
  else opts.precond = -1;
  defaults(opts);
  if (opts.restart > 63) return SCDG_ERR_ARG;
  scdg_solve_info inf{};
  inf.rel_res_guess = -1.0;
  inf.rel_res_full = -1.0;
  scdg_status st = solve_condensed_impl(p, bs, qb, x0, opts, inf);
  if (info) *info = finish_info(inf);
  if (st == SCDG_OK) ST_TRY(sync(p));
  return st;
}

scdg_status scdg_backsolve(scdg_plan *pl, const double *b, const double *qb, double *dq) {
  if (!pl || !b || !qb || !dq) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) return SCDG_ERR_STATE;
  return backsolve_impl(p, b, qb, dq);
}

scdg_status scdg_dg_jacobian_blocks(scdg_dg *dg, scdg_plan *pl, const double *q, double inv_dt, double *aii,
                                    double *aib, double *abi, double *bb_val) {
  if (!dg || !pl || !q || !aii || !aib || !abi || (pl->p.nnzb > 0 && !bb_val) || !(inv_dt >= 0.0) ||
      !std::isfinite(inv_dt))
    return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  int k = 0, order = 0;
  bool cart = false;
  dg_jacobian_shape(dg, &k, &order, &cart);
  const int pp = order + 1;
  const int nb = pp * pp * pp - (order - 1) * (order - 1) * (order - 1);
  const int ni = 5 * (order - 1) * (order - 1) * (order - 1);
  if (!cart) {
    p.last_error = "scdg_dg_jacobian_blocks: Cartesian cubes and the Bassi-Rebay 1 flux only";
    return SCDG_ERR_UNSUPPORTED;
  }
  bool same = p.n_elem == k * k * k;
  const int64_t ncn = p.n_elem > 0 ? p.h_c_ptr[1] - p.h_c_ptr[0] : 0;
  for (int e = 0; same && e < p.n_elem; ++e)
    same = p.order[e] == order && p.ni[e] == ni && p.nc[e] == 5 * ncn && p.bnode_off[e] == (int64_t)e * nb &&
           p.h_c_ptr[e + 1] - p.h_c_ptr[e] == ncn;
  if (!same) {
    p.last_error = "scdg_dg_jacobian_blocks: the plan is not the DG object's periodic mesh of uniform order";
    return SCDG_ERR_UNSUPPORTED;
  }
  if (!p.d_jac_cnode) ST_TRY(upload(p, &p.d_jac_cnode, p.h_c_node));
  JacPlanView v;
  v.plan_uid = p.uid;
  v.ni = ni;
  v.nc = (int)(5 * ncn);
  v.ncn = (int)ncn;
  v.nb = nb;
  v.nnzb = p.nnzb;
  v.c_node = p.d_jac_cnode;
  v.bb_rowptr = p.d_bb_rowptr;
  v.bb_col = p.d_bb_col;
  const scdg_status st = dg_jacobian_blocks_on(dg, v, q, inv_dt, aii, aib, abi, bb_val);
  if (st != SCDG_OK) p.last_error = dg_last_error(dg);
  return st;
}

scdg_status scdg_residual(scdg_plan *pl, const double *b, const double *dq, double *r,
                          double *rel2) {
  if (!pl || !b || !dq) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 1) return SCDG_ERR_STATE;
  double *rr = r ? r : p.w_r;
  ST_TRY(residual_impl(p, b, dq, rr));
  if (rel2) {
    double rn, bn;
    ST_TRY(norm2sq(p, rr, p.n_dof, &rn));
    ST_TRY(norm2sq(p, b, p.n_dof, &bn));
    *rel2 = bn > 0 ? std::sqrt(rn / bn) : std::sqrt(rn);
  }
  return SCDG_OK;
}

scdg_status scdg_solve(scdg_plan *pl, const double *b, double *dq, const double *x0,
                       const scdg_solve_opts *o, scdg_solve_info *info) {
  if (!pl || !b || !dq) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) return SCDG_ERR_STATE;
  scdg_solve_opts opts{};
  if (o) opts = *o;
  else opts.precond = -1;
  defaults(opts);
  if (opts.restart > 63) return SCDG_ERR_ARG;
  scdg_solve_info inf{};
  inf.rel_res_guess = -1.0;
  inf.rel_res_full = -1.0;
  double bn2;
  ST_TRY(norm2sq(p, b, p.n_dof, &bn2));
  if (!std::isfinite(bn2)) {
    p.last_error = "non-finite right-hand side";
    if (info) *info = finish_info(inf);
    return SCDG_ERR_NONFINITE;
  }
  const double bnorm = std::sqrt(bn2);
  // sweep 0 solves A dQ = B (from the boundary part of x0 when given); later
  // sweeps solve A d = r with r = B - A dQ in FP64 and add d to dQ.
  const double *rhs = b;
  const double *guess = nullptr;
  if (x0) {
    HIP_TRY(launch_gather(x0, p.d_bmap, p.w_qb, p.n1, p.stream));
    guess = p.w_qb;
  }
  scdg_status st = SCDG_OK;
  double rel = -1.0;
  for (int sweep = 0; sweep < opts.ir_max; ++sweep) {
    double *target = sweep == 0 ? dq : p.w_dq;
    ST_TRY(condense_rhs_impl(p, rhs, p.w_bs));
    scdg_status s1 = solve_condensed_impl(p, p.w_bs, p.w_qb, sweep == 0 ? guess : nullptr, opts, inf);
    if (s1 != SCDG_OK && s1 != SCDG_ERR_NOCONV) {
      if (info) *info = finish_info(inf);
      return s1;
    }
    if (s1 == SCDG_ERR_NOCONV) st = s1;
    ST_TRY(backsolve_impl(p, rhs, p.w_qb, target));
    if (sweep > 0) HIP_TRY(launch_axpby(p.n_dof, 1.0, p.w_dq, 1.0, dq, p.stream));
    inf.ir_sweeps = sweep + 1;
    ST_TRY(residual_impl(p, b, dq, p.w_r));
    double rn2;
    ST_TRY(norm2sq(p, p.w_r, p.n_dof, &rn2));
    rel = bnorm > 0 ? std::sqrt(rn2) / bnorm : std::sqrt(rn2);
    inf.rel_res_full = rel;
    if (!std::isfinite(rel)) {
      p.last_error = "non-finite full-system residual";
      if (info) *info = finish_info(inf);
      return SCDG_ERR_NONFINITE;
    }
    if (rel <= opts.ir_tol || bnorm == 0.0) {
      st = SCDG_OK;
      break;
    }
    // the next sweep's right-hand side is r; copy it because the next
    // residual evaluation overwrites w_r
    HIP_TRY(hipMemcpyAsync(p.w_vec, p.w_r, sizeof(double) * p.n_dof, hipMemcpyDeviceToDevice, p.stream));
    rhs = p.w_vec;
  }
  if (info) *info = finish_info(inf);
  if (st == SCDG_OK && rel > opts.ir_tol) {
    p.last_error = "iterative refinement did not reach ir_tol";
    st = SCDG_ERR_NOCONV;
  }
  ST_TRY(sync(p));
  return st;
}

scdg_status scdg_newton_step(scdg_plan *pl, scdg_dg *dg, const double *q_s, double inv_dt, double *q,
                             const scdg_newton_opts *o, scdg_newton_info *info) {
  if (!pl || !dg || !q_s || !q || q == q_s) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(on_device(p));
  if (p.state < 3) {
    p.last_error = "scdg_newton_step before scdg_condense";
    return SCDG_ERR_STATE;
  }
  if (dg_dof_count(dg) != p.n_dof) {
    p.last_error = "residual object and plan differ in size";
    return SCDG_ERR_ARG;
  }
  scdg_newton_opts opt{};
  if (o) opt = *o;
  else opt.forcing = -1, opt.precond = -1;
  const double newton_tol = opt.newton_tol > 0 ? opt.newton_tol : 1e-8;
  NewtonSetup ns;
  ns.m = opt.restart > 0 ? opt.restart : 30;
  ns.cycles = opt.cycles > 0 ? opt.cycles : 8;
  ns.pmode = opt.precond < 0 ? 1 : std::min(opt.precond, 2);
  ns.lin_tol = opt.lin_tol > 0 ? opt.lin_tol : 1e-10;
  ns.eta_c = (opt.forcing < 0 ? 0.5 : opt.forcing) * newton_tol;
  ns.eta_max = opt.eta_max > 0 ? opt.eta_max : 0.1;
  ns.inv_dt = inv_dt;
  const int max_newton = opt.max_newton > 0 ? opt.max_newton : 10;
  if (ns.m > 63 || ns.cycles > 64 || !std::isfinite(inv_dt)) return SCDG_ERR_ARG;
  ST_TRY(ensure_gmres(p, ns.m));
  ST_TRY(ensure_krylov_state(p, ns.m));
  if (!p.nw_r) ST_TRY(dalloc(p, &p.nw_r, (size_t)p.n_dof));
  if (!p.nw_dq) ST_TRY(dalloc(p, &p.nw_dq, (size_t)p.n_dof));
  if (!p.nw_stat) ST_TRY(dalloc(p, &p.nw_stat, (size_t)8));
  scdg_newton_info inf{};
  // ||R(Q_s)|| (R(Q_s) kept in nw_dq in case the starting state is rejected)
  double r0sq, rsq;
  HIP_TRY(dg_residual_on(dg, q_s, q_s, inv_dt, p.nw_dq, p.stream));
  ST_TRY(norm2sq(p, p.nw_dq, p.n_dof, &r0sq));
  HIP_TRY(dg_residual_on(dg, q, q_s, inv_dt, p.nw_r, p.stream));
  ST_TRY(norm2sq(p, p.nw_r, p.n_dof, &rsq));
  inf.r0 = std::sqrt(r0sq);
  if (!std::isfinite(inf.r0)) {
    p.last_error = "non-finite residual at Q_s";
    if (info) *info = inf;
    return SCDG_ERR_NONFINITE;
  }
  if (!(rsq <= r0sq)) {
    inf.start_rejected = 1;
    HIP_TRY(hipMemcpyAsync(q, q_s, sizeof(double) * p.n_dof, hipMemcpyDeviceToDevice, p.stream));
    HIP_TRY(hipMemcpyAsync(p.nw_r, p.nw_dq, sizeof(double) * p.n_dof, hipMemcpyDeviceToDevice, p.stream));
    rsq = r0sq;
  }
  double rn = std::sqrt(rsq);
  const double target = newton_tol * inf.r0;
  double *stage = p.h_pinned + 160;
  stage[0] = rsq;
  stage[1] = 0.0;
  stage[2] = inf.r0;
  stage[3] = 0.0;
  HIP_TRY(hipMemcpyAsync(p.nw_stat, stage, sizeof(double) * 4, hipMemcpyHostToDevice, p.stream));
  ST_TRY(newton_graphs(p, dg, q_s, q, ns));
  int32_t kst[8];
  while (rn > target && inf.newton < max_newton) {
    HIP_TRY(hipGraphLaunch(p.nw_exec[0], p.stream));
    // restart cycles until the device flag reports the solve finished
    for (int c = 0; c < ns.cycles; ++c) {
      HIP_TRY(hipGraphLaunch(p.nw_exec[1], p.stream));
      HIP_TRY(hipMemcpyAsync(stage + 4, p.kr_st, sizeof(int32_t) * 8, hipMemcpyDeviceToHost, p.stream));
      ST_TRY(sync(p));
      std::memcpy(kst, stage + 4, sizeof(kst));
      if (kst[3]) break;
    }
    HIP_TRY(hipGraphLaunch(p.nw_exec[2], p.stream));
    HIP_TRY(hipMemcpyAsync(stage, p.nw_stat, sizeof(double), hipMemcpyDeviceToHost, p.stream));
    ST_TRY(sync(p));
    rn = std::sqrt(stage[0]);
    if (inf.newton == 0) inf.first_gmres = kst[4];
    inf.gmres += kst[4];
    inf.lin_unconverged += kst[5] ? 0 : 1;
    ++inf.newton;
    if (!std::isfinite(rn)) {
      p.last_error = "non-finite residual in a Newton iteration";
      inf.rel_res = rn;
      if (info) *info = inf;
      return SCDG_ERR_NONFINITE;
    }
  }
  inf.rel_res = inf.r0 > 0 ? rn / inf.r0 : rn;
  inf.converged = rn <= target ? 1 : 0;
  if (info) *info = inf;
  if (!inf.converged) {
    p.last_error = "Newton iterations did not reach newton_tol";
    return SCDG_ERR_NOCONV;
  }
  return SCDG_OK;
}

scdg_status scdg_enable_timing(scdg_plan *pl, int on) {
  if (!pl) return SCDG_ERR_ARG;
  pl->p.timing = on != 0;
  return SCDG_OK;
}

scdg_status scdg_phase_times(scdg_plan *pl, double *ms, int32_t *count, int32_t n) {
  if (!pl || !ms || !count || n < 0 || n > SCDG_PHASE_COUNT) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  ST_TRY(sync(p));
  for (int i = 0; i < n; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  for (auto &u : p.ev_used) {
    float t = 0.f;
    if (u.first < n && hipEventElapsedTime(&t, u.second.first, u.second.second) == hipSuccess) {
      ms[u.first] += t;
      count[u.first] += 1;
    }
    p.ev_pool.push_back(u.second);
  }
  p.ev_used.clear();
  return SCDG_OK;
}

namespace {

scdg_status set_tiles(Plan &p, bool for_s, int cfg) {
  std::vector<int32_t> tiles = xcd_tile_list(for_s ? p.gs_host : p.gx_host, cfg);
  if (for_s) {
    ST_TRY(upload(p, &p.d_tiles_s, tiles));
    p.n_tiles_s = (int32_t)(tiles.size() / 3);
    p.gemm_cfg_s = cfg;
  } else {
    ST_TRY(upload(p, &p.d_tiles_x, tiles));
    p.n_tiles_x = (int32_t)(tiles.size() / 3);
    p.gemm_cfg_x = cfg;
  }
  return SCDG_OK;
}

}  // namespace

scdg_status scdg_set_gemm_config(scdg_plan *pl, int32_t cfg_x, int32_t cfg_s) {
  if (!pl || cfg_x < 0 || cfg_x >= kGemmConfigs || cfg_s < 0 || cfg_s >= kGemmConfigs)
    return SCDG_ERR_ARG;
  Plan &p = pl->p;
  HIP_TRY(hipStreamSynchronize(p.stream));
  ST_TRY(set_tiles(p, false, cfg_x));
  ST_TRY(set_tiles(p, true, cfg_s));
  if (p.state >= 3) p.state = 2;   // the Schur blocks must be recomputed
  return SCDG_OK;
}

scdg_status scdg_get_gemm_config(const scdg_plan *pl, int32_t *cfg_x, int32_t *cfg_s) {
  if (!pl) return SCDG_ERR_ARG;
  if (cfg_x) *cfg_x = pl->p.gemm_cfg_x;
  if (cfg_s) *cfg_s = pl->p.gemm_cfg_s;
  return SCDG_OK;
}

scdg_status scdg_autotune(scdg_plan *pl, double *ms_x, double *ms_s, int32_t n) {
  if (!pl) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  if (p.state < 2) {
    p.last_error = "scdg_autotune needs scdg_factor first";
    return SCDG_ERR_STATE;
  }
  const int E = p.n_elem;
  const size_t nx = esize(p) * (size_t)p.off_ib[E], ns = esize(p) * (size_t)p.off_cc[E];
  if (nx > p.cap_x) {
    dfree(p.xmat);
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.xmat), nx));
    p.cap_x = nx;
  }
  if (ns > p.cap_s) {
    dfree(p.sloc);
    ST_TRY(dalloc(p, reinterpret_cast<char **>(&p.sloc), ns));
    p.cap_s = ns;
  }
  const void *aib = p.aib, *abi = p.abi;
  if (fp32(p)) {
    if (!p.aib_lo) ST_TRY(dalloc(p, reinterpret_cast<float **>(&p.aib_lo), (size_t)p.off_ib[E]));
    if (!p.abi_lo) ST_TRY(dalloc(p, reinterpret_cast<float **>(&p.abi_lo), (size_t)p.off_ib[E]));
    HIP_TRY(launch_cast_f64_to_f32(p.aib, static_cast<float *>(p.aib_lo), p.off_ib[E], p.stream));
    HIP_TRY(launch_cast_f64_to_f32(p.abi, static_cast<float *>(p.abi_lo), p.off_ib[E], p.stream));
    aib = p.aib_lo;
    abi = p.abi_lo;
  }
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  int best[2] = {p.gemm_cfg_x, p.gemm_cfg_s};
  for (int which = 0; which < 2; ++which) {
    double best_ms = 1e30;
    for (int cfg = 0; cfg < kGemmConfigs; ++cfg) {
      int bm, bn;
      gemm_tile_shape(cfg, &bm, &bn);
      const int rows = which == 0 ? p.max_ni : p.max_nc;
      double ms = -1.0;
      if (bm <= 2 * rows) {   // skip tiles far taller than the problem
        ST_TRY(set_tiles(p, which == 1, cfg));
        float t = 0.f, tmin = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          HIP_TRY(hipEventRecord(t0, p.stream));
          if (which == 0)
            HIP_TRY(launch_gemm_batched(cfg, p.d_gx, p.d_tiles_x, p.n_tiles_x, p.ainv, aib, p.xmat,
                                        1.0, 0.0, fp32(p), p.stream));
          else
            HIP_TRY(launch_gemm_batched(cfg, p.d_gs, p.d_tiles_s, p.n_tiles_s, abi, p.xmat, p.sloc,
                                        -1.0, 0.0, fp32(p), p.stream, p.d_fold_map, p.bb_val));
          HIP_TRY(hipEventRecord(t1, p.stream));
          HIP_TRY(hipEventSynchronize(t1));
          HIP_TRY(hipEventElapsedTime(&t, t0, t1));
          if (rep > 0) tmin = std::min(tmin, t);
        }
        ms = tmin;
        if (ms < best_ms) {
          best_ms = ms;
          best[which] = cfg;
        }
      }
      double *dst = which == 0 ? ms_x : ms_s;
      if (dst && cfg < n) dst[cfg] = ms;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  ST_TRY(set_tiles(p, false, best[0]));
  ST_TRY(set_tiles(p, true, best[1]));
  p.state = 2;   // the tuning runs overwrote X and the Schur blocks
  return SCDG_OK;
}

scdg_status scdg_export(scdg_plan *pl, int what, void *dst, size_t dst_bytes) {
  if (!pl || !dst) return SCDG_ERR_ARG;
  Plan &p = pl->p;
  const void *src = nullptr;
  size_t bytes = 0;
  if (what == SCDG_EXPORT_AII_INV) {
    if (p.state < 2) return SCDG_ERR_STATE;
    src = p.ainv;
    bytes = esize(p) * (size_t)p.off_ii[p.n_elem];
  } else if (what == SCDG_EXPORT_SCHUR) {
    if (p.state < 3 || p.schur_mode != 0) return SCDG_ERR_STATE;
    src = p.sloc;
    bytes = esize(p) * (size_t)p.off_cc[p.n_elem];
  } else if (what == SCDG_EXPORT_X) {
    if (p.state < 3) return SCDG_ERR_STATE;
    src = p.xmat;
    bytes = esize(p) * (size_t)p.off_ib[p.n_elem];
  } else {
    return SCDG_ERR_ARG;
  }
  if (dst_bytes < bytes) return SCDG_ERR_ARG;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, p.stream));
  ST_TRY(sync(p));
  return SCDG_OK;
}

}  // extern "C"
