// Memory-bound kernels of the condensed solve: batched element GEMVs with
// coalesced gathers of the DOFs they read, the (remainder of the) A_bb BSR
// product fused with the "pull" reduction of element contributions, the Jacobi
// preconditioners, and the Krylov vector operations (deterministic two-stage
// multi-dot for Gram-Schmidt, multi-AXPY, scaling).  All vectors are FP64; element matrices may be FP64 or
// FP32 (accumulation is always FP64).
#include <algorithm>

#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerTile = 64;
constexpr int kRowsPerWave = kRowsPerTile / (kThreads / 64);   // 16
constexpr int kRowBatch = 8;                                    // rows streamed together

template <typename TM>
struct Vec;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <>
struct Vec<double> {
  static constexpr int W = 2;
  using V = dvec2;
  static __device__ __forceinline__ void get(const V &v, double *o) {
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct Vec<float> {
  static constexpr int W = 4;
  using V = fvec4;
  static __device__ __forceinline__ void get(const V &v, double *o) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};

// ---------------------------------------------------------------- GEMV
// One workgroup = 64 rows of one element matrix.  The element's input vector is
// gathered once into LDS; each wave streams 16 rows, eight at a time, with
// lanes striding along the rows in 16-byte vectors (coalesced), and reduces
// with cross-lane adds.  Rows whose length or base is not a multiple of the
// vector width take the scalar path.
template <typename TM>
__device__ __forceinline__ void gemv_tile(int tile, const GemvDesc *__restrict__ desc,
                                          const RowTile *__restrict__ tiles, const TM *__restrict__ mat,
                                          const double *__restrict__ x, const int32_t *__restrict__ xmap,
                                          double *__restrict__ y, const int32_t *__restrict__ omap, double alpha,
                                          double beta, const double *__restrict__ y0) {
  using VT = Vec<TM>;
  constexpr int W = VT::W;
  extern __shared__ double xs[];
  const RowTile t = tiles[tile];
  const GemvDesc d = desc[t.prob];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = tid; c < d.cols; c += kThreads) xs[c] = xmap ? x[xmap[d.x_off + c]] : x[d.x_off + c];
  __syncthreads();
  const TM *__restrict__ base = mat + d.m_off;
  const int r_begin = t.row0 + wid * kRowsPerWave;
  const int r_end = min(d.rows, r_begin + kRowsPerWave);
  const bool vec_ok = (d.cols % W) == 0 && (d.m_off % W) == 0;
  const int nvec = d.cols / W;
  for (int r = r_begin; r < r_end; r += kRowBatch) {
    double s[kRowBatch];
#pragma unroll
    for (int q = 0; q < kRowBatch; ++q) s[q] = 0.0;
    if (vec_ok) {
      const typename VT::V *rows[kRowBatch];
#pragma unroll
      for (int q = 0; q < kRowBatch; ++q)
        rows[q] = reinterpret_cast<const typename VT::V *>(base + (int64_t)min(r + q, r_end - 1) * d.cols);
      for (int c = lane; c < nvec; c += 64) {
        double xv[W];
#pragma unroll
        for (int u = 0; u < W; ++u) xv[u] = xs[c * W + u];
        typename VT::V m[kRowBatch];
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q) m[q] = __builtin_nontemporal_load(&rows[q][c]);
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q) {
          double mv[W];
          VT::get(m[q], mv);
#pragma unroll
          for (int u = 0; u < W; ++u) s[q] += mv[u] * xv[u];
        }
      }
    } else {
      const TM *rows[kRowBatch];
#pragma unroll
      for (int q = 0; q < kRowBatch; ++q) rows[q] = base + (int64_t)min(r + q, r_end - 1) * d.cols;
      for (int c = lane; c < d.cols; c += 64) {
        const double xv = xs[c];
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q) s[q] += (double)rows[q][c] * xv;
      }
    }
#pragma unroll
    for (int q = 0; q < kRowBatch; ++q) s[q] = wave_sum(s[q]);
    if (lane < kRowBatch && r + lane < r_end) {
      double v = s[0];
#pragma unroll
      for (int q = 1; q < kRowBatch; ++q)
        if (lane == q) v = s[q];
      const int yi = d.y_off + r + lane;
      v *= alpha;
      if (beta != 0.0) v += beta * y0[yi];
      y[omap ? omap[yi] : yi] = v;
    }
  }
}

template <typename TM>
__global__ __launch_bounds__(kThreads) void gemv_batched_kernel(
    const GemvDesc *__restrict__ desc, const RowTile *__restrict__ tiles, const TM *__restrict__ mat,
    const double *__restrict__ x, const int32_t *__restrict__ xmap, double *__restrict__ y,
    const int32_t *__restrict__ omap, double alpha, double beta, const double *__restrict__ y0,
    const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  gemv_tile<TM>(blockIdx.x, desc, tiles, mat, x, xmap, y, omap, alpha, beta, y0);
}

// ---------------------------------------------------- BSR product + pull
// One wave per boundary node g (5 output rows).  Lanes 0..59 cover 12 blocks of
// row g at a time, lane l taking row (l % 5) of block (l / 5); each lane reads
// 5 contiguous values, so a wave reads 12 whole blocks (2400 bytes) per step,
// two steps per loop trip.  The pull of element contributions (lanes 0..4) is
// loaded before the block loop so its dependent loads overlap it, and the 12
// partial sums of each output row meet through cross-lane adds (lanes l, l+5,
// ..., l+55 hold row l % 5): no LDS and no workgroup barrier.  The block
// values are FP64, or an FP32 copy inside the products of the FP32 forms
// (accumulation in FP64 either way).
template <typename TV, bool TRANS>
__global__ __launch_bounds__(kThreads) void bsr_pull_kernel_impl(
    int64_t n_bnodes, double c0, const double *__restrict__ src0, const int32_t *__restrict__ map0,
    double c1, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ src_idx, const TV *__restrict__ val,
    const double *__restrict__ x, double c2, const int32_t *__restrict__ pull_ptr,
    const int32_t *__restrict__ pull_idx, const double *__restrict__ t, double *__restrict__ out,
    const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (g >= n_bnodes) return;   // whole waves leave together: no barrier below
  double p = 0.0, o0 = 0.0;
  if (lane < 5) {
    const int64_t j = 5 * g + lane;
    if (c2 != 0.0)
      for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q) p += t[5 * (int64_t)pull_idx[q] + lane];
    if (c0 != 0.0) o0 = src0[map0 ? map0[j] : j];
  }
  double s = 0.0;
  const int v = lane % 5, bq = lane / 5;
  // row v of a stored block, or of its transpose (column v)
  constexpr int SW = TRANS ? 5 : 1;
  const int ro = TRANS ? v : v * 5;
  if (c1 != 0.0 && lane < 60) {
    const int64_t b0 = rowptr[g], b1 = rowptr[g + 1];
    double s2 = 0.0;
    int64_t blk = b0 + bq;
    for (; blk + 12 < b1; blk += 24) {
      const int64_t va = src_idx ? (int64_t)src_idx[blk] : blk;
      const int64_t vb = src_idx ? (int64_t)src_idx[blk + 12] : blk + 12;
      const TV *ra = val + va * 25 + ro, *rb = val + vb * 25 + ro;
      const double *xa = x + (int64_t)col[blk] * 5, *xb = x + (int64_t)col[blk + 12] * 5;
      double ma[5], mb[5], ya[5], yb[5];
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        ma[w] = (double)ra[w * SW];
        mb[w] = (double)rb[w * SW];
        ya[w] = xa[w];
        yb[w] = xb[w];
      }
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        s += ma[w] * ya[w];
        s2 += mb[w] * yb[w];
      }
    }
    if (blk < b1) {
      const int64_t va = src_idx ? (int64_t)src_idx[blk] : blk;
      const TV *ra = val + va * 25 + ro;
      const double *xa = x + (int64_t)col[blk] * 5;
#pragma unroll
      for (int w = 0; w < 5; ++w) s += (double)ra[w * SW] * xa[w];
    }
    s += s2;
  }
  // row sums: lanes l < 30 add lane l + 30, l < 15 add l + 15, then l < 5 add l + 5 and l + 10
  s += __shfl_down(s, 30);
  s += __shfl_down(s, 15);
  const double s5 = __shfl_down(s, 5), s10 = __shfl_down(s, 10);
  if (lane < 5) {
    double o = c1 * (s + s5 + s10);
    if (c0 != 0.0) o += c0 * o0;
    if (c2 != 0.0) o += c2 * p;
    out[5 * g + lane] = o;
  }
}

// y[5 g + v] = sum over the BSR blocks of row g of (block x), one wave per
// boundary node g, laid out as in bsr_pull_kernel (12 blocks per step, two
// steps per trip, cross-lane row sums).
template <typename TV>
__device__ __forceinline__ void bsr_rows_wave(int64_t g, const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col, const TV *__restrict__ val,
                                              const double *__restrict__ x, double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  const int v = lane % 5, bq = lane / 5;
  if (lane < 60) {
    const int64_t b0 = rowptr[g], b1 = rowptr[g + 1];
    double s2 = 0.0;
    int64_t blk = b0 + bq;
    for (; blk + 12 < b1; blk += 24) {
      const TV *ra = val + blk * 25 + v * 5, *rb = val + (blk + 12) * 25 + v * 5;
      const double *xa = x + (int64_t)col[blk] * 5, *xb = x + (int64_t)col[blk + 12] * 5;
      double ma[5], mb[5], ya[5], yb[5];
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        ma[w] = (double)ra[w];
        mb[w] = (double)rb[w];
        ya[w] = xa[w];
        yb[w] = xb[w];
      }
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        s += ma[w] * ya[w];
        s2 += mb[w] * yb[w];
      }
    }
    if (blk < b1) {
      const TV *ra = val + blk * 25 + v * 5;
      const double *xa = x + (int64_t)col[blk] * 5;
#pragma unroll
      for (int w = 0; w < 5; ++w) s += (double)ra[w] * xa[w];
    }
    s += s2;
  }
  s += __shfl_down(s, 30);
  s += __shfl_down(s, 15);
  const double s5 = __shfl_down(s, 5), s10 = __shfl_down(s, 10);
  if (lane < 5) y[5 * g + lane] = s + s5 + s10;
}

// The assembled Schur product's two streams in one launch: the element-block
// GEMV tiles (t = T_e x[C_e], HBM-bound) and the rows of the A_bb remainder
// (rx = R x, bound by dependent-load latency: about two dozen blocks per row
// behind the column-index loads) interleaved in one grid, every `ratio`-th
// workgroup a GEMV tile (ratio odd, so tiles dealt to one XCD stay together),
// so that the remainder's latency hides behind the streaming.  A pull then
// adds the element contributions to rx.
template <typename TM, typename TV>
__global__ __launch_bounds__(kThreads) void schur_gemv_rem_kernel(
    const GemvDesc *__restrict__ desc, const RowTile *__restrict__ tiles, int32_t n_tiles, const TM *__restrict__ mat,
    const double *__restrict__ x, const int32_t *__restrict__ xmap, double *__restrict__ t, int64_t ratio,
    int64_t n_bnodes, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, double *__restrict__ rx, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  const int64_t b = blockIdx.x, grp = b / ratio, pos = b % ratio;
  if (pos == 0 && grp < n_tiles) {
    gemv_tile<TM>((int)grp, desc, tiles, mat, x, xmap, t, nullptr, 1.0, 0.0, nullptr);
    return;
  }
  const int64_t j = grp < n_tiles ? b - (grp + 1) : b - n_tiles;     // remainder workgroup index
  const int64_t g = j * (kThreads / 64) + (threadIdx.x >> 6);
  if (g >= n_bnodes) return;
  bsr_rows_wave<TV>(g, rowptr, col, val, x, rx);
}

// 5x5 inverse by Gauss-Jordan with partial pivoting, in registers
__device__ void inv5(const double a[25], double out[25]) {
  double m[5][10];
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c < 10; ++c) m[r][c] = c < 5 ? a[r * 5 + c] : (c - 5 == r ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int p = k;
#pragma unroll
    for (int r = k + 1; r < 5; ++r)
      if (fabs(m[r][k]) > fabs(m[p][k])) p = r;
#pragma unroll
    for (int r = k + 1; r < 5; ++r)
      if (r == p)
#pragma unroll
        for (int c = 0; c < 10; ++c) {
          const double tmp = m[k][c];
          m[k][c] = m[r][c];
          m[r][c] = tmp;
        }
    double d = m[k][k];
    if (!(d != 0.0) || !isfinite(d)) d = 1.0;
    const double id = 1.0 / d;
#pragma unroll
    for (int c = 0; c < 10; ++c) m[k][c] *= id;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (r == k) continue;
      const double f = m[r][k];
#pragma unroll
      for (int c = 0; c < 10; ++c) m[r][c] -= f * m[k][c];
    }
  }
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) out[r * 5 + c] = m[r][c + 5];
}

// D_g = remainder A_bb(g, g) + sum over elements containing g of T_e's diagonal block
template <typename TM>
__global__ void precond_setup_kernel(int64_t n_bnodes, const int64_t *__restrict__ rem_rowptr,
                                     const int32_t *__restrict__ rem_col,
                                     const int32_t *__restrict__ rem_src,
                                     const double *__restrict__ val,
                                     const int32_t *__restrict__ pull_ptr,
                                     const int32_t *__restrict__ pull_idx,
                                     const int64_t *__restrict__ slot_soff,
                                     const int32_t *__restrict__ slot_nc,
                                     const int32_t *__restrict__ slot_pos, const TM *__restrict__ t,
                                     double *__restrict__ pc_blk, double *__restrict__ diag_inv) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_bnodes) return;
  double a[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) a[k] = 0.0;
  for (int64_t b = rem_rowptr[g]; b < rem_rowptr[g + 1]; ++b)
    if (rem_col[b] == g)
#pragma unroll
      for (int k = 0; k < 25; ++k) a[k] += val[(int64_t)rem_src[b] * 25 + k];
  for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q) {
    const int s = pull_idx[q];
    const int64_t base = slot_soff[s] + (int64_t)(5 * slot_pos[s]) * slot_nc[s] + 5 * slot_pos[s];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int w = 0; w < 5; ++w) a[v * 5 + w] += (double)t[base + (int64_t)v * slot_nc[s] + w];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) diag_inv[5 * g + v] = 1.0 / a[v * 5 + v];
  double inv[25];
  inv5(a, inv);
#pragma unroll
  for (int k = 0; k < 25; ++k) pc_blk[g * 25 + k] = inv[k];
}

// Matrix-free mode: the diagonal 5x5 block of A_bi(e) X_e at every slot (rows
// 5 pos .. 5 pos + 4 of A_bi, columns 5 pos .. 5 pos + 4 of X), one wave per
// slot with the lanes striding over the interior index k.
template <typename TM>
__global__ __launch_bounds__(kThreads) void mf_diag_blocks_kernel(
    int64_t n_slots, const int64_t *__restrict__ slot_ib, const int32_t *__restrict__ slot_ni,
    const int32_t *__restrict__ slot_nc, const int32_t *__restrict__ slot_pos, const TM *__restrict__ abi,
    const TM *__restrict__ xmat, double *__restrict__ dblk) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (s >= n_slots) return;   // whole waves leave together
  const int64_t ib = slot_ib[s];
  const int ni = slot_ni[s], nc = slot_nc[s], pos = slot_pos[s];
  const TM *a = abi + ib + (int64_t)(5 * pos) * ni;
  const TM *x = xmat + ib + 5 * pos;
  double acc[25];
#pragma unroll
  for (int q = 0; q < 25; ++q) acc[q] = 0.0;
  for (int k = lane; k < ni; k += 64) {
    double av[5], xv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) av[v] = (double)a[(int64_t)v * ni + k];
#pragma unroll
    for (int w = 0; w < 5; ++w) xv[w] = (double)x[(int64_t)k * nc + w];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int w = 0; w < 5; ++w) acc[v * 5 + w] += av[v] * xv[w];
  }
#pragma unroll
  for (int q = 0; q < 25; ++q) acc[q] = wave_sum(acc[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 25; ++q) dblk[s * 25 + q] = acc[q];
}

// Matrix-free mode: diagonal block of S at node g = A_bb(g, g) minus the
// pulled diagonal blocks of A_bi(e) X_e; point and 5x5 block Jacobi from it.
__global__ void precond_setup_mf_kernel(int64_t n_bnodes, const int64_t *__restrict__ bb_rowptr,
                                        const int32_t *__restrict__ bb_col, const double *__restrict__ val,
                                        const int32_t *__restrict__ pull_ptr,
                                        const int32_t *__restrict__ pull_idx, const double *__restrict__ dblk,
                                        double *__restrict__ pc_blk, double *__restrict__ diag_inv) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_bnodes) return;
  double a[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) a[k] = 0.0;
  for (int64_t b = bb_rowptr[g]; b < bb_rowptr[g + 1]; ++b)
    if (bb_col[b] == g)
#pragma unroll
      for (int k = 0; k < 25; ++k) a[k] += val[b * 25 + k];
  for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q) {
    const int64_t s = pull_idx[q];
#pragma unroll
    for (int k = 0; k < 25; ++k) a[k] -= dblk[s * 25 + k];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) diag_inv[5 * g + v] = 1.0 / a[v * 5 + v];
  double inv[25];
  inv5(a, inv);
#pragma unroll
  for (int k = 0; k < 25; ++k) pc_blk[g * 25 + k] = inv[k];
}

// ------------------------------------------ block-sparse element products
// Nonzero 5x5 blocks of row-major element matrices (5 R rows x 5 C columns,
// element after element): mask[mask_off[e] + rb C + cb] = 1 when an entry of
// block (rb, cb) is nonzero.  blockIdx.y is the element; consecutive threads
// take consecutive blocks of a block row, so each of the 25 loads reads
// neighbouring 40-byte segments.
__global__ void block_mask_kernel(const double *__restrict__ mat, const int64_t *__restrict__ m_off,
                                  const int32_t *__restrict__ rb_n, const int32_t *__restrict__ cb_n,
                                  const int64_t *__restrict__ mask_off, uint8_t *__restrict__ mask) {
  const int e = blockIdx.y;
  const int cn = cb_n[e];
  const int64_t nb = (int64_t)rb_n[e] * cn;
  const int64_t ld = 5 * (int64_t)cn;
  const double *a = mat + m_off[e];
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rb = b / cn, cb = b % cn;
    const double *blk = a + 5 * rb * ld + 5 * cb;
    bool nz = false;
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int w = 0; w < 5; ++w) nz = nz || blk[v * ld + w] != 0.0;
    mask[mask_off[e] + b] = nz ? 1 : 0;
  }
}

// flag[0] = 1 when the two masks differ anywhere (every writer stores 1)
__global__ void mask_diff_kernel(const uint8_t *__restrict__ a, const uint8_t *__restrict__ b, int64_t n,
                                 int32_t *__restrict__ flag) {
  bool diff = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    diff = diff || a[i] != b[i];
  if (diff) flag[0] = 1;
}

// dst[25 b + 5 v + w] = src[src_off[b] + v ld[b] + w]: the listed 5x5 blocks,
// compacted in list order
template <typename TM>
__global__ void gather_blocks_ld_kernel(const TM *__restrict__ src, const int64_t *__restrict__ src_off,
                                        const int32_t *__restrict__ ld, int64_t n, TM *__restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * 25;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / 25;
    const int k = (int)(i % 25);
    dst[i] = src[src_off[b] + (int64_t)(k / 5) * ld[b] + k % 5];
  }
}

// y[ybase[r] + v] = sum over the blocks b of block row r of
// val[b][v][w] x[5 xnode[b] + w]: one wave per block row, lanes as in the
// BSR product below (12 blocks per step, two steps per trip, cross-lane sums).
template <typename TM>
__global__ __launch_bounds__(kThreads) void bsr5_rows_kernel(
    int64_t n_rows, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ xnode,
    const TM *__restrict__ val, const double *__restrict__ x, const int64_t *__restrict__ ybase,
    double *__restrict__ y, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (r >= n_rows) return;   // whole waves leave together
  const int v = lane % 5, bq = lane / 5;
  double s = 0.0;
  if (lane < 60) {
    const int64_t b0 = rowptr[r], b1 = rowptr[r + 1];
    double s2 = 0.0;
    int64_t blk = b0 + bq;
    for (; blk + 12 < b1; blk += 24) {
      const TM *ra = val + blk * 25 + v * 5, *rb = val + (blk + 12) * 25 + v * 5;
      const double *xa = x + (int64_t)xnode[blk] * 5, *xb = x + (int64_t)xnode[blk + 12] * 5;
      double ma[5], mb[5], ya[5], yb[5];
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        ma[w] = (double)ra[w];
        mb[w] = (double)rb[w];
        ya[w] = xa[w];
        yb[w] = xb[w];
      }
#pragma unroll
      for (int w = 0; w < 5; ++w) {
        s += ma[w] * ya[w];
        s2 += mb[w] * yb[w];
      }
    }
    if (blk < b1) {
      const TM *ra = val + blk * 25 + v * 5;
      const double *xa = x + (int64_t)xnode[blk] * 5;
#pragma unroll
      for (int w = 0; w < 5; ++w) s += (double)ra[w] * xa[w];
    }
    s += s2;
  }
  s += __shfl_down(s, 30);
  s += __shfl_down(s, 15);
  const double s5 = __shfl_down(s, 5), s10 = __shfl_down(s, 10);
  if (lane < 5) y[ybase[r] + lane] = s + s5 + s10;
}

__global__ void precond_apply_kernel(int mode, int64_t n_bnodes, const double *__restrict__ diag_inv,
                                     const double *__restrict__ pc_blk,
                                     const double *__restrict__ x, double *__restrict__ y, double a,
                                     const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= 5 * n_bnodes) return;
  double v;
  if (mode == 2) {
    const int64_t g = j / 5;
    const int r = (int)(j % 5);
    const double *m = pc_blk + g * 25 + r * 5;
    const double *xv = x + 5 * g;
    v = m[0] * xv[0] + m[1] * xv[1] + m[2] * xv[2] + m[3] * xv[3] + m[4] * xv[4];
  } else if (mode == 1) {
    v = diag_inv[j] * x[j];
  } else {
    v = x[j];
  }
  y[j] = a * v;
}

// ------------------------------------------------------------ utilities
__global__ void gather_kernel(const double *__restrict__ src, const int32_t *__restrict__ map,
                              double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[map[i]];
}

__global__ void gather_blocks_kernel(const double *__restrict__ src, const int32_t *__restrict__ idx,
                                     double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * 25;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[(int64_t)idx[i / 25] * 25 + i % 25];
}

__global__ void scatter_kernel(const double *__restrict__ src, const int32_t *__restrict__ map,
                               double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[map[i]] = src[i];
}

// Boundary part of a predicted increment's error in natural units: e[k] =
// rc_v (y_i - t_i) for the natural DOF i = map[k] of boundary slot k, with v = i
// mod 5 the conserved variable and rc_v = stats[15 + v] the scale the network's
// outputs and targets were normalised by; a missing y or t counts as zero.
__global__ void guess_err_gather_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                        const double *__restrict__ stats, const int32_t *__restrict__ map,
                                        int64_t n, double *__restrict__ e) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = map[k];
    const double yi = y ? (double)y[i] : 0.0, ti = t ? (double)t[i] : 0.0;
    e[k] = stats[15 + i % 5] * (yi - ti);
  }
}

// dy[map[k]] = a rc_v g[k] (the chain rule through e = rc (y - t)); the caller
// zeroes dy first, so interior DOFs keep a zero gradient
__global__ void guess_grad_scatter_kernel(const double *__restrict__ g, const double *__restrict__ stats,
                                          const int32_t *__restrict__ map, int64_t n, double a,
                                          float *__restrict__ dy) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = map[k];
    dy[i] = (float)(a * stats[15 + i % 5] * g[k]);
  }
}

__global__ void fill_zero_f32_kernel(float *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.f;
}

__global__ void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                             double *__restrict__ y, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

// dst[map[i]] = a * x[map[i]] + b * yin[i]
__global__ void scatter_axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                                     const double *__restrict__ yin, const int32_t *__restrict__ map,
                                     double *__restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = map[i];
    dst[j] = a * x[j] + b * yin[i];
  }
}

__global__ void fill_kernel(double *__restrict__ y, int64_t n, double v, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

__global__ void diag_scale_kernel(const double *__restrict__ x, const double *__restrict__ dinv,
                                  double *__restrict__ y, int64_t n, double a,
                                  const double *__restrict__ a_dev, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  if (a_dev) a *= *a_dev;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] * (dinv ? dinv[i] : 1.0);
}

__global__ void reciprocal_kernel(double *__restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 1.0 / x[i];
}

__global__ void cast_kernel(const double *__restrict__ src, float *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void copy_kernel(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// stage 1: partials[k * nblocks + block] = sum over the block's chunk of V[k] . w
__global__ __launch_bounds__(kThreads) void multidot_kernel(const double *__restrict__ v, int64_t ld,
                                                            int nv, const double *__restrict__ w,
                                                            int64_t n,
                                                            double *__restrict__ partials,
                                                            const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  __shared__ double red[kThreads / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int k = 0; k < nv; ++k) {
    const double *vk = v + (int64_t)k * ld;
    double s = 0.0;
    for (int64_t i = lo + tid; i < hi; i += kThreads) s += vk[i] * w[i];
    s = wave_sum(s);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) tot += red[q];
      partials[(int64_t)k * gridDim.x + blockIdx.x] = tot;
    }
    __syncthreads();
  }
}

// Stage 1 for up to NV vectors at once: each thread reads w[i] once and keeps
// the nv running dot products in registers; one reduction per workgroup
// (cross-lane adds, then the four waves' sums through LDS) writes
// partials[k * nblocks + block].  Same chunks and the same summation tree for
// every k, so results are bitwise repeatable.
template <int NV>
__global__ __launch_bounds__(kThreads) void multidot_regs_kernel(const double *__restrict__ v, int64_t ld,
                                                                 int nv, const double *__restrict__ w,
                                                                 int64_t n, double *__restrict__ partials,
                                                                 const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  __shared__ double red[kThreads / 64][NV];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  // rows past nv repeat row nv - 1 (always in bounds, served from cache) so that
  // the NV loads of an element carry no branch and are all in flight together
  const double *__restrict__ rows[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) rows[k] = v + (int64_t)(k < nv ? k : nv - 1) * ld;
  for (int64_t i = lo + tid; i < hi; i += kThreads) {
    const double wi = w[i];
    double vk[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) vk[k] = rows[k][i];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += vk[k] * wi;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double t = wave_sum(acc[k]);
      if (lane == 0) red[wid][k] = t;
    }
  }
  __syncthreads();
  if (tid < nv) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) tot += red[q][tid];
    partials[(int64_t)tid * gridDim.x + blockIdx.x] = tot;
  }
}

// stage 2: out[k] = sum_b partials[k * nblocks + b], one wave per k
__global__ void multidot_finish_kernel(const double *__restrict__ partials, int nblocks, int nv,
                                       double *__restrict__ out, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (k >= nv) return;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += partials[(int64_t)k * nblocks + b];
  s = wave_sum(s);
  if (lane == 0) out[k] = s;
}

__global__ void multi_axpy_kernel(const double *__restrict__ v, int64_t ld, int nv,
                                  const double *__restrict__ h, double *__restrict__ w, int64_t n,
                                  const int32_t *__restrict__ nv_dev, const int32_t *__restrict__ halt) {
  if (halt && *halt) return;
  if (nv_dev) nv = *nv_dev;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = w[i];
    for (int k = 0; k < nv; ++k) s -= v[(int64_t)k * ld + i] * h[k];
    w[i] = s;
  }
}

inline int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t launch_gemv_batched(const GemvDesc *d_desc, const RowTile *d_tiles, int32_t n_tiles,
                               int32_t max_cols, const void *mat, bool fp32, const double *x,
                               const int32_t *xmap, double *y, const int32_t *omap, double alpha,
                               double beta, const double *y0, hipStream_t s, const int32_t *halt) {
  if (n_tiles <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)max_cols;
  if (fp32) {
    hipLaunchKernelGGL(gemv_batched_kernel<float>, dim3(n_tiles), dim3(kThreads), lds, s, d_desc,
                       d_tiles, static_cast<const float *>(mat), x, xmap, y, omap, alpha, beta, y0, halt);
  } else {
    hipLaunchKernelGGL(gemv_batched_kernel<double>, dim3(n_tiles), dim3(kThreads), lds, s, d_desc,
                       d_tiles, static_cast<const double *>(mat), x, xmap, y, omap, alpha, beta, y0, halt);
  }
  return hipGetLastError();
}

// z_e = T_e^T x[C_e] for every element (the transposed Schur product's
// element part): one workgroup per (element, 256 columns of T_e); each thread
// owns a column and walks the rows, so the workgroup reads every row segment
// contiguously; four rows in flight per thread, FP64 accumulation.
template <typename TM>
__global__ __launch_bounds__(256) void gemv_t_kernel(const GemvDesc *__restrict__ desc,
                                                     const RowTile *__restrict__ tiles, const TM *__restrict__ mat,
                                                     const double *__restrict__ x, const int32_t *__restrict__ xmap,
                                                     double *__restrict__ z) {
  extern __shared__ double xs[];
  const RowTile t = tiles[blockIdx.x];
  const GemvDesc d = desc[t.prob];
  for (int r = threadIdx.x; r < d.rows; r += blockDim.x) xs[r] = x[xmap[d.x_off + r]];
  __syncthreads();
  const int j = t.row0 + threadIdx.x;
  if (j >= d.cols) return;
  const TM *__restrict__ col = mat + d.m_off + j;
  const int64_t ld = d.cols;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int r = 0;
  for (; r + 4 <= d.rows; r += 4) {
    a0 += (double)col[r * ld] * xs[r];
    a1 += (double)col[(r + 1) * ld] * xs[r + 1];
    a2 += (double)col[(r + 2) * ld] * xs[r + 2];
    a3 += (double)col[(r + 3) * ld] * xs[r + 3];
  }
  for (; r < d.rows; ++r) a0 += (double)col[r * ld] * xs[r];
  z[d.y_off + j] = (a0 + a1) + (a2 + a3);
}

// y = S^T x (assembled form): z = T_e^T x[C_e] per element, then
// y = R^T x + pull(z), R^T from the transposed remainder pattern
hipError_t launch_schur_apply_t(const Plan &p, const double *x, double *z, double *y, bool lo) {
  const size_t lds = sizeof(double) * (size_t)std::max(1, p.max_nc);
  if (lo)
    hipLaunchKernelGGL(gemv_t_kernel<float>, dim3(p.n_ct_s), dim3(256), lds, p.stream, p.d_gv_s, p.d_ct_s,
                       static_cast<const float *>(p.sloc), x, p.d_cmap, z);
  else
    hipLaunchKernelGGL(gemv_t_kernel<double>, dim3(p.n_ct_s), dim3(256), lds, p.stream, p.d_gv_s, p.d_ct_s,
                       static_cast<const double *>(p.sloc), x, p.d_cmap, z);
  const int64_t nb = p.n_bnodes;
  const int grid = (int)((nb + (kThreads / 64) - 1) / (kThreads / 64));
  if (lo) {
    if (p.n_rem > 0 && !p.rem_lo) return hipErrorInvalidValue;
    hipLaunchKernelGGL((bsr_pull_kernel_impl<float, true>), dim3(grid), dim3(kThreads), 0, p.stream, nb, 0.0,
                       nullptr, nullptr, 1.0, p.d_remt_rowptr, p.d_remt_col, p.d_remt_src, p.rem_lo, x, 1.0,
                       p.d_pull_ptr, p.d_pull_idx, z, y, nullptr);
  } else {
    hipLaunchKernelGGL((bsr_pull_kernel_impl<double, true>), dim3(grid), dim3(kThreads), 0, p.stream, nb, 0.0,
                       nullptr, nullptr, 1.0, p.d_remt_rowptr, p.d_remt_col, p.d_remt_src, p.rem_val, x, 1.0,
                       p.d_pull_ptr, p.d_pull_idx, z, y, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_bsr_pull(const Plan &p, bool full, double c0, const double *src0,
                           const int32_t *map0, double c1, const double *x, double c2,
                           const double *t, double *out, bool lo) {
  const int64_t nb = p.n_bnodes;
  const int grid = (int)((nb + (kThreads / 64) - 1) / (kThreads / 64));
  const int64_t *rp = full ? p.d_bb_rowptr : p.d_rem_rowptr;
  const int32_t *cl = full ? p.d_bb_col : p.d_rem_col;
  if (lo) {
    const float *v = full ? p.bb_lo : p.rem_lo;
    if (c1 != 0.0 && !v && (full ? p.nnzb : p.n_rem) > 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((bsr_pull_kernel_impl<float, false>), dim3(grid), dim3(kThreads), 0, p.stream, nb, c0, src0, map0, c1,
                       rp, cl, nullptr, v, x, c2, p.d_pull_ptr, p.d_pull_idx, t, out, p.halt);
  } else {
    hipLaunchKernelGGL((bsr_pull_kernel_impl<double, false>), dim3(grid), dim3(kThreads), 0, p.stream, nb, c0, src0, map0, c1,
                       rp, cl, nullptr, full ? p.bb_val : p.rem_val, x, c2, p.d_pull_ptr, p.d_pull_idx, t, out,
                       p.halt);
  }
  return hipGetLastError();
}

hipError_t launch_schur_gemv_rem(const Plan &p, const double *x, double *t, double *rx, bool lo) {
  const int64_t nb = p.n_bnodes;
  const int64_t rem_wg = (nb + (kThreads / 64) - 1) / (kThreads / 64);
  // one GEMV tile every `ratio` workgroups, ratio odd and at most
  // 1 + rem_wg / n_tiles so that the grid of n_tiles + rem_wg workgroups places
  // every tile (the remainder takes the rest, and the tail once tiles run out)
  int64_t ratio = p.n_rt_s > 0 ? 1 + rem_wg / p.n_rt_s : 1;
  if (ratio % 2 == 0) --ratio;
  const int64_t grid = (int64_t)p.n_rt_s + rem_wg;
  const size_t lds = sizeof(double) * (size_t)p.max_nc;
  if (lo) {
    if (!p.rem_lo && p.n_rem > 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((schur_gemv_rem_kernel<float, float>), dim3((unsigned)grid), dim3(kThreads), lds, p.stream,
                       p.d_gv_s, p.d_rt_s, p.n_rt_s, static_cast<const float *>(p.sloc), x, p.d_cmap, t, ratio, nb,
                       p.d_rem_rowptr, p.d_rem_col, p.rem_lo, rx, p.halt);
  } else {
    hipLaunchKernelGGL((schur_gemv_rem_kernel<double, double>), dim3((unsigned)grid), dim3(kThreads), lds,
                       p.stream, p.d_gv_s, p.d_rt_s, p.n_rt_s, static_cast<const double *>(p.sloc), x, p.d_cmap, t,
                       ratio, nb, p.d_rem_rowptr, p.d_rem_col, p.rem_val, rx, p.halt);
  }
  return hipGetLastError();
}

hipError_t launch_precond_setup(const Plan &p, const void *t, bool fp32) {
  const int grid = (int)((p.n_bnodes + 127) / 128);
  if (fp32)
    hipLaunchKernelGGL(precond_setup_kernel<float>, dim3(grid), dim3(128), 0, p.stream, p.n_bnodes,
                       p.d_rem_rowptr, p.d_rem_col, p.d_rem_src, p.bb_val, p.d_pull_ptr,
                       p.d_pull_idx, p.d_slot_soff, p.d_slot_nc, p.d_slot_pos,
                       static_cast<const float *>(t), p.pc_blk, p.diag_s);
  else
    hipLaunchKernelGGL(precond_setup_kernel<double>, dim3(grid), dim3(128), 0, p.stream, p.n_bnodes,
                       p.d_rem_rowptr, p.d_rem_col, p.d_rem_src, p.bb_val, p.d_pull_ptr,
                       p.d_pull_idx, p.d_slot_soff, p.d_slot_nc, p.d_slot_pos,
                       static_cast<const double *>(t), p.pc_blk, p.diag_s);
  return hipGetLastError();
}

hipError_t launch_mf_diag_blocks(const Plan &p, const void *abi, bool fp32) {
  const int64_t n_slots = p.off_c[p.n_elem] / 5;
  if (n_slots <= 0) return hipSuccess;
  const int grid = (int)((n_slots + (kThreads / 64) - 1) / (kThreads / 64));
  if (fp32)
    hipLaunchKernelGGL(mf_diag_blocks_kernel<float>, dim3(grid), dim3(kThreads), 0, p.stream, n_slots, p.d_slot_ib,
                       p.d_slot_ni, p.d_slot_nc, p.d_slot_pos, static_cast<const float *>(abi),
                       static_cast<const float *>(p.xmat), p.mf_dblk);
  else
    hipLaunchKernelGGL(mf_diag_blocks_kernel<double>, dim3(grid), dim3(kThreads), 0, p.stream, n_slots,
                       p.d_slot_ib, p.d_slot_ni, p.d_slot_nc, p.d_slot_pos, static_cast<const double *>(abi),
                       static_cast<const double *>(p.xmat), p.mf_dblk);
  return hipGetLastError();
}

hipError_t launch_precond_setup_mf(const Plan &p) {
  if (p.n_bnodes <= 0) return hipSuccess;
  const int grid = (int)((p.n_bnodes + 127) / 128);
  hipLaunchKernelGGL(precond_setup_mf_kernel, dim3(grid), dim3(128), 0, p.stream, p.n_bnodes, p.d_bb_rowptr,
                     p.d_bb_col, p.bb_val, p.d_pull_ptr, p.d_pull_idx, p.mf_dblk, p.pc_blk, p.diag_s);
  return hipGetLastError();
}

hipError_t launch_block_mask(const double *mat, const int64_t *m_off, const int32_t *rb_n, const int32_t *cb_n,
                             const int64_t *mask_off, uint8_t *mask, int n_elem, hipStream_t s) {
  if (n_elem <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_mask_kernel, dim3(16, n_elem), dim3(kThreads), 0, s, mat, m_off, rb_n, cb_n, mask_off,
                     mask);
  return hipGetLastError();
}

hipError_t launch_mask_diff(const uint8_t *a, const uint8_t *b, int64_t n, int32_t *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_diff_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, a, b, n, flag);
  return hipGetLastError();
}

hipError_t launch_gather_blocks_ld(const void *src, const int64_t *src_off, const int32_t *ld, int64_t n, void *dst,
                                   bool fp32, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(gather_blocks_ld_kernel<float>, dim3(grid_for(n * 25)), dim3(kThreads), 0, s,
                       static_cast<const float *>(src), src_off, ld, n, static_cast<float *>(dst));
  else
    hipLaunchKernelGGL(gather_blocks_ld_kernel<double>, dim3(grid_for(n * 25)), dim3(kThreads), 0, s,
                       static_cast<const double *>(src), src_off, ld, n, static_cast<double *>(dst));
  return hipGetLastError();
}

hipError_t launch_bsr5_rows(int64_t n_rows, const int64_t *rowptr, const int32_t *xnode, const void *val,
                            bool fp32, const double *x, const int64_t *ybase, double *y, hipStream_t s,
                            const int32_t *halt) {
  if (n_rows <= 0) return hipSuccess;
  const int grid = (int)((n_rows + (kThreads / 64) - 1) / (kThreads / 64));
  if (fp32)
    hipLaunchKernelGGL(bsr5_rows_kernel<float>, dim3(grid), dim3(kThreads), 0, s, n_rows, rowptr, xnode,
                       static_cast<const float *>(val), x, ybase, y, halt);
  else
    hipLaunchKernelGGL(bsr5_rows_kernel<double>, dim3(grid), dim3(kThreads), 0, s, n_rows, rowptr, xnode,
                       static_cast<const double *>(val), x, ybase, y, halt);
  return hipGetLastError();
}

hipError_t launch_precond_apply(const Plan &p, int mode, const double *x, double *y, double a) {
  const int64_t n = 5 * p.n_bnodes;
  hipLaunchKernelGGL(precond_apply_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, p.stream, mode, p.n_bnodes, p.diag_s, p.pc_blk, x, y, a, p.halt);
  return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int32_t *map, double *dst, int64_t n,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, src, map, dst, n);
  return hipGetLastError();
}

hipError_t launch_gather_blocks(const double *src, const int32_t *idx, double *dst, int64_t nblocks,
                                hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_blocks_kernel, dim3(grid_for(nblocks * 25)), dim3(kThreads), 0, s, src, idx, dst,
                     nblocks);
  return hipGetLastError();
}

hipError_t launch_guess_err_gather(const float *y, const float *t, const double *stats, const int32_t *map,
                                   int64_t n, double *e, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(guess_err_gather_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, y, t, stats, map, n, e);
  return hipGetLastError();
}

hipError_t launch_guess_grad_scatter(const double *g, const double *stats, const int32_t *map, int64_t n,
                                     int64_t n_dof, double a, float *dy, hipStream_t s) {
  if (n_dof > 0)
    hipLaunchKernelGGL(fill_zero_f32_kernel, dim3(grid_for(n_dof)), dim3(kThreads), 0, s, dy, n_dof);
  if (n > 0)
    hipLaunchKernelGGL(guess_grad_scatter_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, g, stats, map, n, a,
                       dy);
  return hipGetLastError();
}

hipError_t launch_scatter(const double *src, const int32_t *map, double *dst, int64_t n,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, src, map, dst, n);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s,
                        const int32_t *halt) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b, y, halt);
  return hipGetLastError();
}

hipError_t launch_fill(double *y, int64_t n, double v, hipStream_t s, const int32_t *halt) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, y, n, v, halt);
  return hipGetLastError();
}

hipError_t launch_scatter_axpby(int64_t n, double a, const double *x, double b, const double *yin,
                                const int32_t *map, double *dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_axpby_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b,
                     yin, map, dst);
  return hipGetLastError();
}

hipError_t launch_diag_scale(const double *x, const double *dinv, double *y, int64_t n, double a,
                             hipStream_t s, const double *a_dev, const int32_t *halt) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_scale_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, x, dinv, y, n, a, a_dev,
                     halt);
  return hipGetLastError();
}

hipError_t launch_reciprocal(double *x, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reciprocal_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_cast_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_kernel, dim3(grid_for((int64_t)n)), dim3(kThreads), 0, s, src, dst,
                     (int64_t)n);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for((int64_t)n)), dim3(kThreads), 0, s, src, dst,
                     (int64_t)n);
  return hipGetLastError();
}

hipError_t launch_multidot(const double *v, int64_t ld, int32_t nv, const double *w, int64_t n,
                           double *partials, int32_t nblocks, double *out, hipStream_t s,
                           const int32_t *halt) {
#define SCDG_MULTIDOT(NVB)                                                                                      \
  hipLaunchKernelGGL(multidot_regs_kernel<NVB>, dim3(nblocks), dim3(kThreads), 0, s, v, ld, nv, w, n, partials, \
                     halt)
  if (nv <= 0) return hipSuccess;
  if (nv <= 4) {
    SCDG_MULTIDOT(4);
  } else if (nv <= 8) {
    SCDG_MULTIDOT(8);
  } else if (nv <= 12) {
    SCDG_MULTIDOT(12);
  } else if (nv <= 16) {
    SCDG_MULTIDOT(16);
  } else if (nv <= 20) {
    SCDG_MULTIDOT(20);
  } else if (nv <= 24) {
    SCDG_MULTIDOT(24);
  } else if (nv <= 28) {
    SCDG_MULTIDOT(28);
  } else if (nv <= 32) {
    SCDG_MULTIDOT(32);
  } else
    hipLaunchKernelGGL(multidot_kernel, dim3(nblocks), dim3(kThreads), 0, s, v, ld, nv, w, n, partials, halt);
#undef SCDG_MULTIDOT
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int waves_per_block = kThreads / 64;
  hipLaunchKernelGGL(multidot_finish_kernel, dim3((nv + waves_per_block - 1) / waves_per_block),
                     dim3(kThreads), 0, s, partials, nblocks, nv, out, halt);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double *v, int64_t ld, int32_t nv, const double *h, double *w,
                             int64_t n, hipStream_t s, const int32_t *nv_dev, const int32_t *halt) {
  if (n <= 0 || (nv <= 0 && !nv_dev)) return hipSuccess;
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, v, ld, nv, h, w,
                     n, nv_dev, halt);
  return hipGetLastError();
}

// ------------------------------------------------ device-resident GMRES
// State of one restart cycle in device memory (no host round trip per
// iteration): st[0] = halt (1 once converged, broken down or at the cycle's
// iteration limit st[2]), st[1] = number of completed iterations; dev[0] =
// 1 / h_{j+1,j} (scale of the next basis vector), dev[1] = |g_{j+1}| (residual
// estimate), dev[2] = the absolute stopping target.  H is (m+1) x m row-major,
// rotated in place; cs, sn the Givens rotations; g the rotated right-hand side.
__global__ void krylov_start_kernel(double beta, double target, int limit, double *__restrict__ g,
                                    int32_t *__restrict__ st, double *__restrict__ dev) {
  for (int i = threadIdx.x; i <= limit; i += blockDim.x) g[i] = i == 0 ? beta : 0.0;
  if (threadIdx.x == 0) {
    st[0] = (beta <= target || limit <= 0) ? 1 : 0;
    st[1] = 0;
    st[2] = limit;
    dev[0] = 0.0;
    dev[1] = beta;
    dev[2] = target;
  }
}

// Iteration j: the Hessenberg column from the two Gram-Schmidt passes and the
// squared norm of the orthogonalized vector (hc = [pass 1 | pass 2 | norm^2],
// m+1 entries each), then the Givens update and the stopping test.
__global__ void krylov_givens_kernel(int j, int m, const double *__restrict__ hc, double *__restrict__ H,
                                     double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
                                     int32_t *__restrict__ st, double *__restrict__ dev) {
  if (threadIdx.x != 0 || st[0]) return;
  for (int i = 0; i <= j; ++i) H[i * m + j] = hc[i] + hc[(m + 1) + i];
  const double hn = sqrt(fmax(0.0, hc[2 * (m + 1)]));
  H[(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[i * m + j], b = H[(i + 1) * m + j];
    H[i * m + j] = cs[i] * a + sn[i] * b;
    H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[j * m + j];
  const double den = hypot(a, hn);
  cs[j] = den > 0 ? a / den : 1.0;
  sn[j] = den > 0 ? hn / den : 0.0;
  H[j * m + j] = den;
  H[(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  st[1] = j + 1;
  dev[0] = hn > 0 ? 1.0 / hn : 0.0;
  dev[1] = fabs(g[j + 1]);
  if (fabs(g[j + 1]) <= dev[2] || hn == 0.0 || j + 1 >= st[2]) st[0] = 1;
}

// y = H^-1 g over the completed iterations; writes -y (the basis update
// subtracts, see multi_axpy)
__global__ void krylov_solve_kernel(int m, const double *__restrict__ H, const double *__restrict__ g,
                                    const int32_t *__restrict__ st, double *__restrict__ yneg,
                                    const int32_t *__restrict__ halt) {
  if (threadIdx.x != 0 || (halt && *halt)) return;
  const int k = st[1];
  double y[64];
  for (int i = k - 1; i >= 0; --i) {
    double v = g[i];
    for (int q = i + 1; q < k; ++q) v -= H[i * m + q] * y[q];
    y[i] = v / H[i * m + i];
  }
  for (int i = 0; i < k; ++i) yneg[i] = -y[i];
}

hipError_t launch_krylov_start(double beta, double target, int limit, double *g, int32_t *st, double *dev,
                               hipStream_t s) {
  hipLaunchKernelGGL(krylov_start_kernel, dim3(1), dim3(64), 0, s, beta, target, limit, g, st, dev);
  return hipGetLastError();
}

hipError_t launch_krylov_givens(int j, int m, const double *hc, double *H, double *cs, double *sn, double *g,
                                int32_t *st, double *dev, hipStream_t s) {
  hipLaunchKernelGGL(krylov_givens_kernel, dim3(1), dim3(64), 0, s, j, m, hc, H, cs, sn, g, st, dev);
  return hipGetLastError();
}

hipError_t launch_krylov_solve(int m, const double *H, const double *g, const int32_t *st, double *yneg,
                               hipStream_t s, const int32_t *halt) {
  hipLaunchKernelGGL(krylov_solve_kernel, dim3(1), dim3(64), 0, s, m, H, g, st, yneg, halt);
  return hipGetLastError();
}

// ------------------------------------------------ Newton iteration on the device
// GMRES state of the condensed solve inside one Newton iteration (all in device
// memory, so that a whole iteration can be replayed from a graph):
//   stat[0] = ||R(Q)||^2, stat[1] = ||b_S||^2, stat[2] = ||R(Q_s)||,
//   stat[3] = ||b_S - S x||^2 at the end of a restart cycle;
//   st[0] Arnoldi halt, st[1] iterations of the current cycle, st[2] cycle
//   length, st[3] solve finished (gates the end-of-cycle work), st[4] GMRES
//   iterations of this Newton iteration, st[5] 1 if the tolerance was met.
// The GMRES tolerance of the iteration is the inexact-Newton forcing term
// clip(eta_c ||R(Q_s)|| / ||R(Q)||, lin_tol, eta_max) (eta_c <= 0: lin_tol).
__global__ void newton_gmres_setup_kernel(const double *__restrict__ stat, double eta_c, double lin_tol,
                                          double eta_max, int m, double *__restrict__ g,
                                          int32_t *__restrict__ st, double *__restrict__ dev) {
  if (threadIdx.x != 0) return;
  const double rn = sqrt(stat[0]), beta = sqrt(stat[1]);
  double tol = lin_tol;
  if (eta_c > 0.0 && rn > 0.0) tol = fmin(eta_max, fmax(lin_tol, eta_c * stat[2] / rn));
  const double target = tol * beta;
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  const int done = beta > target ? 0 : 1;  // also when beta is not finite
  st[0] = done;
  st[1] = 0;
  st[2] = m;
  st[3] = done;
  st[4] = 0;
  st[5] = beta <= target ? 1 : 0;
  dev[0] = beta > 0.0 ? 1.0 / beta : 0.0;
  dev[1] = beta;
  dev[2] = target;
}

// After the true residual of a cycle: stop, or set up the next cycle.
__global__ void newton_gmres_restart_kernel(const double *__restrict__ stat, int m, double *__restrict__ g,
                                            int32_t *__restrict__ st, double *__restrict__ dev) {
  if (threadIdx.x != 0 || st[3]) return;
  const int it = st[1];
  st[4] += it;
  const double beta = sqrt(stat[3]);
  dev[1] = beta;
  st[1] = 0;
  if (!(beta > dev[2]) || it == 0) {
    // met the tolerance, not finite, or no progress possible
    st[0] = 1;
    st[3] = 1;
    st[5] = beta <= dev[2] ? 1 : 0;
    return;
  }
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  st[0] = 0;
  dev[0] = 1.0 / beta;
}

hipError_t launch_newton_gmres_setup(const double *stat, double eta_c, double lin_tol, double eta_max, int m,
                                     double *g, int32_t *st, double *dev, hipStream_t s) {
  hipLaunchKernelGGL(newton_gmres_setup_kernel, dim3(1), dim3(64), 0, s, stat, eta_c, lin_tol, eta_max, m, g,
                     st, dev);
  return hipGetLastError();
}

hipError_t launch_newton_gmres_restart(const double *stat, int m, double *g, int32_t *st, double *dev,
                                       hipStream_t s) {
  hipLaunchKernelGGL(newton_gmres_restart_kernel, dim3(1), dim3(64), 0, s, stat, m, g, st, dev);
  return hipGetLastError();
}

}  // namespace scdg
