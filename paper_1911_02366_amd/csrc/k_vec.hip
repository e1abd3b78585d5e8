// Memory-bound kernels of the condensed solve: batched element GEMVs with
// coalesced gathers of the DOFs they read, the A_bb BSR product fused with the
// "pull" reduction of element Schur contributions, and the Krylov vector
// operations (deterministic two-stage multi-dot for Gram-Schmidt, multi-AXPY,
// scaling).  All vectors are FP64; matrices may be FP64 or FP32 (accumulation
// is always FP64).
#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerTile = 64;

// ---------------------------------------------------------------- GEMV
// One workgroup = 64 rows of one element matrix.  The element's input vector is
// gathered once into LDS; each wave then streams 16 rows, four at a time, with
// lanes striding along the row (coalesced), and reduces with cross-lane adds.
template <typename TM>
__global__ __launch_bounds__(kThreads) void gemv_batched_kernel(
    const GemvDesc *__restrict__ desc, const RowTile *__restrict__ tiles, const TM *__restrict__ mat,
    const double *__restrict__ x, const int32_t *__restrict__ xmap, double *__restrict__ y,
    const int32_t *__restrict__ omap, double alpha, double beta, const double *__restrict__ y0) {
  extern __shared__ double xs[];
  const RowTile t = tiles[blockIdx.x];
  const GemvDesc d = desc[t.prob];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = tid; c < d.cols; c += kThreads) xs[c] = xmap ? x[xmap[d.x_off + c]] : x[d.x_off + c];
  __syncthreads();
  const TM *__restrict__ base = mat + d.m_off;
  const int r_begin = t.row0 + wid * (kRowsPerTile / 4);
  const int r_end = min(d.rows, r_begin + kRowsPerTile / 4);
  for (int r = r_begin; r < r_end; r += 4) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const TM *rows[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rows[q] = base + (int64_t)min(r + q, d.rows - 1) * d.cols;
    for (int c = lane; c < d.cols; c += 64) {
      const double xv = xs[c];
#pragma unroll
      for (int q = 0; q < 4; ++q) s[q] += (double)rows[q][c] * xv;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = wave_sum(s[q]);
    if (lane < 4 && r + lane < r_end) {
      double v = s[0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (lane == q) v = s[q];
      const int yi = d.y_off + r + lane;
      v *= alpha;
      if (beta != 0.0) v += beta * y0[yi];
      y[omap ? omap[yi] : yi] = v;
    }
  }
}

// ---------------------------------------------------- A_bb product + pull
// One wave per boundary node g (5 output rows).  Lanes take the BSR blocks of
// row g in turn; each block is 25 contiguous doubles.
__global__ __launch_bounds__(kThreads) void bsr_pull_kernel(
    int64_t n_bnodes, double c0, const double *__restrict__ src0, const int32_t *__restrict__ map0,
    double c1, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ x, double c2,
    const int32_t *__restrict__ pull_ptr, const int32_t *__restrict__ pull_idx,
    const double *__restrict__ t, double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (g >= n_bnodes) return;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c1 != 0.0) {
    for (int64_t blk = rowptr[g] + lane; blk < rowptr[g + 1]; blk += 64) {
      const double *v = val + blk * 25;
      const double *xv = x + (int64_t)col[blk] * 5;
      double xw[5];
#pragma unroll
      for (int w = 0; w < 5; ++w) xw[w] = xv[w];
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < 5; ++w) acc += v[r * 5 + w] * xw[w];
        s[r] += acc;
      }
    }
#pragma unroll
    for (int r = 0; r < 5; ++r) s[r] = wave_sum(s[r]);
  }
  if (lane < 5) {
    double mine = s[0];
#pragma unroll
    for (int r = 1; r < 5; ++r)
      if (lane == r) mine = s[r];
    const int64_t j = 5 * g + lane;
    double v = c1 * mine;
    if (c0 != 0.0) v += c0 * src0[map0 ? map0[j] : j];
    if (c2 != 0.0) {
      double p = 0.0;
      for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q) p += t[5 * (int64_t)pull_idx[q] + lane];
      v += c2 * p;
    }
    out[j] = v;
  }
}

// ------------------------------------------------------------ utilities
__global__ void gather_kernel(const double *__restrict__ src, const int32_t *__restrict__ map,
                              double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[map[i]];
}

__global__ void scatter_kernel(const double *__restrict__ src, const int32_t *__restrict__ map,
                               double *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[map[i]] = src[i];
}

__global__ void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                             double *__restrict__ y) {
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

__global__ void diag_scale_kernel(const double *__restrict__ x, const double *__restrict__ dinv,
                                  double *__restrict__ y, int64_t n, double a) {
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
                                                            double *__restrict__ partials) {
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

// stage 2: out[k] = sum_b partials[k * nblocks + b], one wave per k
__global__ void multidot_finish_kernel(const double *__restrict__ partials, int nblocks, int nv,
                                       double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (k >= nv) return;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += partials[(int64_t)k * nblocks + b];
  s = wave_sum(s);
  if (lane == 0) out[k] = s;
}

__global__ void multi_axpy_kernel(const double *__restrict__ v, int64_t ld, int nv,
                                  const double *__restrict__ h, double *__restrict__ w, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = w[i];
    for (int k = 0; k < nv; ++k) s -= v[(int64_t)k * ld + i] * h[k];
    w[i] = s;
  }
}

// diag(S) = diag(A_bb) - sum over elements containing the node of the element block diagonal
template <typename TM>
__global__ void diag_schur_kernel(int64_t n_bnodes, const int64_t *__restrict__ rowptr,
                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                  const int32_t *__restrict__ pull_ptr,
                                  const int32_t *__restrict__ pull_idx,
                                  const int64_t *__restrict__ slot_elem_off,
                                  const int32_t *__restrict__ slot_nc,
                                  const int32_t *__restrict__ slot_pos, const TM *__restrict__ sloc,
                                  double *__restrict__ diag) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= 5 * n_bnodes) return;
  const int64_t g = j / 5;
  const int v = (int)(j % 5);
  double dval = 0.0;
  for (int64_t b = rowptr[g]; b < rowptr[g + 1]; ++b)
    if (col[b] == g) dval += val[b * 25 + v * 5 + v];
  for (int q = pull_ptr[g]; q < pull_ptr[g + 1]; ++q) {
    const int s = pull_idx[q];
    const int64_t row = 5 * (int64_t)slot_pos[s] + v;
    dval -= (double)sloc[slot_elem_off[s] + row * slot_nc[s] + row];
  }
  diag[j] = dval;
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
                               double beta, const double *y0, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)max_cols;
  if (fp32) {
    hipLaunchKernelGGL(gemv_batched_kernel<float>, dim3(n_tiles), dim3(kThreads), lds, s, d_desc,
                       d_tiles, static_cast<const float *>(mat), x, xmap, y, omap, alpha, beta, y0);
  } else {
    hipLaunchKernelGGL(gemv_batched_kernel<double>, dim3(n_tiles), dim3(kThreads), lds, s, d_desc,
                       d_tiles, static_cast<const double *>(mat), x, xmap, y, omap, alpha, beta, y0);
  }
  return hipGetLastError();
}

hipError_t launch_bsr_pull(const Plan &p, double c0, const double *src0, const int32_t *map0,
                           double c1, const double *x, double c2, const double *t, double *out) {
  const int64_t nb = p.n_bnodes;
  const int grid = (int)((nb + (kThreads / 64) - 1) / (kThreads / 64));
  hipLaunchKernelGGL(bsr_pull_kernel, dim3(grid), dim3(kThreads), 0, p.stream, nb, c0, src0, map0,
                     c1, p.d_bb_rowptr, p.d_bb_col, p.bb_val, x, c2, p.d_pull_ptr, p.d_pull_idx, t,
                     out);
  return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int32_t *map, double *dst, int64_t n,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, src, map, dst, n);
  return hipGetLastError();
}

hipError_t launch_scatter(const double *src, const int32_t *map, double *dst, int64_t n,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, src, map, dst, n);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b, y);
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
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_scale_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, x, dinv, y, n, a);
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
                           double *partials, int32_t nblocks, double *out, hipStream_t s) {
  hipLaunchKernelGGL(multidot_kernel, dim3(nblocks), dim3(kThreads), 0, s, v, ld, nv, w, n,
                     partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int waves_per_block = kThreads / 64;
  hipLaunchKernelGGL(multidot_finish_kernel, dim3((nv + waves_per_block - 1) / waves_per_block),
                     dim3(kThreads), 0, s, partials, nblocks, nv, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double *v, int64_t ld, int32_t nv, const double *h, double *w,
                             int64_t n, hipStream_t s) {
  if (n <= 0 || nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, v, ld, nv, h, w,
                     n);
  return hipGetLastError();
}

hipError_t launch_diag_schur(const Plan &p, const void *sloc, bool fp32, double *diag) {
  const int64_t n = 5 * p.n_bnodes;
  const int grid = (int)((n + kThreads - 1) / kThreads);
  if (fp32) {
    hipLaunchKernelGGL(diag_schur_kernel<float>, dim3(grid), dim3(kThreads), 0, p.stream,
                       p.n_bnodes, p.d_bb_rowptr, p.d_bb_col, p.bb_val, p.d_pull_ptr, p.d_pull_idx,
                       p.d_slot_soff, p.d_slot_nc, p.d_slot_pos, static_cast<const float *>(sloc),
                       diag);
  } else {
    hipLaunchKernelGGL(diag_schur_kernel<double>, dim3(grid), dim3(kThreads), 0, p.stream,
                       p.n_bnodes, p.d_bb_rowptr, p.d_bb_col, p.bb_val, p.d_pull_ptr, p.d_pull_idx,
                       p.d_slot_soff, p.d_slot_nc, p.d_slot_pos, static_cast<const double *>(sloc),
                       diag);
  }
  return hipGetLastError();
}

}  // namespace scdg
