// Dense direct solve of the condensed system S Q_b = b_S (the paper solves the
// condensed system with a direct LU solver; Section 4, Tables 'Advantages').
//
// S is assembled densely from A_bb and the element Schur blocks, then factored
// by right-looking blocked LU with partial pivoting (LAPACK getrf semantics:
// lowest row index on ties, swaps applied across the whole row):
//   panel (one workgroup, unblocked, in place) -> row swaps outside the panel
//   -> U12 = L11^-1 A12 -> A22 -= L21 U12 on the matrix cores (batched GEMM).
// The triangular solves run in one workgroup.  Used for small n1 only.
#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 256;
constexpr int kPanel = 32;

// remainder blocks of A_bb (those not folded into an element block)
__global__ void dense_fill_bb_kernel(int64_t n_bnodes, const int64_t *__restrict__ rowptr,
                                     const int32_t *__restrict__ col,
                                     const int32_t *__restrict__ src,
                                     const double *__restrict__ val, double *__restrict__ s,
                                     int64_t ld) {
  const int64_t g = blockIdx.x;
  if (g >= n_bnodes) return;
  for (int64_t b = rowptr[g]; b < rowptr[g + 1]; ++b) {
    const int64_t h = col[b];
    for (int q = threadIdx.x; q < 25; q += blockDim.x) {
      const int r = q / 5, w = q % 5;
      s[(5 * g + r) * ld + 5 * h + w] += val[(int64_t)src[b] * 25 + q];
    }
  }
}

// S[C_e, C_e] += T_e for one element (launched element after element so that
// overlapping entries are summed in a fixed order)
template <typename TM>
__global__ void dense_sub_elem_kernel(const TM *__restrict__ sloc, int nc,
                                      const int32_t *__restrict__ cmap, double *__restrict__ s,
                                      int64_t ld) {
  const int64_t n2 = (int64_t)nc * nc;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n2;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(q / nc), c = (int)(q % nc);
    s[(int64_t)cmap[r] * ld + cmap[c]] += (double)sloc[q];
  }
}

__global__ void zero_kernel(double *__restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// unblocked LU of the panel a[kb:n, kb:kb+nbw] (ld = n), pivots in piv[kb:kb+nbw]
__global__ __launch_bounds__(kThreads) void panel_lu_kernel(double *__restrict__ a, int n, int kb,
                                                            int nbw, int32_t *__restrict__ piv,
                                                            int32_t *__restrict__ info) {
  __shared__ double red_v[kThreads / 64];
  __shared__ int red_i[kThreads / 64];
  __shared__ double pivot_row[kPanel];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = 0; c < nbw; ++c) {
    const int k = kb + c;
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += kThreads) {
      const double v = fabs(a[(int64_t)i * n + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wid] = best;
      red_i[wid] = bi;
    }
    __syncthreads();
    best = red_v[0];
    bi = red_i[0];
    for (int w = 1; w < kThreads / 64; ++w)
      if (red_v[w] > best || (red_v[w] == best && red_i[w] < bi)) {
        best = red_v[w];
        bi = red_i[w];
      }
    const int pr = (bi < n) ? bi : k;
    if (tid < nbw && pr != k) {
      const int j = kb + tid;
      const double t = a[(int64_t)k * n + j];
      a[(int64_t)k * n + j] = a[(int64_t)pr * n + j];
      a[(int64_t)pr * n + j] = t;
    }
    if (tid == 0) piv[k] = pr;
    __syncthreads();
    if (tid < nbw) pivot_row[tid] = a[(int64_t)k * n + kb + tid];
    __syncthreads();
    double d = pivot_row[c];
    if (!(d != 0.0) || !isfinite(d)) {
      if (tid == 0 && info[0] == 0) info[0] = k + 1;
      d = 1.0;
    }
    const double inv_d = 1.0 / d;
    for (int i = k + 1 + tid; i < n; i += kThreads) {
      double *row = a + (int64_t)i * n;
      const double l = row[k] * inv_d;
      row[k] = l;
      for (int j = c + 1; j < nbw; ++j) row[kb + j] -= l * pivot_row[j];
    }
    __syncthreads();
  }
}

// apply the panel's row swaps to every column outside [kb, kb+nbw)
__global__ void dense_swap_kernel(double *__restrict__ a, int n, int kb, int nbw,
                                  const int32_t *__restrict__ piv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= kb && j < kb + nbw)) return;
  for (int c = 0; c < nbw; ++c) {
    const int k = kb + c, pr = piv[k];
    if (pr != k) {
      const double t = a[(int64_t)k * n + j];
      a[(int64_t)k * n + j] = a[(int64_t)pr * n + j];
      a[(int64_t)pr * n + j] = t;
    }
  }
}

// U12 = L11^-1 A12 for the columns right of the panel (one thread per column)
__global__ void dense_trsm_kernel(double *__restrict__ a, int n, int kb, int nbw) {
  __shared__ double l11[kPanel * kPanel];
  for (int q = threadIdx.x; q < nbw * nbw; q += blockDim.x)
    l11[q] = a[(int64_t)(kb + q / nbw) * n + kb + q % nbw];
  __syncthreads();
  const int j = kb + nbw + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double x[kPanel];
  for (int r = 0; r < nbw; ++r) {
    double v = a[(int64_t)(kb + r) * n + j];
    for (int q = 0; q < r; ++q) v -= l11[r * nbw + q] * x[q];
    x[r] = v;
    a[(int64_t)(kb + r) * n + j] = v;
  }
}

// forward (unit L, with row swaps) and backward substitution, one workgroup
__global__ __launch_bounds__(1024) void dense_solve_kernel(const double *__restrict__ lu, int n,
                                                           const int32_t *__restrict__ piv,
                                                           double *__restrict__ x) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < n; ++k) {
      const int pr = piv[k];
      if (pr != k) {
        const double t = x[k];
        x[k] = x[pr];
        x[pr] = t;
      }
    }
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double xj = x[j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) x[i] -= lu[(int64_t)i * n + j] * xj;
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (threadIdx.x == 0) x[j] /= lu[(int64_t)j * n + j];
    __syncthreads();
    const double xj = x[j];
    for (int i = threadIdx.x; i < j; i += blockDim.x) x[i] -= lu[(int64_t)i * n + j] * xj;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_dense_assemble(const Plan &p, double *s) {
  const int64_t n = p.n1;
  hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(kThreads), 0, p.stream, s, n * n);
  hipLaunchKernelGGL(dense_fill_bb_kernel, dim3((unsigned)p.n_bnodes), dim3(32), 0, p.stream,
                     p.n_bnodes, p.d_rem_rowptr, p.d_rem_col, p.d_rem_src, p.bb_val, s, n);
  const bool fp32 = p.prec == SCDG_FP32;
  const size_t esz = fp32 ? sizeof(float) : sizeof(double);
  for (int e = 0; e < p.n_elem; ++e) {
    const int nc = p.nc[e];
    const char *base = static_cast<const char *>(p.sloc) + esz * p.off_cc[e];
    const int grid = (int)std::min<int64_t>(1024, ((int64_t)nc * nc + kThreads - 1) / kThreads);
    if (fp32)
      hipLaunchKernelGGL(dense_sub_elem_kernel<float>, dim3(grid), dim3(kThreads), 0, p.stream,
                         reinterpret_cast<const float *>(base), nc, p.d_cmap + p.off_c[e], s, n);
    else
      hipLaunchKernelGGL(dense_sub_elem_kernel<double>, dim3(grid), dim3(kThreads), 0, p.stream,
                         reinterpret_cast<const double *>(base), nc, p.d_cmap + p.off_c[e], s, n);
  }
  return hipGetLastError();
}

hipError_t launch_dense_lu(Plan &p, double *a, int32_t n, int32_t *piv, int32_t *info) {
  hipError_t err = hipMemsetAsync(info, 0, sizeof(int32_t), p.stream);
  if (err != hipSuccess) return err;
  const int n_panels = (n + kPanel - 1) / kPanel;
  std::vector<GemmDesc> descs(n_panels);
  for (int t = 0; t < n_panels; ++t) {
    const int kb = t * kPanel, nbw = std::min(kPanel, n - kb);
    const int rest = n - kb - nbw;
    descs[t] = GemmDesc{(int64_t)(kb + nbw) * n + kb, (int64_t)kb * n + kb + nbw,
                        (int64_t)(kb + nbw) * n + kb + nbw, rest, rest, nbw, n, n, n};
  }
  GemmDesc *d_desc = nullptr;
  err = hipMalloc(&d_desc, sizeof(GemmDesc) * n_panels);
  if (err != hipSuccess) return err;
  err = hipMemcpy(d_desc, descs.data(), sizeof(GemmDesc) * n_panels, hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d_desc);
    return err;
  }
  for (int t = 0; t < n_panels && err == hipSuccess; ++t) {
    const int kb = t * kPanel, nbw = std::min(kPanel, n - kb);
    hipLaunchKernelGGL(panel_lu_kernel, dim3(1), dim3(kThreads), 0, p.stream, a, n, kb, nbw, piv,
                       info);
    hipLaunchKernelGGL(dense_swap_kernel, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       p.stream, a, n, kb, nbw, piv);
    const int rest = n - kb - nbw;
    if (rest > 0) {
      hipLaunchKernelGGL(dense_trsm_kernel, dim3((rest + 127) / 128), dim3(128), 0, p.stream, a, n,
                         kb, nbw);
      const int cfg = rest >= 512 ? kGemm128x128 : kGemm64x64;
      int bm, bn;
      gemm_tile_shape(cfg, &bm, &bn);
      const int tiles = ((rest + bm - 1) / bm) * ((rest + bn - 1) / bn);
      err = launch_gemm_batched(cfg, d_desc + t, nullptr, tiles, a, a, a, -1.0, 1.0, false, p.stream);
    }
    if (err == hipSuccess) err = hipGetLastError();
  }
  hipError_t err2 = hipStreamSynchronize(p.stream);
  (void)hipFree(d_desc);
  return err != hipSuccess ? err : err2;
}

hipError_t launch_dense_solve(const double *lu, int32_t n, const int32_t *piv, double *x,
                              hipStream_t s) {
  hipLaunchKernelGGL(dense_solve_kernel, dim3(1), dim3(1024), 0, s, lu, n, piv, x);
  return hipGetLastError();
}

}  // namespace scdg
