// Batched (grouped) dense GEMM on the CDNA4 matrix cores, FP64 and FP32:
//   C_p = alpha A_p B_p + beta C_p    for every problem p of the batch,
// row-major operands with per-problem sizes and leading dimensions.
//
// It forms X_e = A_ii(e)^-1 A_ib(e) and the element Schur blocks
// A_bi(e) X_e of eq. SC_step1, and the trailing updates of the dense LU of S.
//
// Tiling: a 256-thread workgroup computes a 64x64 tile of one problem; its four
// waves each own a 32x32 quarter made of 2x2 blocks of the 16x16x4 MFMA.  A and
// B tiles of depth 16 are staged through LDS (A stored k-major so that the 16
// lanes reading one MFMA operand column hit consecutive addresses).  The tile
// list is ordered so that consecutive tiles of one problem land on the same XCD
// (workgroups are dealt to the 8 XCDs round-robin), which keeps an element's
// operands in that XCD's L2.
#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void gemm_batched_kernel(const GemmDesc *__restrict__ desc,
                                                                const int32_t *__restrict__ tiles,
                                                                const T *__restrict__ A,
                                                                const T *__restrict__ B,
                                                                T *__restrict__ C, T alpha, T beta) {
  using M = Mfma<T>;
  __shared__ T as[BK][BM + 1];
  __shared__ T bs[BK][BN + 1];
  int prob, tm, tn;
  if (tiles != nullptr) {
    prob = tiles[3 * blockIdx.x];
    tm = tiles[3 * blockIdx.x + 1];
    tn = tiles[3 * blockIdx.x + 2];
    if (prob < 0) return;
  } else {
    prob = 0;
    const int tiles_m = (desc[0].m + BM - 1) / BM;
    tm = blockIdx.x % tiles_m;
    tn = blockIdx.x / tiles_m;
  }
  const GemmDesc d = desc[prob];
  const T *__restrict__ a = A + d.a_off;
  const T *__restrict__ b = B + d.b_off;
  T *__restrict__ c = C + d.c_off;
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= d.m || n0 >= d.n) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  typename M::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();

  // per-thread load coordinates
  const int a_row = tid >> 2, a_k = (tid & 3) * 4;      // A: 64 rows x 16 k
  const int b_k = tid >> 4, b_col = (tid & 15) * 4;     // B: 16 k x 64 cols

  for (int k0 = 0; k0 < d.k; k0 += BK) {
    {
      const int gr = m0 + a_row;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gk = k0 + a_k + u;
        as[a_k + u][a_row] = (gr < d.m && gk < d.k) ? a[(int64_t)gr * d.lda + gk] : T(0);
      }
      const int gk = k0 + b_k;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gc = n0 + b_col + u;
        bs[b_k][b_col + u] = (gk < d.k && gc < d.n) ? b[(int64_t)gk * d.ldb + gc] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = as[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = bs[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = M::mma(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + (lane & 15);
      if (col >= d.n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + M::row(lane, r);
        if (row < d.m) {
          T *dst = c + (int64_t)row * d.ldc + col;
          T v = alpha * acc[i][j][r];
          if (beta != T(0)) v += beta * (*dst);
          *dst = v;
        }
      }
    }
}

}  // namespace

int gemm_tile_m() { return BM; }
int gemm_tile_n() { return BN; }

hipError_t launch_gemm_batched(const GemmDesc *d_desc, const int32_t *d_tiles, int32_t n_tiles,
                               const void *a, const void *b, void *c, double alpha, double beta,
                               bool fp32, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (fp32) {
    hipLaunchKernelGGL(gemm_batched_kernel<float>, dim3(n_tiles), dim3(kThreads), 0, s, d_desc,
                       d_tiles, static_cast<const float *>(a), static_cast<const float *>(b),
                       static_cast<float *>(c), (float)alpha, (float)beta);
  } else {
    hipLaunchKernelGGL(gemm_batched_kernel<double>, dim3(n_tiles), dim3(kThreads), 0, s, d_desc,
                       d_tiles, static_cast<const double *>(a), static_cast<const double *>(b),
                       static_cast<double *>(c), alpha, beta);
  }
  return hipGetLastError();
}

}  // namespace scdg
