// Per-element multilayer perceptron for the learned initial guess of the
// implicit-step solve, with its training kernels (forward, backward, Adam,
// mean-squared loss) and the feature/target maps between DG vectors and the
// network.  FP32 storage; the matrix products run on FP32 MFMA, or with
// operands rounded to bfloat16 on the bf16 MFMA (scdg_mlp_set_compute), both
// with FP32 accumulation.
//
// Network: x (n_in) -> tanh(W_1^T x + b_1) -> ... (n_layers hidden layers of
// width n_hidden) -> W_out^T a + b_out (n_out, linear).  Row-major batches:
// X [batch x n_in], Y [batch x n_out].  Flat parameter vector, layer after
// layer: W_l [fan_in x fan_out] row-major, then b_l [fan_out].
//
// Backward (chain rule, batch rows independent):
//   dZ_L = dY;  dW_l = A_{l-1}^T dZ_l;  db_l = sum over rows of dZ_l;
//   dZ_{l-1} = (dZ_l W_l^T) * (1 - A_{l-1}^2)   (tanh' = 1 - tanh^2),  A_0 = X.
//
// Every reduction (bias gradients, loss, statistics) runs in a fixed order, so
// results are bitwise repeatable.
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kTile = 64;     // C tile rows and columns
constexpr int kBK = 16;       // K slab
constexpr int kThreads = 256; // 4 waves in a 2 x 2 grid, 32 x 32 each
constexpr int kRedBlocks = 256;

enum Epilogue { kEpiNone = 0, kEpiTanh = 1 };

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// Nearest bfloat16 of an FP32 value (ties to even), kept as an FP32 bit pattern
// whose low 16 bits are zero; NaN stays NaN.
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return __uint_as_float((u & 0x007fffffu) ? ((u | 0x00400000u) & 0xffff0000u) : u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(x) >> 16); }

// C = op(A) op(B) (+ bias[col]) (tanh) (* (1 - D^2)); op(A) is M x K, op(B) K x N.
// BF: the operands are rounded to bfloat16 when staged in LDS and multiplied
// by the 16x16x16 bf16 MFMA with FP32 accumulation (products of two bf16
// values are exact in FP32); otherwise FP32 operands and the 16x16x4 FP32 MFMA.
template <bool TA, bool TB, bool BF>
__global__ __launch_bounds__(kThreads) void mlp_gemm_kernel(int M, int N, int K,
                                                            const float *__restrict__ A, int lda,
                                                            const float *__restrict__ B, int ldb,
                                                            float *__restrict__ C, int ldc,
                                                            const float *__restrict__ bias, int epi,
                                                            const float *__restrict__ dact, int ldd) {
  using MF = Mfma<float>;
  __shared__ float as[2][kBK][kTile + 4];
  __shared__ float bs[2][kBK][kTile + 4];
  const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  float ra[4], rb[4];

  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int r, k;
      if (TA) {
        r = tid % kTile;
        k = tid / kTile + 4 * u;
      } else {
        k = tid % kBK;
        r = tid / kBK + 16 * u;
      }
      const int gr = m0 + r, gk = k0 + k;
      float v = 0.f;
      if (gr < M && gk < K) v = TA ? A[(int64_t)gk * lda + gr] : A[(int64_t)gr * lda + gk];
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int c, k;
      if (TB) {
        k = tid % kBK;
        c = tid / kBK + 16 * u;
      } else {
        c = tid % kTile;
        k = tid / kTile + 4 * u;
      }
      const int gc = n0 + c, gk = k0 + k;
      float v = 0.f;
      if (gc < N && gk < K) v = TB ? B[(int64_t)gc * ldb + gk] : B[(int64_t)gk * ldb + gc];
      rb[u] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float va = BF ? bf16_round(ra[u]) : ra[u];
      const float vb = BF ? bf16_round(rb[u]) : rb[u];
      if (TA)
        as[buf][tid / kTile + 4 * u][tid % kTile] = va;
      else
        as[buf][tid % kBK][tid / kBK + 16 * u] = va;
      if (TB)
        bs[buf][tid % kBK][tid / kBK + 16 * u] = vb;
      else
        bs[buf][tid / kTile + 4 * u][tid % kTile] = vb;
    }
  };

  MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();

  const int nk = (K + kBK - 1) / kBK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * kBK);
    if constexpr (BF) {
      // 16x16x16: lane l holds A[l % 16][4 (l / 16) + t] and B[4 (l / 16) + t][l % 16], t = 0..3
      bf16x4 af[2], bf[2];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 4 * (lane >> 4) + t;
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i][t] = bf16_bits(as[buf][k][wm * 32 + i * 16 + (lane & 15)]);
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j][t] = bf16_bits(bs[buf][k][wn * 32 + j * 16 + (lane & 15)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bf[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 4) {
        float af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = as[buf][kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = bs[buf][kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = MF::mma(af[i], bf[j], acc[i][j]);
      }
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + MF::row(lane, r);
        if (row >= M) continue;
        float v = acc[i][j][r];
        if (bias) v += bias[col];
        if (epi == kEpiTanh) v = tanhf(v);
        if (dact) {
          const float t = dact[(int64_t)row * ldd + col];
          v *= 1.f - t * t;
        }
        C[(int64_t)row * ldc + col] = v;
      }
    }
}

template <bool BF>
hipError_t gemm_typed(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                      float *C, int ldc, const float *bias, int epi, const float *dact, int ldd, hipStream_t s) {
  const dim3 grid((M + kTile - 1) / kTile, (N + kTile - 1) / kTile);
  if (!ta && !tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<false, false, BF>), grid, dim3(kThreads), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, bias, epi, dact, ldd);
  else if (ta && !tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<true, false, BF>), grid, dim3(kThreads), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, bias, epi, dact, ldd);
  else if (!ta && tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<false, true, BF>), grid, dim3(kThreads), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, bias, epi, dact, ldd);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                float *C, int ldc, const float *bias, int epi, const float *dact, int ldd, bool bf16,
                hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  return bf16 ? gemm_typed<true>(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, bias, epi, dact, ldd, s)
              : gemm_typed<false>(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, bias, epi, dact, ldd, s);
}

// Column sums of a row-major [rows x cols] matrix in two fixed-order stages:
// partial[c][chunk] over row chunks, then the sum over chunks.
constexpr int kColChunks = 64;

__global__ void colsum_partial_kernel(const float *__restrict__ a, int rows, int cols,
                                      float *__restrict__ partial) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  if (c >= cols) return;
  const int per = (rows + kColChunks - 1) / kColChunks;
  const int r0 = chunk * per, r1 = min(rows, r0 + per);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += a[(int64_t)r * cols + c];
  partial[(int64_t)c * kColChunks + chunk] = s;
}

__global__ void colsum_final_kernel(const float *__restrict__ partial, int cols, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int k = 0; k < kColChunks; ++k) s += partial[(int64_t)c * kColChunks + k];
  out[c] = s;
}

__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                            float *__restrict__ m2, int64_t n, float lr, float b1, float b2, float eps,
                            float corr1, float corr2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float mhat = a / corr1, vhat = b / corr2;
    w[i] -= lr * mhat / (sqrtf(vhat) + eps);
  }
}

// dY = 2 (Y - T) / n and per-block partial sums of (Y - T)^2 (in double)
__global__ void mse_partial_kernel(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                                   float *__restrict__ dy, double *__restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.f / (float)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    if (dy) dy[i] = scale * d;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_final_kernel(const double *__restrict__ partial, int n, int width, double scale,
                                 double *__restrict__ out) {
  // out[c] = scale * sum_k partial[k * width + c], one thread per column
  const int c = threadIdx.x;
  if (c >= width) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += partial[(int64_t)k * width + c];
  out[c] = s * scale;
}

// Field statistics in two passes (the second sums squared deviations from the
// mean, which avoids the cancellation of E[q^2] - E[q]^2).  Pass 1 sums q_v,
// dqp_v^2 (dqp: previous increment) and r_v^2 (r: residual, when given); pass 2
// sums (q_v - mean_v)^2 and, when the increment dq is given, (dq_v - dqp_v)^2.
// Each block writes its 15 partial sums.
__global__ void stats_partial_kernel(const double *__restrict__ q, const double *__restrict__ dqp,
                                     const double *__restrict__ dq, const double *__restrict__ r,
                                     const double *__restrict__ mean, int64_t n_nodes,
                                     double *__restrict__ partial) {
  __shared__ double red[15][256];
  double s[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) s[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_nodes;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double b = dqp[i * 5 + v];
      if (mean) {
        const double a = q[i * 5 + v] - mean[v];
        s[v] += a * a;
        if (dq) {
          const double c = dq[i * 5 + v] - b;
          s[5 + v] += c * c;
        }
      } else {
        s[v] += q[i * 5 + v];
        s[5 + v] += b * b;
        if (r) {
          const double c = r[i * 5 + v];
          s[10 + v] += c * c;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 15; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 15) partial[(int64_t)blockIdx.x * 15 + threadIdx.x] = red[threadIdx.x][0];
}

// stats = [mean[5], std[5], rms_prev[5], rms_corr[5], rms_res[5]].  Pass 1 fills
// mean, rms_prev and rms_res; pass 2 fills std and rms_corr (rms_prev when no
// increment is given).  A zero spread or root mean square maps to 1.
__global__ void stats_final_kernel(const double *__restrict__ partial, int n_blocks, int64_t n_nodes,
                                   int pass, int have_dq, double *__restrict__ stats) {
  const int v = threadIdx.x;
  if (v >= 5) return;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k = 0; k < n_blocks; ++k) {
    s1 += partial[(int64_t)k * 15 + v];
    s2 += partial[(int64_t)k * 15 + 5 + v];
    s3 += partial[(int64_t)k * 15 + 10 + v];
  }
  const double n = (double)n_nodes;
  if (pass == 1) {
    stats[v] = s1 / n;
    const double rms = sqrt(s2 / n);
    stats[10 + v] = rms > 0.0 ? rms : 1.0;
    const double rr = sqrt(s3 / n);
    stats[20 + v] = rr > 0.0 ? rr : 1.0;
  } else {
    const double sd = sqrt(s1 / n);
    stats[5 + v] = (sd > 0.0 && sd > 1e-12 * fabs(stats[v])) ? sd : 1.0;
    const double rc = sqrt(s2 / n);
    stats[15 + v] = have_dq ? (rc > 0.0 ? rc : 1.0) : stats[10 + v];
  }
}

// x[e] = [(q_e - mean) / std, dq_prev_e / rms_prev (, r_e / rms_res)] in FP32;
// nb = 2 or 3 blocks of dpe values per element
__global__ void features_kernel(const double *__restrict__ q, const double *__restrict__ dq,
                                const double *__restrict__ r, const double *__restrict__ stats, int64_t n_elem,
                                int dpe, int nb, float *__restrict__ x) {
  const int64_t total = n_elem * dpe;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / dpe;
    const int j = (int)(i - e * dpe);
    const int v = j % 5;
    float *xe = x + e * nb * dpe;
    xe[j] = (float)((q[i] - stats[v]) / stats[5 + v]);
    xe[dpe + j] = (float)(dq[i] / stats[10 + v]);
    if (nb == 3) xe[2 * dpe + j] = (float)(r[i] / stats[20 + v]);
  }
}

// t = (dq - dq_prev) / rms_corr  (training target)
__global__ void target_kernel(const double *__restrict__ dq, const double *__restrict__ dq_prev,
                              const double *__restrict__ stats, int64_t n, float *__restrict__ t) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    t[i] = (float)((dq[i] - dq_prev[i]) / stats[15 + (int)(i % 5)]);
}

// dq = dq_prev + rms_corr * y  (prediction)
__global__ void apply_kernel(const double *__restrict__ dq_prev, const float *__restrict__ y,
                             const double *__restrict__ stats, int64_t n, double *__restrict__ dq) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dq[i] = dq_prev[i] + stats[15 + (int)(i % 5)] * (double)y[i];
}

__global__ void gather_rows_kernel(const float *__restrict__ src, int width, const int32_t *__restrict__ idx,
                                   int count, float *__restrict__ dst) {
  const int64_t total = (int64_t)count * width;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / width;
    const int c = (int)(i - r * width);
    dst[i] = src[(int64_t)idx[r] * width + c];
  }
}

int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

}  // namespace

struct MlpContext {
  int n_in = 0, n_hidden = 0, n_layers = 0, n_out = 0, max_batch = 0;
  hipStream_t stream = nullptr;
  float *act = nullptr;       // hidden activations of the last forward, n_layers x max_batch x n_hidden
  float *dz = nullptr;        // two ping-pong buffers of max_batch x max(n_hidden, n_out)
  float *colpart = nullptr;   // kColChunks x max width
  double *red = nullptr;      // reduction partials
  int last_batch = -1;
  bool bf16 = false;          // GEMM operands rounded to bfloat16 (FP32 accumulation)
  std::vector<int64_t> w_off, b_off;
  std::vector<int> fan_in, fan_out;
  int64_t n_params = 0;
};

}  // namespace scdg

struct scdg_mlp {
  scdg::MlpContext c;
};

namespace {

using scdg::MlpContext;

scdg_status hip_status(hipError_t e) { return e == hipSuccess ? SCDG_OK : SCDG_ERR_HIP; }

void free_ctx(MlpContext &c) {
  if (c.act) (void)hipFree(c.act);
  if (c.dz) (void)hipFree(c.dz);
  if (c.colpart) (void)hipFree(c.colpart);
  if (c.red) (void)hipFree(c.red);
  c.act = c.dz = c.colpart = nullptr;
  c.red = nullptr;
}

}  // namespace

extern "C" {

scdg_status scdg_mlp_create(scdg_mlp **out, const scdg_mlp_shape *s, void *hip_stream) {
  if (!out || !s || s->n_in <= 0 || s->n_hidden <= 0 || s->n_layers < 0 || s->n_out <= 0 ||
      s->max_batch <= 0 || s->n_layers > 16)
    return SCDG_ERR_ARG;
  scdg_mlp *m = new (std::nothrow) scdg_mlp();
  if (!m) return SCDG_ERR_NOMEM;
  auto &c = m->c;
  c.n_in = s->n_in;
  c.n_hidden = s->n_hidden;
  c.n_layers = s->n_layers;
  c.n_out = s->n_out;
  c.max_batch = s->max_batch;
  c.stream = static_cast<hipStream_t>(hip_stream);
  int64_t off = 0;
  for (int l = 0; l <= c.n_layers; ++l) {
    const int fi = l == 0 ? c.n_in : c.n_hidden;
    const int fo = l == c.n_layers ? c.n_out : c.n_hidden;
    c.fan_in.push_back(fi);
    c.fan_out.push_back(fo);
    c.w_off.push_back(off);
    off += (int64_t)fi * fo;
    c.b_off.push_back(off);
    off += fo;
  }
  c.n_params = off;
  const int64_t wmax = std::max(std::max(c.n_hidden, c.n_out), c.n_in);
  bool ok = hipMalloc(&c.act, sizeof(float) * (size_t)std::max(1, c.n_layers) * c.max_batch * c.n_hidden) == hipSuccess &&
            hipMalloc(&c.dz, sizeof(float) * 2 * (size_t)c.max_batch * wmax) == hipSuccess &&
            hipMalloc(&c.colpart, sizeof(float) * scdg::kColChunks * (size_t)wmax) == hipSuccess &&
            hipMalloc(&c.red, sizeof(double) * 15 * scdg::kRedBlocks) == hipSuccess;
  if (!ok) {
    free_ctx(c);
    delete m;
    return SCDG_ERR_NOMEM;
  }
  *out = m;
  return SCDG_OK;
}

scdg_status scdg_mlp_destroy(scdg_mlp *m) {
  if (!m) return SCDG_OK;
  (void)hipStreamSynchronize(m->c.stream);
  free_ctx(m->c);
  delete m;
  return SCDG_OK;
}

scdg_status scdg_mlp_set_compute(scdg_mlp *m, int32_t mode) {
  if (!m || (mode != SCDG_MLP_FP32 && mode != SCDG_MLP_BF16)) return SCDG_ERR_ARG;
  m->c.bf16 = mode == SCDG_MLP_BF16;
  return SCDG_OK;
}

scdg_status scdg_mlp_param_count(const scdg_mlp *m, int64_t *n) {
  if (!m || !n) return SCDG_ERR_ARG;
  *n = m->c.n_params;
  return SCDG_OK;
}

scdg_status scdg_mlp_forward(scdg_mlp *m, const float *w, const float *x, int32_t batch, float *y) {
  if (!m || !w || !x || !y || batch <= 0 || batch > m->c.max_batch) return SCDG_ERR_ARG;
  auto &c = m->c;
  const float *in = x;
  int ld_in = c.n_in;
  for (int l = 0; l <= c.n_layers; ++l) {
    const bool last = l == c.n_layers;
    float *out = last ? y : c.act + (size_t)l * c.max_batch * c.n_hidden;
    const int ld_out = last ? c.n_out : c.n_hidden;
    hipError_t e = scdg::gemm(false, false, batch, c.fan_out[l], c.fan_in[l], in, ld_in, w + c.w_off[l],
                              c.fan_out[l], out, ld_out, w + c.b_off[l],
                              last ? scdg::kEpiNone : scdg::kEpiTanh, nullptr, 0, c.bf16, c.stream);
    if (e != hipSuccess) return SCDG_ERR_HIP;
    in = out;
    ld_in = ld_out;
  }
  c.last_batch = batch;
  return SCDG_OK;
}

scdg_status scdg_mlp_backward(scdg_mlp *m, const float *w, const float *x, const float *dy, int32_t batch,
                              float *dw, float *dx) {
  if (!m || !w || !x || !dy || !dw || batch <= 0) return SCDG_ERR_ARG;
  auto &c = m->c;
  if (batch != c.last_batch) return SCDG_ERR_STATE;  // activations belong to another batch
  const int64_t wmax = std::max(std::max(c.n_hidden, c.n_out), c.n_in);
  float *buf[2] = {c.dz, c.dz + (size_t)c.max_batch * wmax};
  const float *dz = dy;   // gradient with respect to the pre-activation of layer l
  int cur = 0;
  for (int l = c.n_layers; l >= 0; --l) {
    const float *a_prev = l == 0 ? x : c.act + (size_t)(l - 1) * c.max_batch * c.n_hidden;
    const int fi = c.fan_in[l], fo = c.fan_out[l];
    // dW_l = A_{l-1}^T dZ_l  [fi x fo]
    hipError_t e = scdg::gemm(true, false, fi, fo, batch, a_prev, fi, dz, fo, dw + c.w_off[l], fo, nullptr,
                              scdg::kEpiNone, nullptr, 0, c.bf16, c.stream);
    if (e != hipSuccess) return SCDG_ERR_HIP;
    // db_l = column sums of dZ_l
    hipLaunchKernelGGL(scdg::colsum_partial_kernel, dim3((fo + 255) / 256, scdg::kColChunks), dim3(256), 0,
                       c.stream, dz, batch, fo, c.colpart);
    hipLaunchKernelGGL(scdg::colsum_final_kernel, dim3((fo + 255) / 256), dim3(256), 0, c.stream, c.colpart,
                       fo, dw + c.b_off[l]);
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l^T) * (1 - A_{l-1}^2)
      float *next = buf[cur];
      e = scdg::gemm(false, true, batch, fi, fo, dz, fo, w + c.w_off[l], fo, next, fi, nullptr,
                     scdg::kEpiNone, a_prev, fi, c.bf16, c.stream);
      if (e != hipSuccess) return SCDG_ERR_HIP;
      dz = next;
      cur ^= 1;
    } else if (dx) {
      e = scdg::gemm(false, true, batch, fi, fo, dz, fo, w + c.w_off[l], fo, dx, fi, nullptr, scdg::kEpiNone,
                     nullptr, 0, c.bf16, c.stream);
      if (e != hipSuccess) return SCDG_ERR_HIP;
    }
  }
  return hip_status(hipGetLastError());
}

scdg_status scdg_mlp_adam(scdg_mlp *m, float *w, const float *dw, float *m1, float *m2, float lr, float beta1,
                          float beta2, float eps, int32_t step) {
  if (!m || !w || !dw || !m1 || !m2 || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return SCDG_ERR_ARG;
  auto &c = m->c;
  const float corr1 = 1.f - powf(beta1, (float)step), corr2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(scdg::adam_kernel, dim3(scdg::grid_for(c.n_params)), dim3(256), 0, c.stream, w, dw, m1,
                     m2, c.n_params, lr, beta1, beta2, eps, corr1, corr2);
  return hip_status(hipGetLastError());
}

scdg_status scdg_mlp_mse(scdg_mlp *m, const float *y, const float *t, int64_t n, float *dy, double *loss) {
  if (!m || !y || !t || !loss || n <= 0) return SCDG_ERR_ARG;
  auto &c = m->c;
  hipLaunchKernelGGL(scdg::mse_partial_kernel, dim3(scdg::kRedBlocks), dim3(256), 0, c.stream, y, t, n, dy,
                     c.red);
  hipLaunchKernelGGL(scdg::sum_final_kernel, dim3(1), dim3(64), 0, c.stream, c.red, scdg::kRedBlocks, 1,
                     1.0 / (double)n, loss);
  return hip_status(hipGetLastError());
}

scdg_status scdg_mlp_gather(scdg_mlp *m, const float *src, int32_t width, const int32_t *idx, int32_t count,
                            float *dst) {
  if (!m || !src || !idx || !dst || width <= 0 || count < 0) return SCDG_ERR_ARG;
  if (count == 0) return SCDG_OK;
  hipLaunchKernelGGL(scdg::gather_rows_kernel, dim3(scdg::grid_for((int64_t)count * width)), dim3(256), 0,
                     m->c.stream, src, width, idx, count, dst);
  return hip_status(hipGetLastError());
}

scdg_status scdg_guess_stats(scdg_mlp *m, const double *q, const double *dq_prev, const double *dq,
                             const double *r, int64_t n_dof, double *stats) {
  if (!m || !q || !dq_prev || !stats || n_dof <= 0 || n_dof % 5) return SCDG_ERR_ARG;
  auto &c = m->c;
  const int64_t nodes = n_dof / 5;
  hipLaunchKernelGGL(scdg::stats_partial_kernel, dim3(scdg::kRedBlocks), dim3(256), 0, c.stream, q, dq_prev,
                     nullptr, r, nullptr, nodes, c.red);
  hipLaunchKernelGGL(scdg::stats_final_kernel, dim3(1), dim3(64), 0, c.stream, c.red, scdg::kRedBlocks, nodes,
                     1, 0, stats);
  hipLaunchKernelGGL(scdg::stats_partial_kernel, dim3(scdg::kRedBlocks), dim3(256), 0, c.stream, q, dq_prev,
                     dq, nullptr, stats, nodes, c.red);
  hipLaunchKernelGGL(scdg::stats_final_kernel, dim3(1), dim3(64), 0, c.stream, c.red, scdg::kRedBlocks, nodes,
                     2, dq ? 1 : 0, stats);
  return hip_status(hipGetLastError());
}

scdg_status scdg_guess_features(scdg_mlp *m, const double *q, const double *dq_prev, const double *r,
                                const double *stats, int32_t n_elem, float *x) {
  if (!m || !q || !dq_prev || !stats || !x || n_elem <= 0) return SCDG_ERR_ARG;
  auto &c = m->c;
  const int dpe = c.n_out;
  const int nb = c.n_in / dpe;
  if (dpe % 5 || c.n_in != nb * dpe || (nb != 2 && nb != 3) || (nb == 3 && !r)) return SCDG_ERR_ARG;
  hipLaunchKernelGGL(scdg::features_kernel, dim3(scdg::grid_for((int64_t)n_elem * dpe)), dim3(256), 0,
                     c.stream, q, dq_prev, r, stats, (int64_t)n_elem, dpe, nb, x);
  return hip_status(hipGetLastError());
}

scdg_status scdg_guess_target(scdg_mlp *m, const double *dq, const double *dq_prev, const double *stats,
                              int32_t n_elem, float *t) {
  if (!m || !dq || !dq_prev || !stats || !t || n_elem <= 0) return SCDG_ERR_ARG;
  auto &c = m->c;
  const int64_t n = (int64_t)n_elem * c.n_out;
  hipLaunchKernelGGL(scdg::target_kernel, dim3(scdg::grid_for(n)), dim3(256), 0, c.stream, dq, dq_prev, stats,
                     n, t);
  return hip_status(hipGetLastError());
}

scdg_status scdg_guess_apply(scdg_mlp *m, const double *dq_prev, const float *y, const double *stats,
                             int32_t n_elem, double *dq) {
  if (!m || !dq_prev || !y || !stats || !dq || n_elem <= 0) return SCDG_ERR_ARG;
  auto &c = m->c;
  const int64_t n = (int64_t)n_elem * c.n_out;
  hipLaunchKernelGGL(scdg::apply_kernel, dim3(scdg::grid_for(n)), dim3(256), 0, c.stream, dq_prev, y, stats, n,
                     dq);
  return hip_status(hipGetLastError());
}

}  // extern "C"
