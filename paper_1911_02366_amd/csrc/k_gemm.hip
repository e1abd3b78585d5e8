// Batched (grouped) dense GEMM on the CDNA4 matrix cores, FP64 and FP32:
//   C_p = alpha A_p B_p + beta C_p    for every problem p of the batch,
// row-major operands with per-problem sizes and leading dimensions.
//
// It forms X_e = A_ii(e)^-1 A_ib(e) and the element blocks T_e = F_e - A_bi(e) X_e
// of the condensed matrix (eq. SC_step1; F_e the A_bb node blocks folded into
// the element, added from a per-element map in the epilogue, so T_e is written
// once), and the trailing updates of the dense LU of S.
//
// Tiling: a workgroup computes a BM x BN tile of one problem; its waves form a
// WM x WN grid, each owning (BM/WM) x (BN/WN) as a block of 16x16x4 MFMAs.  K advances in steps of 16: the next A and B slabs are loaded
// into registers (coalesced: consecutive lanes read consecutive addresses)
// while the current slabs, double-buffered in LDS, feed the matrix cores.  A is
// stored k-major in LDS so the 16 lanes of one MFMA operand column read
// consecutive words.  The tile list orders tiles so that one problem's tiles
// share an XCD (workgroups are dealt to the 8 XCDs round-robin), keeping an
// element's operands in that XCD's L2.
#include <type_traits>

#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int BK = 16;

template <typename T, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm_batched_kernel(const GemmDesc *__restrict__ desc,
                                                                const int32_t *__restrict__ tiles,
                                                                const T *__restrict__ A,
                                                                const T *__restrict__ B,
                                                                T *__restrict__ C, T alpha, T beta,
                                                                const int32_t *__restrict__ fmap,
                                                                const double *__restrict__ fval) {
  using M = Mfma<T>;
  constexpr int kThreads = 64 * WM * WN;
  constexpr int PA = BM + 4;             // LDS row strides (padding against bank conflicts)
  constexpr int PB = BN + 4;
  constexpr int WTM = BM / WM, WTN = BN / WN;          // wave tile
  constexpr int TM = WTM / 16, TN = WTN / 16;          // MFMA blocks per wave
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((BM * BK) % kThreads == 0 && kThreads % BK == 0, "A slab split");
  static_assert((BN * BK) % kThreads == 0 && kThreads % BN == 0, "B slab split");
  constexpr int A_ELEMS = BM * BK / kThreads;          // per-thread slab loads
  constexpr int B_ELEMS = BN * BK / kThreads;
  constexpr int A_ROWS_PER_STEP = kThreads / BK;       // rows of A covered per load step
  constexpr int B_ROWS_PER_STEP = kThreads / BN;       // k rows of B covered per load step
  __shared__ T as[2][BK][PA];
  __shared__ T bs[2][BK][PB];

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
  const int wm = wid / WN, wn = wid % WN;

  // A slab: lane t reads k = t % 16 of rows t / 16 + step * 16
  const int a_k = tid % BK, a_r = tid / BK;
  // B slab: lane t reads column t % BN of k rows t / BN + step * (threads / BN)
  const int b_c = tid % BN, b_k = tid / BN;

  T ra[A_ELEMS], rb[B_ELEMS];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_ELEMS; ++u) {
      const int row = m0 + a_r + u * A_ROWS_PER_STEP, k = k0 + a_k;
      ra[u] = (row < d.m && k < d.k) ? a[(int64_t)row * d.lda + k] : T(0);
    }
#pragma unroll
    for (int u = 0; u < B_ELEMS; ++u) {
      const int k = k0 + b_k + u * B_ROWS_PER_STEP, col = n0 + b_c;
      rb[u] = (k < d.k && col < d.n) ? b[(int64_t)k * d.ldb + col] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < A_ELEMS; ++u) as[buf][a_k][a_r + u * A_ROWS_PER_STEP] = ra[u];
#pragma unroll
    for (int u = 0; u < B_ELEMS; ++u) bs[buf][b_k + u * B_ROWS_PER_STEP][b_c] = rb[u];
  };

  typename M::acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = M::zero();

  // 16x16 blocks of this wave's tile that hold real rows / columns: blocks lying
  // wholly in the zero padding of a ragged tile skip their MFMAs (wave-uniform)
  const int tm_valid = min(TM, max(0, (d.m - (m0 + wm * WTM) + 15) / 16));
  const int tn_valid = min(TN, max(0, (d.n - (n0 + wn * WTN) + 15) / 16));
  const int nk = (d.k + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  // the K loop is compiled twice: without per-block guards for a wave whose
  // blocks all hold real rows and columns (every wave but those on the ragged
  // edge), so the matrix-core instructions issue back to back with the LDS
  // reads scheduled around them, and with the guards for the others
  auto kloop = [&](auto full_c) {
    constexpr bool FULL = decltype(full_c)::value;
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          af[i] = as[buf][kk + (lane >> 4)][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bf[j] = bs[buf][kk + (lane >> 4)][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (FULL || (i < tm_valid && j < tn_valid)) acc[i][j] = M::mma(af[i], bf[j], acc[i][j]);
      }
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  };
  if (tm_valid == TM && tn_valid == TN)
    kloop(std::true_type{});
  else
    kloop(std::false_type{});

  // the folded A_bb node blocks of this problem's C (Schur GEMM only): the
  // tile's part of the fold map is staged in LDS (free after the K loop), and
  // for each row group of 16 the epilogue first issues every fold-value load
  // of its entries (entries without a fold read block 0, which exists when the
  // tile has any fold, and discard it), then adds and stores, so the loads are
  // in flight together
  const bool fold = fmap != nullptr && d.f_off >= 0;
  int *fm_s = reinterpret_cast<int *>(&as[0][0][0]);
  const int rb0 = m0 / 5, cb0 = n0 / 5;
  const int frw = (min(m0 + BM, d.m) - 1) / 5 - rb0 + 1, fcw = (min(n0 + BN, d.n) - 1) / 5 - cb0 + 1;
  static_assert((BM / 5 + 2) * (BN / 5 + 2) * sizeof(int) <= sizeof(as), "fold map tile fits in LDS");
  bool tile_fold = false;
  if (fold) {
    const int32_t *__restrict__ fm = fmap + d.f_off;
    const int fbn = d.n / 5;
    int any = 0;
    for (int q = threadIdx.x; q < frw * fcw; q += kThreads) {
      const int a = q / fcw, b = q - a * fcw;
      const int32_t f = fm[(int64_t)(rb0 + a) * fbn + cb0 + b];
      fm_s[q] = f;
      any |= f >= 0;
    }
    tile_fold = __syncthreads_or(any) != 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    double fv[TN][4];
    int fok = 0;   // bit 4 j + r: entry (j, r) has a folded value
    if (tile_fold) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * WTN + j * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WTM + i * 16 + M::row(lane, r);
          int f = -1, off = 0;
          if (col < d.n && row < d.m) {
            const int rb = row / 5, cb = col / 5;
            f = fm_s[(rb - rb0) * fcw + cb - cb0];
            off = (row - 5 * rb) * 5 + (col - 5 * cb);
          }
          fok |= (f >= 0 ? 1 : 0) << (4 * j + r);
          fv[j][r] = fval[(int64_t)(f >= 0 ? f : 0) * 25 + (f >= 0 ? off : 0)];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * WTN + j * 16 + (lane & 15);
      if (col >= d.n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + i * 16 + M::row(lane, r);
        if (row < d.m) {
          T *dst = c + (int64_t)row * d.ldc + col;
          T v = alpha * acc[i][j][r];
          if (beta != T(0)) v += beta * (*dst);
          if ((fok >> (4 * j + r)) & 1) v = (T)((double)v + fv[j][r]);
          *dst = v;
        }
      }
    }
  }
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_cfg(const GemmDesc *d_desc, const int32_t *d_tiles, int32_t n_tiles,
                      const void *a, const void *b, void *c, double alpha, double beta, bool fp32,
                      hipStream_t s, const int32_t *fmap, const double *fval) {
  const dim3 block(64 * WM * WN);
  if (fp32) {
    hipLaunchKernelGGL((gemm_batched_kernel<float, BM, BN, WM, WN>), dim3(n_tiles), block, 0, s,
                       d_desc, d_tiles, static_cast<const float *>(a), static_cast<const float *>(b),
                       static_cast<float *>(c), (float)alpha, (float)beta, fmap, fval);
  } else {
    hipLaunchKernelGGL((gemm_batched_kernel<double, BM, BN, WM, WN>), dim3(n_tiles), block, 0, s,
                       d_desc, d_tiles, static_cast<const double *>(a), static_cast<const double *>(b),
                       static_cast<double *>(c), alpha, beta, fmap, fval);
  }
  return hipGetLastError();
}

}  // namespace

// Tile configurations: C tile rows x columns and the wave grid.
//   0: 64x64 (2x2 waves)    1: 64x128 (2x2)    2: 128x128 (2x2)
//   3: 128x128 (2x4 waves)  4: 128x64 (2x2)    5: 240x80 (5x1; divides 1200 = n_c at N = 5)
//   6: 80x80 (5x1 waves)   7: 256x128 (4x2 waves)   8: 128x256 (2x4 waves)
void gemm_tile_shape(int cfg, int *bm, int *bn) {
  static const int shapes[kGemmConfigs][2] = {{64, 64}, {64, 128}, {128, 128}, {128, 128}, {128, 64},
                                              {240, 80}, {80, 80},          {256, 128}, {128, 256}};
  if (cfg < 0 || cfg >= kGemmConfigs) cfg = 0;
  *bm = shapes[cfg][0];
  *bn = shapes[cfg][1];
}

hipError_t launch_gemm_batched(int cfg, const GemmDesc *d_desc, const int32_t *d_tiles,
                               int32_t n_tiles, const void *a, const void *b, void *c, double alpha,
                               double beta, bool fp32, hipStream_t s, const int32_t *fold_map,
                               const double *fold_val) {
  if (n_tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 1: return launch_cfg<64, 128, 2, 2>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 2: return launch_cfg<128, 128, 2, 2>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 3: return launch_cfg<128, 128, 2, 4>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 4: return launch_cfg<128, 64, 2, 2>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 5: return launch_cfg<240, 80, 5, 1>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 6: return launch_cfg<80, 80, 5, 1>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 7: return launch_cfg<256, 128, 4, 2>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    case 8: return launch_cfg<128, 256, 2, 4>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
    default: return launch_cfg<64, 64, 2, 2>(d_desc, d_tiles, n_tiles, a, b, c, alpha, beta, fp32, s, fold_map, fold_val);
  }
}

}  // namespace scdg
