// Batched inversion of the interior blocks A_ii(e) by blocked Gauss-Jordan
// elimination with partial pivoting.
//
// The paper inverts every interior block independently with LU routines and
// uses A_ii^-1 in the Schur product and in both condensation steps
// (Section 3.2; eq. SC_step1, SC_step2).  Here one 512-thread workgroup owns one
// element and the pivoting is implicit: rows are never exchanged; each column's
// pivot row (largest |a| among rows not yet used as pivots, lowest row on ties)
// is recorded, and the inverse is read out at the end through that
// permutation.  With p_k the pivot row of column k and q = p^-1,
//     A^-1[k][m] = W[p_k][q_m],
// where W is the in-place Gauss-Jordan result (the eliminated column slot keeps
// the running inverse).
//
// Per panel of NB columns:
//   1. the panel (all rows) is loaded into LDS and eliminated column by column,
//      one workgroup barrier per column (the pivot reduction);
//   2. the other columns get the rank-NB update
//        W[i][j] <- (i pivot row of this panel ? 0 : W[i][j]) + sum_c P[i][c] R[c][j]
//      with P the transformed panel and R the panel's pivot rows, on the 16x16x4
//      matrix cores, five output tiles per wave in flight.
// The first panel reads A_ii directly (no separate copy).  Flops: 2 n^3 per
// element.  A zero or non-finite pivot is recorded LAPACK-style (info = column
// + 1) and replaced by 1 so the launch always completes.
#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 64;           // columns per update chunk
constexpr int kRStride = kChunk + 16;  // LDS row stride of the pivot-row chunk
constexpr int kRowsPerThread = 3;    // rows owned per thread (n <= 1536)
constexpr int kGroup = 5;            // output tiles per wave in flight

template <typename T>
constexpr int panel_stride(int nb) {
  return nb + (sizeof(T) == 8 ? 2 : 4);
}

template <typename T, int NB>
size_t gj_lds_bytes(int max_n) {
  const int rp = (max_n + 15) & ~15;
  return sizeof(T) * ((size_t)rp * panel_stride<T>(NB) + (size_t)NB * kRStride + 2 * NB) +
         sizeof(int) * 2 * (size_t)rp + (size_t)rp;
}

template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void gj_inverse_kernel(const double *__restrict__ src,
                                                              T *__restrict__ work,
                                                              T *__restrict__ out,
                                                              const int32_t *__restrict__ n_arr,
                                                              const int64_t *__restrict__ off_arr,
                                                              int32_t *__restrict__ info) {
  using M = Mfma<T>;
  constexpr int PS = panel_stride<T>(NB);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_v[2][kWaves];
  __shared__ int red_i[2][kWaves];

  const int e = blockIdx.x;
  const int n = n_arr[e];
  const int64_t off = off_arr[e];
  const double *__restrict__ a0 = src + off;
  T *__restrict__ w = work + off;
  const int rp = (n + 15) & ~15;
  T *pnl = reinterpret_cast<T *>(smem);           // [rp][PS]
  T *rl = pnl + (size_t)rp * PS;                   // [NB][kRStride]
  T *pend_buf = rl + NB * kRStride;                // [2][NB] parked pivot rows
  int *piv = reinterpret_cast<int *>(pend_buf + 2 * NB);   // [rp] pivot row of column k
  int *qinv = piv + rp;                            // [rp] column whose pivot row is m
  unsigned char *inpanel = reinterpret_cast<unsigned char *>(qinv + rp);  // [rp]

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  bool used[kRowsPerThread];
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) used[u] = false;
  for (int i = tid; i < rp; i += kThreads) inpanel[i] = 0;
  int my_info = 0;

  for (int kb = 0; kb < n; kb += NB) {
    const int nbw = min(NB, n - kb);
    const bool first = kb == 0;
    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      T v = T(0);
      if (i < n && c < nbw) v = first ? (T)a0[(int64_t)i * n + c] : w[(int64_t)i * n + kb + c];
      pnl[i * PS + c] = v;
    }
    __syncthreads();

    // One barrier per column: a pivot row is read by every thread right after
    // the barrier, so its owner parks the scaled row in a side buffer (LDS,
    // alternating by column parity) and writes it back into the panel after the
    // next column's barrier, applying that column's elimination.
    bool pend_valid = false;
    int pend_row = 0;
    for (int c = 0; c < nbw; ++c) {
      const int par = c & 1;
      double best = -1.0;
      int bi = n;
#pragma unroll
      for (int u = 0; u < kRowsPerThread; ++u) {
        const int i = tid + u * kThreads;
        if (i < n && !used[u]) {
          const double v = fabs((double)pnl[i * PS + c]);
          if (v > best) {
            best = v;
            bi = i;
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_v[par][wid] = best;
        red_i[par][wid] = bi;
      }
      __syncthreads();
      best = red_v[par][0];
      bi = red_i[par][0];
#pragma unroll
      for (int q = 1; q < kWaves; ++q)
        if (red_v[par][q] > best || (red_v[par][q] == best && red_i[par][q] < bi)) {
          best = red_v[par][q];
          bi = red_i[par][q];
        }
      const int pr = bi < n ? bi : 0;
      T d = pnl[pr * PS + c];
      if (tid == 0) {
        piv[kb + c] = pr;
        inpanel[pr] = 1;
      }
      if (!(d != T(0)) || !isfinite((double)d)) {
        if (my_info == 0) my_info = kb + c + 1;
        d = T(1);
      }
      const T inv_d = T(1) / d;
      T sp[NB];   // scaled pivot row
#pragma unroll
      for (int j = 0; j < NB; ++j) sp[j] = (j == c) ? inv_d : pnl[pr * PS + j] * inv_d;
      int handled = -1;   // the parked row of the previous column, written back here
      if (pend_valid) {
        const T *pend = pend_buf + (par ^ 1) * NB;
        const T f = pend[c];
        T *row = pnl + pend_row * PS;
#pragma unroll
        for (int j = 0; j < NB; ++j) row[j] = (j == c ? T(0) : pend[j]) - f * sp[j];
        pend_valid = false;
        handled = pend_row;
      }
#pragma unroll
      for (int u = 0; u < kRowsPerThread; ++u) {
        const int i = tid + u * kThreads;
        if (i >= n || i == handled) continue;
        if (i == pr) {
          used[u] = true;
          pend_valid = true;
          pend_row = i;
          T *pend = pend_buf + par * NB;
#pragma unroll
          for (int j = 0; j < NB; ++j) pend[j] = sp[j];
        } else {
          T *row = pnl + i * PS;
          const T f = row[c];
#pragma unroll
          for (int j = 0; j < NB; ++j) row[j] = (j == c ? T(0) : row[j]) - f * sp[j];
        }
      }
    }
    __syncthreads();
    if (pend_valid) {
      const T *pend = pend_buf + ((nbw - 1) & 1) * NB;
      T *row = pnl + pend_row * PS;
#pragma unroll
      for (int j = 0; j < NB; ++j) row[j] = pend[j];
    }
    __syncthreads();

    // rank-NB update of the columns outside the panel
    const int row_tiles = rp / 16;
    const int ct = wid & 3;           // 16-column tile of the chunk
    const int rt0 = wid >> 2;         // row tiles rt0, rt0 + 2, ...
    for (int j0 = 0; j0 < n; j0 += kChunk) {
      for (int idx = tid; idx < NB * kChunk; idx += kThreads) {
        const int c = idx / kChunk, jj = idx % kChunk, j = j0 + jj;
        T v = T(0);
        if (c < nbw && j < n && !(j >= kb && j < kb + nbw)) {
          const int64_t at = (int64_t)piv[kb + c] * n + j;
          v = first ? (T)a0[at] : w[at];
        }
        rl[c * kRStride + jj] = v;
      }
      __syncthreads();
      const int jc = j0 + ct * 16 + (lane & 15);
      const bool col_ok = jc < n && !(jc >= kb && jc < kb + nbw);
      for (int rtb = rt0; rtb < row_tiles; rtb += 2 * kGroup) {
        T old[kGroup][4];
        typename M::acc_t acc[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
          const int rt = rtb + 2 * g;
          acc[g] = M::zero();
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = rt * 16 + M::row(lane, r);
            T v = T(0);
            if (col_ok && rt < row_tiles && i < n && !inpanel[i])
              v = first ? (T)a0[(int64_t)i * n + jc] : w[(int64_t)i * n + jc];
            old[g][r] = v;
          }
        }
#pragma unroll
        for (int kk = 0; kk < NB; kk += 4) {
          const T bv = rl[(kk + (lane >> 4)) * kRStride + ct * 16 + (lane & 15)];
#pragma unroll
          for (int g = 0; g < kGroup; ++g) {
            const int rt = min(rtb + 2 * g, row_tiles - 1);
            const T av = pnl[(rt * 16 + (lane & 15)) * PS + kk + (lane >> 4)];
            acc[g] = M::mma(av, bv, acc[g]);
          }
        }
        if (col_ok) {
#pragma unroll
          for (int g = 0; g < kGroup; ++g) {
            const int rt = rtb + 2 * g;
            if (rt >= row_tiles) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = rt * 16 + M::row(lane, r);
              if (i < n) w[(int64_t)i * n + jc] = old[g][r] + acc[g][r];
            }
          }
        }
      }
      __syncthreads();
    }

    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      if (i < n && c < nbw) w[(int64_t)i * n + kb + c] = pnl[i * PS + c];
    }
    for (int c = tid; c < nbw; c += kThreads) inpanel[piv[kb + c]] = 0;
    __syncthreads();
  }

  // read the inverse out through the pivot permutation
  for (int k = tid; k < n; k += kThreads) qinv[piv[k]] = k;
  __syncthreads();
  T *__restrict__ o = out + off;
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += kThreads) {
    const int k = (int)(idx / n), m = (int)(idx % n);
    o[idx] = w[(int64_t)piv[k] * n + qinv[m]];
  }
  if (tid == 0) info[e] = my_info;
}

template <typename T, int NB>
hipError_t gj_launch(Plan &p, T *work, T *out) {
  const size_t lds = gj_lds_bytes<T, NB>(p.max_ni);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(gj_inverse_kernel<T, NB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((gj_inverse_kernel<T, NB>), dim3(p.n_elem), dim3(kThreads), lds, p.stream,
                     p.aii, work, out, p.d_inv_n, p.d_inv_off, p.d_info);
  return hipGetLastError();
}

constexpr size_t kLdsLimit = 160 * 1024 - 512;

template <typename T>
hipError_t gj_dispatch(Plan &p, T *work, T *out) {
  if (gj_lds_bytes<T, 32>(p.max_ni) <= kLdsLimit) return gj_launch<T, 32>(p, work, out);
  if (gj_lds_bytes<T, 16>(p.max_ni) <= kLdsLimit) return gj_launch<T, 16>(p, work, out);
  return gj_launch<T, 8>(p, work, out);
}

}  // namespace

bool gj_supported(int max_n, bool fp32) {
  if (max_n > kRowsPerThread * kThreads) return false;
  return fp32 ? gj_lds_bytes<float, 8>(max_n) <= kLdsLimit
              : gj_lds_bytes<double, 8>(max_n) <= kLdsLimit;
}

hipError_t launch_gj_inverse(Plan &p, void *work, void *out, bool fp32) {
  if (fp32) return gj_dispatch<float>(p, static_cast<float *>(work), static_cast<float *>(out));
  return gj_dispatch<double>(p, static_cast<double *>(work), static_cast<double *>(out));
}

}  // namespace scdg
