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
#include <algorithm>

#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kRowsPerThread = 3;    // rows owned per thread (n <= 1536)
constexpr int kGroup = 2;            // output tiles per wave in flight (keeps VGPRs <= 128: two workgroups per CU)

// LDS layout of one element's workgroup: panel width NB, panel row stride PS
// (padded against bank conflicts; the compact layouts use NB + 1), the number
// of columns per update chunk, and whether the pivot permutation is kept in
// LDS (the single-kernel form) or in global memory (the blocked form).
template <typename T_, int NB_, int PS_, int CHUNK_, bool PERM_>
struct GjLayout {
  using T = T_;
  static constexpr int NB = NB_, PS = PS_, CHUNK = CHUNK_, RSTRIDE = CHUNK_ + 16;
  static constexpr bool PERM = PERM_;
  static size_t lds_bytes(int max_n) {
    const int rp = (max_n + 15) & ~15;
    return sizeof(T) * ((size_t)rp * PS + (size_t)NB * RSTRIDE + 2 * NB) +
           (PERM ? sizeof(int) * 2 * (size_t)rp : 0) + (size_t)rp;
  }
};

template <typename T, int NB, bool PERM>
using GjWide = GjLayout<T, NB, NB + (sizeof(T) == 8 ? 2 : 4), 64, PERM>;
template <typename T, int NB, bool PERM>
using GjCompact = GjLayout<T, NB, NB + 1, 32, PERM>;
// 24 columns with 32-column update chunks: the widest FP64 panel with which
// two n_i = 320 workgroups share a CU (79 KB of LDS each)
template <typename T, bool PERM>
using GjWide24 = GjLayout<T, 24, 26, 32, PERM>;

// Shared memory of one element's workgroup: the panel (all rows x NB columns),
// a chunk of the panel's pivot rows, the parked pivot rows, pivot bookkeeping.
template <class L>
struct GjSmem {
  using T = typename L::T;
  T *pnl;             // [rp][PS]
  T *rl;              // [NB][RSTRIDE]
  T *pend_buf;        // [2][NB] parked pivot rows
  int *piv;           // [rp] pivot row of column k (single-kernel form only)
  int *qinv;          // [rp] column whose pivot row is m (single-kernel form only)
  unsigned char *inpanel;  // [rp] row is a pivot row of the current panel
  __device__ GjSmem(unsigned char *smem, int rp) {
    pnl = reinterpret_cast<T *>(smem);
    rl = pnl + (size_t)rp * L::PS;
    pend_buf = rl + L::NB * L::RSTRIDE;
    piv = reinterpret_cast<int *>(pend_buf + 2 * L::NB);
    qinv = piv + (L::PERM ? rp : 0);
    inpanel = reinterpret_cast<unsigned char *>(qinv + (L::PERM ? rp : 0));
  }
};

// Eliminate the panel held in LDS (columns kb .. kb + nbw - 1 of the matrix):
// for each column, the pivot is the largest |a| among rows not yet used
// (lowest row on ties); the pivot row is scaled and the column eliminated from
// every other row (Gauss-Jordan).  One barrier per column: a pivot row is read
// by every thread right after the barrier, so its owner parks the scaled row in
// a side buffer (alternating by column parity) and writes it back after the
// next column's barrier, applying that column's elimination.  piv (LDS or
// global) receives the pivot row of each column; used[] marks the rows this
// thread owns that have served as pivots.
template <class L>
__device__ void gj_eliminate(GjSmem<L> &sm, int n, int kb, int nbw, bool (&used)[kRowsPerThread],
                             int *piv, unsigned char *flags, int &my_info, double (*red_v)[kWaves],
                             int (*red_i)[kWaves]) {
  using T = typename L::T;
  constexpr int NB = L::NB, PS = L::PS;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T *pnl = sm.pnl;
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
      sm.inpanel[pr] = 1;
      if (flags) flags[pr] = 1;
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
      const T *pend = sm.pend_buf + (par ^ 1) * NB;
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
        T *pend = sm.pend_buf + par * NB;
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
    const T *pend = sm.pend_buf + ((nbw - 1) & 1) * NB;
    T *row = pnl + pend_row * PS;
#pragma unroll
    for (int j = 0; j < NB; ++j) row[j] = pend[j];
  }
  __syncthreads();
}

// Rank-NB update of the columns [j_lo, j_hi) outside the panel:
//   W[i][j] <- (i pivot row of this panel ? 0 : W[i][j]) + sum_c P[i][c] R[c][j]
// with P the transformed panel (LDS) and R the panel's pivot rows read from src
// (a0 in double on the first panel of the single-kernel form, else w).
template <class L>
__device__ void gj_update(GjSmem<L> &sm, const double *__restrict__ a0, bool first, typename L::T *__restrict__ w,
                          int n, int kb, int nbw, const int *piv, int j_lo, int j_hi) {
  using T = typename L::T;
  using M = Mfma<T>;
  constexpr int NB = L::NB, PS = L::PS, kChunk = L::CHUNK, kRStride = L::RSTRIDE;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rp = (n + 15) & ~15;
  const int row_tiles = rp / 16;
  constexpr int kColTiles = kChunk / 16;              // 16-column tiles per chunk
  constexpr int kRowLanes = kWaves / kColTiles;       // waves sharing a column tile
  const int ct = wid % kColTiles;
  const int rt0 = wid / kColTiles;  // row tiles rt0, rt0 + kRowLanes, ...
  for (int j0 = j_lo; j0 < j_hi; j0 += kChunk) {
    for (int idx = tid; idx < NB * kChunk; idx += kThreads) {
      const int c = idx / kChunk, jj = idx % kChunk, j = j0 + jj;
      T v = T(0);
      if (c < nbw && j < j_hi && !(j >= kb && j < kb + nbw)) {
        const int64_t at = (int64_t)piv[kb + c] * n + j;
        v = first ? (T)a0[at] : w[at];
      }
      sm.rl[c * kRStride + jj] = v;
    }
    __syncthreads();
    const int jc = j0 + ct * 16 + (lane & 15);
    const bool col_ok = jc < j_hi && !(jc >= kb && jc < kb + nbw);
    for (int rtb = rt0; rtb < row_tiles; rtb += kRowLanes * kGroup) {
      T old[kGroup][4];
      typename M::acc_t acc[kGroup];
#pragma unroll
      for (int g = 0; g < kGroup; ++g) {
        const int rt = rtb + kRowLanes * g;
        acc[g] = M::zero();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rt * 16 + M::row(lane, r);
          T v = T(0);
          if (col_ok && rt < row_tiles && i < n && !sm.inpanel[i])
            v = first ? (T)a0[(int64_t)i * n + jc] : w[(int64_t)i * n + jc];
          old[g][r] = v;
        }
      }
#pragma unroll
      for (int kk = 0; kk < NB; kk += 4) {
        const T bv = sm.rl[(kk + (lane >> 4)) * kRStride + ct * 16 + (lane & 15)];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
          const int rt = min(rtb + kRowLanes * g, row_tiles - 1);
          const T av = sm.pnl[(rt * 16 + (lane & 15)) * PS + kk + (lane >> 4)];
          acc[g] = M::mma(av, bv, acc[g]);
        }
      }
      if (col_ok) {
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
          const int rt = rtb + kRowLanes * g;
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
}

// Single-kernel form: one workgroup runs every panel of its element, updating
// all columns after each panel, then reads the inverse out.
template <class L>
__global__ __launch_bounds__(kThreads) void gj_inverse_kernel(const double *__restrict__ src,
                                                              typename L::T *__restrict__ work,
                                                              typename L::T *__restrict__ out,
                                                              const int32_t *__restrict__ n_arr,
                                                              const int64_t *__restrict__ off_arr,
                                                              const int32_t *__restrict__ elem_order,
                                                              int32_t *__restrict__ info) {
  using T = typename L::T;
  constexpr int NB = L::NB, PS = L::PS;
  static_assert(L::PERM, "the single-kernel form keeps the permutation in LDS");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_v[2][kWaves];
  __shared__ int red_i[2][kWaves];

  // elements in longest-first order: XCD blockIdx % 8 receives a balanced share
  const int e = elem_order[blockIdx.x];
  const int n = n_arr[e];
  const int64_t off = off_arr[e];
  const double *__restrict__ a0 = src + off;
  T *__restrict__ w = work + off;
  const int rp = (n + 15) & ~15;
  GjSmem<L> sm(smem, rp);

  const int tid = threadIdx.x;
  bool used[kRowsPerThread];
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) used[u] = false;
  for (int i = tid; i < rp; i += kThreads) sm.inpanel[i] = 0;
  int my_info = 0;

  for (int kb = 0; kb < n; kb += NB) {
    const int nbw = min(NB, n - kb);
    const bool first = kb == 0;
    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      T v = T(0);
      if (i < n && c < nbw) v = first ? (T)a0[(int64_t)i * n + c] : w[(int64_t)i * n + kb + c];
      sm.pnl[i * PS + c] = v;
    }
    __syncthreads();
    gj_eliminate<L>(sm, n, kb, nbw, used, sm.piv, nullptr, my_info, red_v, red_i);
    gj_update<L>(sm, a0, first, w, n, kb, nbw, sm.piv, 0, n);
    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      if (i < n && c < nbw) w[(int64_t)i * n + kb + c] = sm.pnl[i * PS + c];
    }
    for (int c = tid; c < nbw; c += kThreads) sm.inpanel[sm.piv[kb + c]] = 0;
    __syncthreads();
  }

  // read the inverse out through the pivot permutation
  for (int k = tid; k < n; k += kThreads) sm.qinv[sm.piv[k]] = k;
  __syncthreads();
  T *__restrict__ o = out + off;
  {
    const int lane = tid & 63, wave = tid >> 6;
    for (int k = wave; k < n; k += kWaves) {
      const T *__restrict__ row = w + (int64_t)sm.piv[k] * n;
      for (int m = lane; m < n; m += 64) o[(int64_t)k * n + m] = row[sm.qinv[m]];
    }
  }
  if (tid == 0) info[e] = my_info;
}

// ---------------------------------------------------------------------------
// Blocked form for large blocks.  Columns are taken in outer panels of
// kOuter; inside an outer panel, inner panels of NB columns are eliminated
// by gj_panel_kernel, which updates only the outer panel's other columns.
// The rest of the matrix then receives the outer panel's transformation at
// once, as the rank-kOuter update of the same formula,
//     W[i][j] <- (i pivot row of the outer panel ? 0 : W[i][j]) + sum_c P[i][c] R[c][j],
// a batched GEMM (W += P R) after gj_outer_gather_kernel has copied the
// transformed outer panel P, gathered its pivot rows R (zero inside the panel)
// and cleared those rows outside it.  The composition of the inner steps is
// the Gauss-Jordan transformation of the whole outer panel, so the result is
// the same elimination as the single-kernel form (same pivots), with the bulk
// of the flops in matrix-core GEMMs with K = kOuter.
// ---------------------------------------------------------------------------
constexpr int kOuter = kGjOuter;

template <typename T>
__global__ void gj_prepare_kernel(const double *__restrict__ src, T *__restrict__ work, int64_t total,
                                  unsigned char *__restrict__ flags, int64_t n_rows, int32_t *__restrict__ info,
                                  int n_elem) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    work[i] = (T)src[i];
    if (i < n_rows) flags[i] = 0;
    if (i < n_elem) info[i] = 0;
  }
}

template <class L>
__global__ __launch_bounds__(kThreads) void gj_panel_kernel(typename L::T *__restrict__ work,
                                                            const int32_t *__restrict__ n_arr,
                                                            const int64_t *__restrict__ off_arr,
                                                            const int64_t *__restrict__ voff_arr,
                                                            int32_t *__restrict__ piv_all,
                                                            unsigned char *__restrict__ flags_all,
                                                            int32_t *__restrict__ info, int kb, int ko) {
  using T = typename L::T;
  constexpr int NB = L::NB, PS = L::PS;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_v[2][kWaves];
  __shared__ int red_i[2][kWaves];
  const int e = blockIdx.x;
  const int n = n_arr[e];
  if (kb >= n) return;
  const int nbw = min(NB, n - kb);
  T *__restrict__ w = work + off_arr[e];
  int *piv = piv_all + voff_arr[e];
  unsigned char *flags = flags_all + voff_arr[e];
  const int rp = (n + 15) & ~15;
  GjSmem<L> sm(smem, rp);
  const int tid = threadIdx.x;
  bool used[kRowsPerThread];
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int i = tid + u * kThreads;
    used[u] = i < n ? flags[i] != 0 : true;
  }
  for (int i = tid; i < rp; i += kThreads) sm.inpanel[i] = 0;
  for (int idx = tid; idx < rp * NB; idx += kThreads) {
    const int i = idx / NB, c = idx % NB;
    T v = T(0);
    if (i < n && c < nbw) v = w[(int64_t)i * n + kb + c];
    sm.pnl[i * PS + c] = v;
  }
  __syncthreads();
  int my_info = 0;
  gj_eliminate<L>(sm, n, kb, nbw, used, piv, flags, my_info, red_v, red_i);
  gj_update<L>(sm, nullptr, false, w, n, kb, nbw, piv, ko, min(n, ko + kOuter));
  for (int idx = tid; idx < rp * NB; idx += kThreads) {
    const int i = idx / NB, c = idx % NB;
    if (i < n && c < nbw) w[(int64_t)i * n + kb + c] = sm.pnl[i * PS + c];
  }
  if (tid == 0 && my_info != 0 && info[e] == 0) info[e] = my_info;
}

// P[i][c] = W[i][ko + c];  R[c][j] = W[p_c][j] outside the outer panel (0 inside),
// and W[p_c][j] = 0 outside the outer panel.
template <typename T>
__global__ void gj_outer_gather_kernel(T *__restrict__ work, const int32_t *__restrict__ n_arr,
                                       const int64_t *__restrict__ off_arr, const int64_t *__restrict__ voff_arr,
                                       const int32_t *__restrict__ piv_all, T *__restrict__ pbuf,
                                       T *__restrict__ rbuf, int ko) {
  const int e = blockIdx.x;
  const int n = n_arr[e];
  if (ko >= n) return;
  const int nbo = min(kOuter, n - ko);
  T *__restrict__ w = work + off_arr[e];
  const int32_t *piv = piv_all + voff_arr[e] + ko;
  T *__restrict__ pb = pbuf + voff_arr[e] * kOuter;
  T *__restrict__ rb = rbuf + voff_arr[e] * kOuter;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  // panel copy, a wave per row
  for (int i = wave; i < n; i += waves)
    for (int c = lane; c < nbo; c += 64) pb[(int64_t)i * kOuter + c] = w[(int64_t)i * n + ko + c];
  // pivot rows, a wave per row (the panel columns themselves are not touched here)
  for (int c = wave; c < nbo; c += waves) {
    T *__restrict__ src = w + (int64_t)piv[c] * n;
    T *__restrict__ dst = rb + (int64_t)c * n;
    for (int j = lane; j < n; j += 64) {
      if (j >= ko && j < ko + nbo) {
        dst[j] = T(0);
      } else {
        dst[j] = src[j];
        src[j] = T(0);
      }
    }
  }
}

// A^-1[k][m] = W[p_k][q_m]
template <typename T>
__global__ __launch_bounds__(kThreads) void gj_readout_kernel(const T *__restrict__ work, T *__restrict__ out,
                                                              const int32_t *__restrict__ n_arr,
                                                              const int64_t *__restrict__ off_arr,
                                                              const int64_t *__restrict__ voff_arr,
                                                              const int32_t *__restrict__ piv_all) {
  __shared__ int pv[kRowsPerThread * kThreads];
  __shared__ int qinv[kRowsPerThread * kThreads];
  const int e = blockIdx.x;
  const int n = n_arr[e];
  const int32_t *piv = piv_all + voff_arr[e];
  for (int k = threadIdx.x; k < n; k += kThreads) {
    pv[k] = piv[k];
    qinv[piv[k]] = k;
  }
  __syncthreads();
  const T *__restrict__ w = work + off_arr[e];
  T *__restrict__ o = out + off_arr[e];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < n; k += kWaves) {
    const T *__restrict__ row = w + (int64_t)pv[k] * n;
    for (int m = lane; m < n; m += 64) o[(int64_t)k * n + m] = row[qinv[m]];
  }
}

template <class L>
hipError_t gj_launch(Plan &p, typename L::T *work, typename L::T *out) {
  const size_t lds = L::lds_bytes(p.max_ni);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(gj_inverse_kernel<L>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((gj_inverse_kernel<L>), dim3(p.n_elem), dim3(kThreads), lds, p.stream,
                     p.aii, work, out, p.d_inv_n, p.d_inv_off, p.d_inv_order, p.d_info);
  return hipGetLastError();
}

constexpr size_t kLdsLimit = 160 * 1024 - 512;

// the widest panel whose layout fits the LDS of one workgroup
template <typename T>
hipError_t gj_dispatch(Plan &p, T *work, T *out) {
  // the widest panel with which two workgroups share a CU (latency hiding beats
  // fewer passes over the block), else the widest that fits at all
  const int n = p.max_ni;
  if (GjWide<T, 32, true>::lds_bytes(n) <= kLdsLimit / 2) return gj_launch<GjWide<T, 32, true>>(p, work, out);
  if (sizeof(T) == 8 && GjWide24<T, true>::lds_bytes(n) <= kLdsLimit / 2)
    return gj_launch<GjWide24<T, true>>(p, work, out);
  if (GjWide<T, 16, true>::lds_bytes(n) <= kLdsLimit / 2) return gj_launch<GjWide<T, 16, true>>(p, work, out);
  if (GjWide<T, 32, true>::lds_bytes(n) <= kLdsLimit) return gj_launch<GjWide<T, 32, true>>(p, work, out);
  if (GjWide<T, 16, true>::lds_bytes(n) <= kLdsLimit) return gj_launch<GjWide<T, 16, true>>(p, work, out);
  return gj_launch<GjWide<T, 8, true>>(p, work, out);
}

template <class L>
hipError_t gj_blocked_run(Plan &p, typename L::T *work, typename L::T *out) {
  using T = typename L::T;
  const size_t lds = L::lds_bytes(p.max_ni);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(gj_panel_kernel<L>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  const int64_t total = p.off_ii[p.n_elem];
  const int64_t grid = std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL((gj_prepare_kernel<T>), dim3((unsigned)grid), dim3(256), 0, p.stream, p.aii, work, total,
                     p.d_gj_flag, p.sum_ni, p.d_info, p.n_elem);
  T *pbuf = static_cast<T *>(p.gj_pbuf), *rbuf = static_cast<T *>(p.gj_rbuf);
  for (int s = 0; s * kOuter < p.max_ni; ++s) {
    const int ko = s * kOuter;
    for (int kb = ko; kb < std::min(p.max_ni, ko + kOuter); kb += L::NB)
      hipLaunchKernelGGL((gj_panel_kernel<L>), dim3(p.n_elem), dim3(kThreads), lds, p.stream, work,
                         p.d_inv_n, p.d_inv_off, p.d_gj_voff, p.d_gj_piv, p.d_gj_flag, p.d_info, kb, ko);
    if (p.gj_ntiles[s] > 0) {
      hipLaunchKernelGGL((gj_outer_gather_kernel<T>), dim3(p.n_elem), dim3(512), 0, p.stream, work,
                         p.d_inv_n, p.d_inv_off, p.d_gj_voff, p.d_gj_piv, pbuf, rbuf, ko);
      err = launch_gemm_batched(p.gj_cfg, p.d_gj_desc + p.gj_desc_off[s], p.d_gj_tiles + 3 * p.gj_tile_off[s],
                                p.gj_ntiles[s], pbuf, rbuf, work, 1.0, 1.0, sizeof(T) == 4, p.stream);
      if (err != hipSuccess) return err;
    }
  }
  hipLaunchKernelGGL((gj_readout_kernel<T>), dim3(p.n_elem), dim3(kThreads), 0, p.stream, work, out, p.d_inv_n,
                     p.d_inv_off, p.d_gj_voff, p.d_gj_piv);
  return hipGetLastError();
}

// the widest inner panel that fits: padded layouts first, then the compact ones
template <typename T>
hipError_t gj_blocked_dispatch(Plan &p, T *work, T *out) {
  const int n = p.max_ni;
  // as in the single-kernel form: first the widest layout with which two
  // workgroups share a CU, then the widest that fits
  if (GjWide<T, 32, false>::lds_bytes(n) <= kLdsLimit / 2) return gj_blocked_run<GjWide<T, 32, false>>(p, work, out);
  if (GjCompact<T, 32, false>::lds_bytes(n) <= kLdsLimit / 2)
    return gj_blocked_run<GjCompact<T, 32, false>>(p, work, out);
  if (GjWide<T, 16, false>::lds_bytes(n) <= kLdsLimit / 2) return gj_blocked_run<GjWide<T, 16, false>>(p, work, out);
  if (GjCompact<T, 16, false>::lds_bytes(n) <= kLdsLimit / 2)
    return gj_blocked_run<GjCompact<T, 16, false>>(p, work, out);
  if (GjWide<T, 32, false>::lds_bytes(n) <= kLdsLimit) return gj_blocked_run<GjWide<T, 32, false>>(p, work, out);
  if (GjCompact<T, 32, false>::lds_bytes(n) <= kLdsLimit)
    return gj_blocked_run<GjCompact<T, 32, false>>(p, work, out);
  if (GjWide<T, 16, false>::lds_bytes(n) <= kLdsLimit) return gj_blocked_run<GjWide<T, 16, false>>(p, work, out);
  if (GjCompact<T, 16, false>::lds_bytes(n) <= kLdsLimit)
    return gj_blocked_run<GjCompact<T, 16, false>>(p, work, out);
  return gj_blocked_run<GjWide<T, 8, false>>(p, work, out);
}

}  // namespace

bool gj_supported(int max_n, bool fp32) {
  if (max_n > kRowsPerThread * kThreads) return false;
  return fp32 ? GjWide<float, 8, true>::lds_bytes(max_n) <= kLdsLimit
              : GjWide<double, 8, true>::lds_bytes(max_n) <= kLdsLimit;
}

hipError_t launch_gj_inverse(Plan &p, void *work, void *out, bool fp32) {
  if (fp32) return gj_dispatch<float>(p, static_cast<float *>(work), static_cast<float *>(out));
  return gj_dispatch<double>(p, static_cast<double *>(work), static_cast<double *>(out));
}

hipError_t launch_gj_inverse_blocked(Plan &p, void *work, void *out, bool fp32) {
  if (fp32) return gj_blocked_dispatch<float>(p, static_cast<float *>(work), static_cast<float *>(out));
  return gj_blocked_dispatch<double>(p, static_cast<double *>(work), static_cast<double *>(out));
}

}  // namespace scdg
