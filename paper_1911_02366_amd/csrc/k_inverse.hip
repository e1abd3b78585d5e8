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
#include <type_traits>

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
// Resident-panel form (n_i <= kResMaxN).  One workgroup per element, as in the
// single-kernel form, but the LDS holds an outer panel of NBO columns (48 in
// FP64, 64 in FP32), so the rest of the block in global memory is read and
// written once per NBO columns instead of once per 24 or 32.
//   * The block is bordered to rp = n rounded up to 16 with an identity block
//     (rows and columns n..rp-1).  Its inverse is the inverse of A bordered
//     with the same identity, the border never mixes with A (its rows and
//     columns stay zero outside the diagonal block, and no row of the border
//     can win a pivot search of a column of A while a row of A is unused), and
//     every inner panel is a whole 16 columns.
//   * Inside the outer panel, inner panels of 16 columns are eliminated by the
//     first four waves, each lane holding two rows (128 w + l and
//     128 w + 64 + l) in registers.  One barrier per column: each wave finds
//     its candidate pivot (the largest |a| among its unused rows, lowest row
//     on ties) with DPP row reductions and ballots, and the winning lane
//     publishes its 16-value row next to the candidate value, so the row
//     that wins is read straight from LDS after the barrier.
//   * The inner panel's transformation reaches the other columns of the outer
//     panel as a rank-16 update on the matrix cores, inside LDS.
//   * The outer panel's transformation reaches the rest of the block as one
//     rank-NBO matrix-core pass: every wave loads the outer panel's pivot rows
//     for its column tiles into registers (the B operands) before a barrier,
//     after which those rows may be overwritten, then streams its contiguous
//     share of the output tiles (A operands from the LDS panel), loading the
//     next group of tiles while the matrix cores work on the current one.
// Same formulas, pivot rule and read-out as the single-kernel form.
// ---------------------------------------------------------------------------
constexpr int kResThreads = 512;
constexpr int kResWaves = kResThreads / 64;
constexpr int kResElimWaves = 4;                     // waves holding rows during the column steps
constexpr int kResMaxN = 400;                        // 25 column tiles; 2 rows per lane of 4 waves
constexpr int kResInner = 16;

// column tiles one wave's contiguous share of an outer pass can span: its
// share is at most ceil(out / W) tiles in column-major order over n_rt-tile
// columns, so it spans at most floor(out / W) + 2 column tiles, with out the
// column tiles outside the outer panel (worst case over every padded size)
constexpr int res_slots(int panel_tiles, int max_tiles, int waves) {
  int worst = 0;
  for (int nt = 1; nt <= max_tiles; ++nt)
    for (int kt = 0; kt < nt; kt += panel_tiles) {
      const int pt = panel_tiles < nt - kt ? panel_tiles : nt - kt;
      worst = worst > nt - pt ? worst : nt - pt;
    }
  return worst / waves + 2;
}

template <typename T_, int NBO_, int G_, int MAXN_, int NT_ = kResThreads>
struct GjRes {
  using T = T_;
  static constexpr int NBO = NBO_, G = G_, MAXN = MAXN_, NT = NT_, W = NT_ / 64;
  static constexpr int SLOTS = res_slots(NBO_ / 16, (MAXN_ + 15) / 16, NT_ / 64);
  static_assert(NT_ >= 64 * kResElimWaves && MAXN_ <= 128 * kResElimWaves, "rows held two per lane by four waves");
  static constexpr int PS = NBO_ + (sizeof(T_) == 8 ? 2 : 4);   // 100 / 68 dwords at FP64 48 / FP32 64: conflict-free A reads
  static size_t lds_bytes(int max_n) {
    const size_t rp = (size_t)((max_n + 15) & ~15);
    return sizeof(T) * (rp * PS + 2 * kResElimWaves * kResInner + 4 * kResElimWaves) +
           sizeof(int) * (2 * kResElimWaves + 2 * rp) + rp;
  }
};

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// maximum over the 64 lanes (no NaN among the inputs), uniform
template <typename T>
__device__ __forceinline__ T wave_max_dpp(T v) {
  v = fmax(v, dpp_mov<0xB1>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_mov<0x4E>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_mov<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_mov<0x140>(v));   // row_mirror: every lane holds its 16-lane row's maximum
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// search value of a row: |a| if unused, -1 if used; a NaN wins (and is then
// reported as a bad pivot)
template <typename T>
__device__ __forceinline__ T pivot_key(T a, bool live) {
  T v = live ? fabs(a) : T(-1);
  return v != v ? T(INFINITY) : v;
}

template <class L>
__global__ __launch_bounds__(L::NT) void gj_resident_kernel(const double *__restrict__ src,
                                                                  typename L::T *__restrict__ work,
                                                                  typename L::T *__restrict__ out,
                                                                  const int32_t *__restrict__ n_arr,
                                                                  const int64_t *__restrict__ off_arr,
                                                                  const int32_t *__restrict__ elem_order,
                                                                  int32_t *__restrict__ info) {
  using T = typename L::T;
  using M = Mfma<T>;
  constexpr int NBO = L::NBO, PS = L::PS, G = L::G, W = L::W, NT = L::NT, EW = kResElimWaves, NI = kResInner;
  constexpr int NQ = NBO / 4;                                          // K steps of the outer pass
  constexpr int NLD = (L::MAXN * NBO + NT - 1) / NT;                   // panel values per thread
  constexpr int NLB = NLD < 40 ? NLD : 40;                             // loaded per batch
  constexpr int SL = L::SLOTS;
  extern __shared__ __align__(16) unsigned char smem[];

  const int e = elem_order[blockIdx.x];
  const int n = n_arr[e];
  const int64_t off = off_arr[e];
  const double *__restrict__ a0 = src + off;
  T *__restrict__ w = work + off;
  const int rp = (n + 15) & ~15;
  const int n_rt = rp / 16, n_ct = rp / 16;

  T *pnl = reinterpret_cast<T *>(smem);          // [rp][PS] outer panel
  T *cand_row = pnl + (size_t)rp * PS;           // [2][EW][NI] candidate rows
  T *cand_v = cand_row + 2 * EW * NI;             // [2][EW] candidate |a|
  T *cand_inv = cand_v + 2 * EW;                  // [2][EW] reciprocal of the candidate pivot
  int *cand_r = reinterpret_cast<int *>(cand_inv + 2 * EW);   // [2][EW] candidate row
  int *piv = cand_r + 2 * EW;                     // [rp] pivot row of each column
  int *qinv = piv + rp;                           // [rp] column whose pivot row is m
  unsigned char *pflag = reinterpret_cast<unsigned char *>(qinv + rp);  // [rp] inner panel + 1 if a pivot row of this outer panel

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const bool elim = wid < EW;
  const int r0 = 128 * wid + lane, r1 = r0 + 64;   // rows held during the column steps (waves 0..3)
  const bool own0 = elim && r0 < rp, own1 = elim && r1 < rp;
  bool used0 = false, used1 = false;
  int my_info = 0;

  for (int kb = 0; kb < rp; kb += NBO) {
    const int nbo = min(NBO, rp - kb);
    const bool first = kb == 0;
    // load the outer panel (all loads in flight before the LDS stores); the
    // border holds the identity
    {
      // the thread index passes through an empty asm statement so that the
      // per-value indices are formed here, not hoisted out of the kb loop and
      // kept live across the whole kernel
#pragma unroll 1
      for (int u0 = 0; u0 < NLD; u0 += NLB) {
        int tl = tid + u0 * NT;
        asm volatile("" : "+v"(tl));
        T tmp[NLB];
#pragma unroll
        for (int u = 0; u < NLB; ++u) {
          const int idx = tl + u * NT;
          const int i = idx / NBO, c = idx % NBO, col = kb + c;
          T v = T(0);
          if (idx < rp * NBO) {
            if (i < n && col < n)
              v = first ? (T)a0[(int64_t)i * n + col] : w[(int64_t)i * n + col];
            else if (col >= n && col < rp && i == col)
              v = T(1);
          }
          tmp[u] = v;
        }
#pragma unroll
        for (int u = 0; u < NLB; ++u) {
          const int idx = tl + u * NT;
          if (idx < rp * NBO) pnl[(idx / NBO) * PS + idx % NBO] = tmp[u];
        }
      }
    }
    for (int i = tid; i < rp; i += NT) pflag[i] = 0;
    __syncthreads();

    for (int c0 = 0; c0 < nbo; c0 += NI) {
      const int sp1 = c0 / NI + 1;
      T x0[NI], x1[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        x0[j] = own0 ? pnl[r0 * PS + c0 + j] : T(0);
        x1[j] = own1 ? pnl[r1 * PS + c0 + j] : T(0);
      }
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int par = c & 1;
        if (elim) {
          const T v0 = pivot_key(x0[c], own0 && !used0);
          const T v1 = pivot_key(x1[c], own1 && !used1);
          const bool take1 = v1 > v0;          // ties keep the lower row
          const T v = take1 ? v1 : v0;
          // reciprocal of this lane's candidate, formed beside the reduction
          // (1 for a zero or non-finite pivot, which is reported instead)
          const T xd = take1 ? x1[c] : x0[c];
          const T rcp = (xd != T(0) && isfinite((double)xd)) ? T(1) / xd : T(1);
          const T m = wave_max_dpp(v);
          const unsigned long long b0 = __ballot(v == m && !take1);
          const unsigned long long b1 = __ballot(v == m && take1);
          const bool hi = b0 == 0ull;          // first-half rows are the lower rows of the wave
          const unsigned long long bw = hi ? b1 : b0;
          const int wl = bw ? __ffsll((long long)bw) - 1 : 0;
          if (lane == wl) {
            T *dst = cand_row + (par * EW + wid) * NI;
            if (hi) {
#pragma unroll
              for (int j = 0; j < NI; ++j) dst[j] = x1[j];
            } else {
#pragma unroll
              for (int j = 0; j < NI; ++j) dst[j] = x0[j];
            }
          }
          if (lane == wl) {
            cand_inv[par * EW + wid] = rcp;
            cand_v[par * EW + wid] = m;
            cand_r[par * EW + wid] = 128 * wid + wl + (hi ? 64 : 0);
          }
        }
        __syncthreads();
        if (elim) {
          T cv[EW];
          int cr[EW];
#pragma unroll
          for (int q = 0; q < EW; ++q) {
            cv[q] = cand_v[par * EW + q];
            cr[q] = cand_r[par * EW + q];
          }
          T best = cv[0];
          int ws = 0, pr = cr[0];
#pragma unroll
          for (int q = 1; q < EW; ++q) {
            if (cv[q] > best) {
              best = cv[q];
              ws = q;
              pr = cr[q];
            }
          }
          const T *prow = cand_row + (par * EW + ws) * NI;
          const T d = prow[c];
          T inv_d = cand_inv[par * EW + ws];
          if (pr >= rp) {   // cannot happen while unused rows remain; keeps every index in range
            pr = rp - 1;
            inv_d = T(1);
            if (my_info == 0) my_info = kb + c0 + c + 1;
          }
          if (!(d != T(0)) || !isfinite((double)d)) {
            if (my_info == 0) my_info = kb + c0 + c + 1;
          }
          if (tid == 0) piv[kb + c0 + c] = pr;
          // the scaled pivot row, once per column; every held row loses f times
          // it (the pivot row too), then the pivot row's lane overwrites its row
          T sp[NI];
#pragma unroll
          for (int j = 0; j < NI; ++j) sp[j] = (j == c) ? inv_d : prow[j] * inv_d;
          {
            const T f0 = x0[c], f1 = x1[c];
#pragma unroll
            for (int j = 0; j < NI; ++j) {
              x0[j] = (j == c ? T(0) : x0[j]) - f0 * sp[j];
              x1[j] = (j == c ? T(0) : x1[j]) - f1 * sp[j];
            }
          }
          if (own0 && r0 == pr) {
#pragma unroll
            for (int j = 0; j < NI; ++j) x0[j] = sp[j];
            used0 = true;
            pflag[r0] = (unsigned char)sp1;
          }
          if (own1 && r1 == pr) {
#pragma unroll
            for (int j = 0; j < NI; ++j) x1[j] = sp[j];
            used1 = true;
            pflag[r1] = (unsigned char)sp1;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (own0) pnl[r0 * PS + c0 + j] = x0[j];
        if (own1) pnl[r1 * PS + c0 + j] = x1[j];
      }
      __syncthreads();
      // rank-16 update of the outer panel's other column tiles, in LDS.  The
      // B operands (the inner panel's pivot rows, read before any of them is
      // overwritten) go to registers ahead of a barrier; every column tile is
      // then updated in straight-line code, the inner panel's own tile
      // computed but not stored (its B operands are not zero).  Columns past a
      // short last panel hold zeros and stay zero.
      {
        constexpr int kCt = NBO / 16;
        const int ct_in = c0 / NI;
        T bi[kCt][NI / 4];
#pragma unroll
        for (int q = 0; q < NI / 4; ++q) {
          const int prow_k = piv[kb + c0 + 4 * q + (lane >> 4)];
#pragma unroll
          for (int ct = 0; ct < kCt; ++ct) bi[ct][q] = pnl[prow_k * PS + ct * 16 + (lane & 15)];
        }
        __syncthreads();
        for (int rt = wid; rt < n_rt; rt += W) {
          T av[NI / 4];
#pragma unroll
          for (int q = 0; q < NI / 4; ++q) av[q] = pnl[(rt * 16 + (lane & 15)) * PS + c0 + 4 * q + (lane >> 4)];
          bool keep[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) keep[r] = pflag[rt * 16 + M::row(lane, r)] != sp1;
#pragma unroll
          for (int ct = 0; ct < kCt; ++ct) {
            const int col = ct * 16 + (lane & 15);
            typename M::acc_t acc = M::zero();
#pragma unroll
            for (int q = 0; q < NI / 4; ++q) acc = M::mma(av[q], bi[ct][q], acc);
            T old[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) old[r] = keep[r] ? pnl[(rt * 16 + M::row(lane, r)) * PS + col] : T(0);
            if (ct != ct_in) {
#pragma unroll
              for (int r = 0; r < 4; ++r) pnl[(rt * 16 + M::row(lane, r)) * PS + col] = old[r] + acc[r];
            }
          }
        }
      }
      __syncthreads();
    }

    // rank-NBO pass over the column tiles outside the outer panel.  The lane
    // index passes through an empty asm statement so that the pass's operand
    // offsets are formed here instead of being hoisted out of the kb loop and
    // held in registers across the whole kernel.
    int lane_g = lane;
    asm volatile("" : "+v"(lane_g));
    const int pt0 = kb / 16, pt1 = min(n_ct, (kb + NBO) / 16);
    const int n_ct_out = n_ct - (pt1 - pt0);
    const int tiles = n_ct_out * n_rt;
    const int t0 = (int)((int64_t)wid * tiles / W), t1 = (int)((int64_t)(wid + 1) * tiles / W);
    const int g0 = t0 / n_rt;
    // the pass is compiled twice: the first reads A_ii (FP64) directly, the
    // others the working block; loaded values stay raw until the final add
    // (masking and conversion there), so nothing waits on a load early
    auto pass = [&](auto first_c) {
      constexpr bool FIRST = decltype(first_c)::value;
      using LT = typename std::conditional<FIRST, double, T>::type;
      const LT *__restrict__ gsrc;
      if constexpr (FIRST)
        gsrc = a0;
      else
        gsrc = w;
      T bf[SL][NQ];
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int g = g0 + s;
        const bool live = t0 < t1 && g * n_rt < t1;
        const int ct = g < pt0 ? g : g + (pt1 - pt0);
        const int col = ct * 16 + (lane_g & 15);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int k = 4 * q + (lane_g >> 4);
          T v = T(0);
          if (live && k < nbo && col < n) {
            const int pk = piv[kb + k];
            if (pk < n) v = (T)gsrc[pk * n + col];
          }
          bf[s][q] = v;
        }
      }
      // the transformed outer panel goes back to global memory (columns of A only)
      for (int idx = tid; idx < n * NBO; idx += NT) {
        const int i = idx / NBO, c = idx % NBO;
        if (kb + c < n) w[i * n + kb + c] = pnl[i * PS + c];
      }
      // every B operand is in registers before any pivot row is overwritten
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int g = g0 + s;
        if (t0 < t1 && g * n_rt < t1) {
          const int ct = g < pt0 ? g : g + (pt1 - pt0);
          const int col = ct * 16 + (lane_g & 15);
          const bool col_ok = col < n;
          const int rlo = max(t0, g * n_rt) - g * n_rt, rhi = min(t1, (g + 1) * n_rt) - g * n_rt;
          // unconditional loads from in-range addresses; keep marks the values
          // that enter the update (inside the block, not a pivot row of the panel)
          auto load_group = [&](int rt, LT (&raw)[G][4], unsigned &keep) {
            keep = 0u;
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = (rt + gi) * 16 + M::row(lane_g, r);
                const bool in = (rt + gi < rhi) & col_ok & (i < n);
                // per-lane clamped address: a uniform one would become a scalar
                // load, whose wait also drains the vector loads in flight
                raw[gi][r] = gsrc[min(i, n - 1) * n + min(col, n - 1)];
                const bool kp = in & (pflag[min(i, rp - 1)] == 0);
                keep |= kp ? 1u << (4 * gi + r) : 0u;
              }
            }
          };
          // the padded K steps of a short last panel multiply exact zeros
          auto update_group = [&](int rt, const LT (&raw)[G][4], unsigned keep) {
            typename M::acc_t acc[G];
            int arow[G];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
              acc[gi] = M::zero();
              arow[gi] = (min(rt + gi, rhi - 1) * 16 + (lane_g & 15)) * PS + (lane_g >> 4);
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
              for (int gi = 0; gi < G; ++gi) acc[gi] = M::mma(pnl[arow[gi] + 4 * q], bf[s][q], acc[gi]);
              // bounds how far the LDS reads run ahead of the matrix cores
              if (q % 4 == 3) asm volatile("" ::: "memory");
            }
            const bool full = rt + G <= rhi && (ct + 1) * 16 <= n && (rt + G) * 16 <= n;
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = (rt + gi) * 16 + M::row(lane_g, r);
                const T old = ((keep >> (4 * gi + r)) & 1u) ? (T)raw[gi][r] : T(0);
                if (full || (rt + gi < rhi && col_ok && i < n)) w[i * n + col] = old + acc[gi][r];
              }
            }
          };
          // two groups of loads in flight: load the next while updating this one
          LT ra[G][4], rb[G][4];
          unsigned ka, kb2;
          int rt = rlo;
          load_group(rt, ra, ka);
          while (true) {
            if (rt + G < rhi) load_group(rt + G, rb, kb2);
            update_group(rt, ra, ka);
            rt += G;
            if (rt >= rhi) break;
            if (rt + G < rhi) load_group(rt + G, ra, ka);
            update_group(rt, rb, kb2);
            rt += G;
            if (rt >= rhi) break;
          }
        }
      }
    };
    if (first)
      pass(std::true_type{});
    else
      pass(std::false_type{});
    __syncthreads();
  }

  // read the inverse out through the pivot permutation: A^-1[k][m] = W[p_k][q_m]
  for (int k = tid; k < rp; k += NT) qinv[piv[k]] = k;
  __syncthreads();
  {
    // 6 columns of 64 at least: at n_i <= 320 five would do, but the register
    // allocation of the FP64 kernel then spills
    constexpr int kCols = (L::MAXN > 384 ? L::MAXN + 63 : 384) / 64, kRows = 4;
    int qc[kCols];
#pragma unroll
    for (int t = 0; t < kCols; ++t) {
      const int m = lane + 64 * t;
      qc[t] = m < n ? qinv[m] : n;
    }
    T *__restrict__ o = out + off;
    for (int k0 = wid * kRows; k0 < n; k0 += W * kRows) {
      T v[kRows][kCols];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int k = k0 + r;
        const int pk = k < n ? piv[k] : n;
#pragma unroll
        for (int t = 0; t < kCols; ++t)
          v[r][t] = (pk < n && qc[t] < n) ? w[(int64_t)pk * n + qc[t]] : T(0);
      }
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int k = k0 + r;
#pragma unroll
        for (int t = 0; t < kCols; ++t) {
          const int m = lane + 64 * t;
          if (k < n && m < n) o[(int64_t)k * n + m] = v[r][t];
        }
      }
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

template <class L>
hipError_t gj_res_launch(Plan &p, typename L::T *work, typename L::T *out) {
  const size_t lds = L::lds_bytes(p.max_ni);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(gj_resident_kernel<L>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((gj_resident_kernel<L>), dim3(p.n_elem), dim3(L::NT), lds, p.stream, p.aii, work, out,
                     p.d_inv_n, p.d_inv_off, p.d_inv_order, p.d_info);
  return hipGetLastError();
}

// outer panels of 48 FP64 / 64 FP32 columns, one 512-thread workgroup per CU.
// Measured at n_i = 320 (8^3 x N = 5): FP32 112 / 96 / 80 / 64 / 48 / 32
// columns take 1.54 / 1.62 / 1.55 / 1.43 / 1.64 / 1.81 ms (wider panels: fewer
// passes but a larger in-LDS update per inner panel); two 256-thread
// workgroups per CU with 48 columns 1.53 ms.  FP64 48 is the widest that fits.
// Each comes in two sizes: up to n_i = 320 (N <= 5; fewer column tiles, so
// fewer registers for the B operands of a wave's share: FP32 1.43 against
// 1.54 ms) and up to kResMaxN = 400 (N = 5 elements with a wall face among
// their interior nodes), where an FP64 panel of 48 columns no longer fits in
// LDS and the FP64 form takes 32.
using GjRes64 = GjRes<double, 32, 2, kResMaxN>;
using GjRes32 = GjRes<float, 64, 2, kResMaxN>;
using GjRes64n5 = GjRes<double, 48, 2, 320>;
using GjRes32n5 = GjRes<float, 64, 2, 320>;

}  // namespace

bool gj_resident_supported(int max_n, bool fp32) {
  if (max_n > kResMaxN) return false;
  return fp32 ? GjRes32::lds_bytes(max_n) <= kLdsLimit : GjRes64::lds_bytes(max_n) <= kLdsLimit;
}

hipError_t launch_gj_inverse_resident(Plan &p, void *work, void *out, bool fp32) {
  float *wf = static_cast<float *>(work), *of = static_cast<float *>(out);
  double *wd = static_cast<double *>(work), *od = static_cast<double *>(out);
  if (p.max_ni <= GjRes32n5::MAXN)
    return fp32 ? gj_res_launch<GjRes32n5>(p, wf, of) : gj_res_launch<GjRes64n5>(p, wd, od);
  return fp32 ? gj_res_launch<GjRes32>(p, wf, of) : gj_res_launch<GjRes64>(p, wd, od);
}

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
