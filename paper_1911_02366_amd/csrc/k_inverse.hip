// Batched in-place inversion of the interior blocks A_ii(e) by blocked
// Gauss-Jordan elimination with partial pivoting.
//
// The paper inverts every interior block independently with LU routines and
// uses A_ii^-1 in the Schur product and in both condensation steps
// (Section 3.2; eq. SC_step1, SC_step2).  Here one workgroup owns one element:
//   for each panel of NB columns
//     1. the panel (all rows) is copied to LDS and eliminated column by column
//        (pivot = largest |a| among unused rows, lowest row on ties; the pivot
//        row is scaled, every other row is eliminated, and the eliminated
//        column slot stores the running inverse);
//     2. the panel's row interchanges are applied to the other columns;
//     3. the other columns get the rank-NB update  W[:, J] <- W0[:, J] + P R,
//        with P the transformed panel (LDS) and R the panel's pivot rows, on the
//        16x16x4 matrix cores;
//   finally the column interchanges are undone in reverse order.
// Flops: 2 n^3 per element.  A zero or non-finite pivot is recorded LAPACK-
// style (info = step + 1) and replaced by 1 so the launch always completes.
#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 64;

template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void gj_inverse_kernel(T *__restrict__ wbuf,
                                                              const int32_t *__restrict__ n_arr,
                                                              const int64_t *__restrict__ off_arr,
                                                              int32_t *__restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  using M = Mfma<T>;
  const int e = blockIdx.x;
  const int n = n_arr[e];
  T *__restrict__ a = wbuf + off_arr[e];
  const int rp = (n + 15) & ~15;
  T *pnl = reinterpret_cast<T *>(smem);   // [rp][NB]
  T *rl = pnl + rp * NB;                   // [NB][kChunk]
  T *fcol = rl + NB * kChunk;              // [rp]
  int *piv = reinterpret_cast<int *>(fcol + rp);  // [rp]
  __shared__ double red_v[kThreads / 64];
  __shared__ int red_i[kThreads / 64];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  int my_info = 0;

  for (int kb = 0; kb < n; kb += NB) {
    const int nbw = min(NB, n - kb);
    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      pnl[idx] = (i < n && c < nbw) ? a[(int64_t)i * n + kb + c] : T(0);
    }
    __syncthreads();

    for (int c = 0; c < nbw; ++c) {
      const int k = kb + c;
      double best = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += kThreads) {
        const double v = fabs((double)pnl[i * NB + c]);
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
#pragma unroll
      for (int w = 1; w < kThreads / 64; ++w) {
        if (red_v[w] > best || (red_v[w] == best && red_i[w] < bi)) {
          best = red_v[w];
          bi = red_i[w];
        }
      }
      const int pr = (bi < n) ? bi : k;
      if (pr != k && tid < NB) {
        const T t = pnl[k * NB + tid];
        pnl[k * NB + tid] = pnl[pr * NB + tid];
        pnl[pr * NB + tid] = t;
      }
      if (tid == 0) piv[k] = pr;
      __syncthreads();
      T d = pnl[k * NB + c];
      if (!(d != T(0)) || !isfinite((double)d)) {
        if (my_info == 0) my_info = k + 1;
        d = T(1);
      }
      const T inv_d = T(1) / d;
      for (int i = tid; i < rp; i += kThreads) fcol[i] = pnl[i * NB + c];
      __syncthreads();
      if (tid < NB) {
        const T v = (tid == c) ? T(1) : pnl[k * NB + tid];
        pnl[k * NB + tid] = v * inv_d;
      }
      __syncthreads();
      for (int idx = tid; idx < rp * NB; idx += kThreads) {
        const int i = idx / NB, j = idx % NB;
        if (i == k) continue;
        const T av = (j == c) ? T(0) : pnl[idx];
        pnl[idx] = av - fcol[i] * pnl[k * NB + j];
      }
      __syncthreads();
    }

    // row interchanges of this panel on the columns outside it
    for (int j = tid; j < n; j += kThreads) {
      if (j >= kb && j < kb + nbw) continue;
      for (int c = 0; c < nbw; ++c) {
        const int k = kb + c, pr = piv[k];
        if (pr != k) {
          const T t = a[(int64_t)k * n + j];
          a[(int64_t)k * n + j] = a[(int64_t)pr * n + j];
          a[(int64_t)pr * n + j] = t;
        }
      }
    }
    __syncthreads();

    // rank-NB update of the columns outside the panel
    for (int j0 = 0; j0 < n; j0 += kChunk) {
      if (j0 >= kb && j0 + kChunk <= kb + nbw) continue;
      for (int idx = tid; idx < NB * kChunk; idx += kThreads) {
        const int c = idx / kChunk, j = j0 + idx % kChunk;
        const bool ok = c < nbw && j < n && !(j >= kb && j < kb + nbw);
        rl[idx] = ok ? a[(int64_t)(kb + c) * n + j] : T(0);
      }
      __syncthreads();
      const int jl = wid * 16 + (lane & 15);
      const int jc = j0 + jl;
      const bool col_ok = jc < n && !(jc >= kb && jc < kb + nbw);
      for (int r0 = 0; r0 < rp; r0 += 16) {
        typename M::acc_t acc = M::zero();
#pragma unroll
        for (int kk = 0; kk < NB; kk += 4) {
          const T av = pnl[(r0 + (lane & 15)) * NB + kk + (lane >> 4)];
          const T bv = rl[(kk + (lane >> 4)) * kChunk + jl];
          acc = M::mma(av, bv, acc);
        }
        if (col_ok) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = r0 + M::row(lane, r);
            if (i < n) {
              const bool in_k = i >= kb && i < kb + nbw;
              const T old = in_k ? T(0) : a[(int64_t)i * n + jc];
              a[(int64_t)i * n + jc] = old + acc[r];
            }
          }
        }
      }
      __syncthreads();
    }

    for (int idx = tid; idx < rp * NB; idx += kThreads) {
      const int i = idx / NB, c = idx % NB;
      if (i < n && c < nbw) a[(int64_t)i * n + kb + c] = pnl[idx];
    }
    __syncthreads();
  }

  // undo the column interchanges in reverse order
  for (int i = tid; i < n; i += kThreads) {
    T *row = a + (int64_t)i * n;
    for (int k = n - 1; k >= 0; --k) {
      const int pr = piv[k];
      if (pr != k) {
        const T t = row[k];
        row[k] = row[pr];
        row[pr] = t;
      }
    }
  }
  if (tid == 0) info[e] = my_info;
}

template <typename T, int NB>
size_t gj_lds_bytes(int max_n) {
  const int rp = (max_n + 15) & ~15;
  return sizeof(T) * ((size_t)rp * NB + NB * kChunk + rp) + sizeof(int) * rp;
}

template <typename T, int NB>
hipError_t gj_launch(Plan &p, T *w) {
  const size_t lds = gj_lds_bytes<T, NB>(p.max_ni);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(gj_inverse_kernel<T, NB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((gj_inverse_kernel<T, NB>), dim3(p.n_elem), dim3(kThreads), lds, p.stream, w,
                     p.d_inv_n, p.d_inv_off, p.d_info);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gj_inverse(Plan &p, void *w, bool fp32) {
  if (fp32) return gj_launch<float, 16>(p, static_cast<float *>(w));
  return gj_launch<double, 16>(p, static_cast<double *>(w));
}

size_t gj_lds_limit_check(int max_n, bool fp32) {
  return fp32 ? gj_lds_bytes<float, 16>(max_n) : gj_lds_bytes<double, 16>(max_n);
}

}  // namespace scdg
