// Measured ceilings for the rooflines: matrix-core throughput (back-to-back
// 16x16x4 MFMAs on register operands, no memory traffic in the loop) and HBM
// streaming-read bandwidth (16-byte nontemporal loads, one contiguous chunk per
// workgroup, over a buffer much larger than the caches).  These are
// measurement utilities beside the solver; the vendor figures stay the
// reference peaks, the probes show what a kernel can reach on the part at hand.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "mfma.hpp"

namespace scdg {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocksPerCu = 8;      // 32 waves per CU, 8 per SIMD
constexpr int kChains = 4;                // independent accumulators per wave

template <typename T>
__global__ __launch_bounds__(kProbeThreads) void mfma_peak_kernel(int32_t iters, T seed, T *__restrict__ out) {
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63;
  const T a = seed + (T)lane * (T)1e-3;
  const T b = seed - (T)lane * (T)1e-3;
  typename M::acc_t c[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) c[k] = M::zero();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) c[k] = M::mma(a, b, c[k]);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

typedef double probe_d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kProbeThreads) void hbm_fill_kernel(probe_d2 *__restrict__ buf, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride)
    buf[i] = probe_d2{(double)(i & 1023), 1.0};
}

// Each workgroup reads one contiguous chunk of the buffer (whole DRAM pages per
// workgroup), each thread 16-byte vectors with four loads in flight; one
// partial sum per thread keeps the loads live.
__global__ __launch_bounds__(kProbeThreads) void hbm_read_kernel(const probe_d2 *__restrict__ buf, int64_t n,
                                                                 double *__restrict__ out) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n ? b0 + per : n;
  int64_t i = b0 + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (; i + 3 * kProbeThreads < b1; i += 4 * kProbeThreads) {
    const probe_d2 v0 = __builtin_nontemporal_load(&buf[i]);
    const probe_d2 v1 = __builtin_nontemporal_load(&buf[i + kProbeThreads]);
    const probe_d2 v2 = __builtin_nontemporal_load(&buf[i + 2 * kProbeThreads]);
    const probe_d2 v3 = __builtin_nontemporal_load(&buf[i + 3 * kProbeThreads]);
    s0 += v0.x + v1.x + v2.x + v3.x;
    s1 += v0.y + v1.y + v2.y + v3.y;
  }
  for (; i < b1; i += kProbeThreads) {
    const probe_d2 v = __builtin_nontemporal_load(&buf[i]);
    s0 += v.x;
    s1 += v.y;
  }
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s0 + s1;
}

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

// Time `launch` (already warmed up) with events on s; best of `reps`.
template <typename F>
hipError_t best_ms(hipStream_t s, int reps, F launch, float *ms) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e0);
    return err;
  }
  float best = -1.f;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    if (err == hipSuccess && (best < 0.f || t < best)) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return err;
}

}  // namespace

}  // namespace scdg

using namespace scdg;

extern "C" {

scdg_status scdg_probe_mfma(int32_t precision, int32_t iters, void *hip_stream, double *tflops) {
  if (!tflops || (precision != 0 && precision != 1) || iters < 1 || iters > (1 << 20)) return SCDG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int blocks = cu_count() * kProbeBlocksPerCu;
  const size_t elem = precision == 0 ? sizeof(double) : sizeof(float);
  void *out = nullptr;
  if (hipMalloc(&out, elem * (size_t)blocks * kProbeThreads) != hipSuccess) return SCDG_ERR_NOMEM;
  auto launch = [&](int32_t it) -> hipError_t {
    if (precision == 0)
      hipLaunchKernelGGL(mfma_peak_kernel<double>, dim3(blocks), dim3(kProbeThreads), 0, s, it, 1.0,
                         static_cast<double *>(out));
    else
      hipLaunchKernelGGL(mfma_peak_kernel<float>, dim3(blocks), dim3(kProbeThreads), 0, s, it, 1.0f,
                         static_cast<float *>(out));
    return hipGetLastError();
  };
  hipError_t err = launch(iters < 64 ? iters : 64);       // warm-up
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  float ms = 0.f;
  if (err == hipSuccess) err = best_ms(s, 3, [&] { return launch(iters); }, &ms);
  (void)hipFree(out);
  if (err != hipSuccess) return SCDG_ERR_HIP;
  const double waves = (double)blocks * (kProbeThreads / 64);
  const double flops = waves * (double)iters * kChains * (2.0 * 16 * 16 * 4);
  *tflops = ms > 0.f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  return SCDG_OK;
}

scdg_status scdg_probe_hbm_read(int64_t bytes, void *hip_stream, double *gbs) {
  if (!gbs || bytes < ((int64_t)64 << 20) || bytes > ((int64_t)16 << 30) || bytes % 16 != 0) return SCDG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t n = bytes / 16;
  const int blocks = cu_count() * kProbeBlocksPerCu;
  void *buf = nullptr, *out = nullptr;
  if (hipMalloc(&buf, (size_t)bytes) != hipSuccess) return SCDG_ERR_NOMEM;
  if (hipMalloc(&out, sizeof(double) * (size_t)blocks * kProbeThreads) != hipSuccess) {
    (void)hipFree(buf);
    return SCDG_ERR_NOMEM;
  }
  hipLaunchKernelGGL(hbm_fill_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, static_cast<probe_d2 *>(buf), n);
  hipError_t err = hipGetLastError();
  auto launch = [&]() -> hipError_t {
    hipLaunchKernelGGL(hbm_read_kernel, dim3(blocks), dim3(kProbeThreads), 0, s,
                       static_cast<const probe_d2 *>(buf), n, static_cast<double *>(out));
    return hipGetLastError();
  };
  if (err == hipSuccess) err = launch();                   // warm-up
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  float ms = 0.f;
  if (err == hipSuccess) err = best_ms(s, 5, launch, &ms);
  (void)hipFree(out);
  (void)hipFree(buf);
  if (err != hipSuccess) return SCDG_ERR_HIP;
  *gbs = ms > 0.f ? (double)bytes / (ms * 1e-3) / 1e9 : 0.0;
  return SCDG_OK;
}

}  // extern "C"
