// k_peak.hip -- measured ceilings of this GPU for the rooflines: vector
// FMA throughput in FP32 (as this library compiles it: unpacked) and FP64,
// and HBM bandwidth of a streaming copy.  Diagnostics only; not on any step
// path.
#include "rb_internal.h"

// eight independent FMA chains per thread, ITER rounds; the result is
// stored only when it cannot be (a runtime flag) so that the chains stay live
template <typename T, int ITER>
__global__ __launch_bounds__(256) void k_peak_fma(T *__restrict__ sink, T a, T b, int store) {
  T c0 = (T)threadIdx.x, c1 = c0 + (T)1, c2 = c0 + (T)2, c3 = c0 + (T)3;
  T c4 = c0 + (T)4, c5 = c0 + (T)5, c6 = c0 + (T)6, c7 = c0 + (T)7;
#pragma unroll 16
  for (int i = 0; i < ITER; ++i) {
    c0 = fma(c0, a, b); c1 = fma(c1, a, b); c2 = fma(c2, a, b); c3 = fma(c3, a, b);
    c4 = fma(c4, a, b); c5 = fma(c5, a, b); c6 = fma(c6, a, b); c7 = fma(c7, a, b);
  }
  const T s = ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7));
  if (store) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// streaming copy, 16 bytes per thread and iteration, grid-strided
__global__ __launch_bounds__(256) void k_peak_copy(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

extern "C" int rb_peak_probe(int32_t kind, double *value) {
  if (!value || kind < 0 || kind > 2) return RB_EINVAL;
  constexpr int ITER = 4096;
  const unsigned grid = 256 * 64, block = 256;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return RB_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RB_EHIP;
  }
  void *buf = nullptr, *buf2 = nullptr;
  int rc = RB_OK;
  const uint64_t copy_bytes = 1ull << 31;  // 2 GiB each way
  if (kind == 2) {
    if (hipMalloc(&buf, copy_bytes) != hipSuccess || hipMalloc(&buf2, copy_bytes) != hipSuccess)
      rc = RB_EHIP;
    if (rc == RB_OK) rc = hipMemset(buf, 1, copy_bytes) == hipSuccess ? RB_OK : RB_EHIP;
  } else {
    rc = hipMalloc(&buf, (size_t)grid * block * 8) == hipSuccess ? RB_OK : RB_EHIP;
  }
  float best = 1e30f;
  for (int rep = 0; rc == RB_OK && rep < 4; ++rep) {
    (void)hipEventRecord(e0, 0);
    if (kind == 0)
      hipLaunchKernelGGL((k_peak_fma<float, ITER>), dim3(grid), dim3(block), 0, 0,
                         (float *)buf, 0.999f, 1e-3f, 0);
    else if (kind == 1)
      hipLaunchKernelGGL((k_peak_fma<double, ITER>), dim3(grid), dim3(block), 0, 0,
                         (double *)buf, 0.999, 1e-3, 0);
    else
      hipLaunchKernelGGL(k_peak_copy, dim3(256 * 32), dim3(block), 0, 0, (const uint4 *)buf,
                         (uint4 *)buf2, copy_bytes / 16);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
      rc = RB_EHIP;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) best = ms;
  }
  if (rc == RB_OK) {
    if (kind == 2)
      *value = 2.0 * (double)copy_bytes / (best * 1e-3);  // bytes read + written per s
    else
      *value = 2.0 * 8.0 * ITER * (double)grid * block / (best * 1e-3);  // flop/s
  }
  if (buf) (void)hipFree(buf);
  if (buf2) (void)hipFree(buf2);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
