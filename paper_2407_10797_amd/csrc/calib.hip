// calib.hip -- measured peaks of the resources the roofline is drawn against:
// the FP64 and the (unpacked) FP32 fused multiply-add rates of the vector ALU,
// and the HBM bandwidth of a plain device-to-device copy.  Not part of the
// statistic; bench.py reports these next to the published MI355X figures.
#include <cstdint>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"

namespace fstat {

constexpr int kChains = 8;        // independent FMA chains per lane
constexpr int kCalibBlock = 256;

// Each lane runs kChains independent chains x <- x * a + b for `iters` rounds
// (a < 1, so the chains settle at b / (1 - a) and never overflow or go
// subnormal).  One FMA = 2 FLOP.  The sum is written so that nothing is dead.
template <typename T>
__global__ __launch_bounds__(kCalibBlock) void k_fma_chain(T* __restrict__ out, int32_t iters,
                                                           T a, T b) {
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)(threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// grid-stride copy, 16 bytes per lane per access
__global__ __launch_bounds__(kCalibBlock) void k_copy16(const int4* __restrict__ src,
                                                        int4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace fstat

using namespace fstat;

extern "C" int fstat_calibrate(int32_t kind, int64_t size, int32_t reps, double* rate,
                               double* ms, void* hip_stream) {
  if (!rate || !ms) return set_error(FSTAT_EINVAL, "null rate or ms");
  if (kind < FSTAT_CALIB_FMA64 || kind > FSTAT_CALIB_COPY)
    return set_error(FSTAT_EINVAL, "unknown calibration kind %d", kind);
  if (size < 1 || reps < 1) return set_error(FSTAT_EINVAL, "size and reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0, ncu = 0;
  int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                          "device attribute");
  if (rc) return rc;
  void* a = nullptr;
  void* b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const unsigned blocks = (unsigned)ncu * 16u;   // 16 blocks x 4 waves per CU
  int64_t n16 = 0;
  if (kind == FSTAT_CALIB_COPY) {
    if (size > ((int64_t)1 << 36)) return set_error(FSTAT_EINVAL, "copy size above 64 GiB");
    n16 = (size + 15) / 16;
    rc = hip_check(hipMalloc(&a, (size_t)n16 * 16), "alloc copy source");
    if (!rc) rc = hip_check(hipMalloc(&b, (size_t)n16 * 16), "alloc copy destination");
    if (!rc) rc = hip_check(hipMemsetAsync(a, 0, (size_t)n16 * 16, s), "clear copy source");
  } else {
    if (size > (1 << 24)) return set_error(FSTAT_EINVAL, "FMA rounds above 2^24");
    rc = hip_check(hipMalloc(&a, (size_t)blocks * kCalibBlock * sizeof(double)), "alloc out");
  }
  if (!rc) rc = hip_check(hipEventCreate(&e0), "event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "event");
  auto launch = [&]() {
    if (kind == FSTAT_CALIB_FMA64)
      hipLaunchKernelGGL(k_fma_chain<double>, dim3(blocks), dim3(kCalibBlock), 0, s, (double*)a,
                         (int32_t)size, 0.999999, 1e-7);
    else if (kind == FSTAT_CALIB_FMA32)
      hipLaunchKernelGGL(k_fma_chain<float>, dim3(blocks), dim3(kCalibBlock), 0, s, (float*)a,
                         (int32_t)size, 0.9999f, 1e-4f);
    else
      hipLaunchKernelGGL(k_copy16, dim3((unsigned)ncu * 32u), dim3(kCalibBlock), 0, s,
                         (const int4*)a, (int4*)b, n16);
  };
  if (!rc) {
    launch();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, s);
    rc = hip_check(hipGetLastError(), "calibration launch");
  }
  float t = 0.0f;
  if (!rc) rc = hip_check(hipEventSynchronize(e1), "calibration sync");
  if (!rc) rc = hip_check(hipEventElapsedTime(&t, e0, e1), "calibration time");
  if (!rc) {
    *ms = (double)t / reps;
    const double sec = 1e-3 * (*ms);
    if (kind == FSTAT_CALIB_COPY)
      *rate = 2.0 * 16.0 * (double)n16 / sec / 1e9;                      // GB/s read + written
    else
      *rate = 2.0 * kChains * 16.0 * (double)size * blocks * kCalibBlock / sec / 1e12;  // TFLOP/s
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}
