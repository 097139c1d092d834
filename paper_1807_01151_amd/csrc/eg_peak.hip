// Achievable peaks of the GPU the library runs on (a profiling aid for the
// roofline figures; no part of the method): HBM bandwidth by a streaming
// copy, FP64 matrix-core and FP64 vector FMA throughput by independent
// multiply-add chains, each timed with HIP events on the caller's stream.

#include <hip/hip_runtime.h>

#include "eg_device.h"
#include "eg_launch.h"

namespace eg {

namespace {

// y = x over n double2 values, grid-stride, 16-byte non-temporal loads and
// stores, four loads in flight per thread before the stores.
typedef double dv2_t __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_peak_copy(const dv2_t* __restrict__ x, dv2_t* __restrict__ y, size_t n) {
  const size_t st = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i + 3 * st < n; i += 4 * st) {
    dv2_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(x + i + k * st);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], y + i + k * st);
  }
  for (; i < n; i += st) __builtin_nontemporal_store(__builtin_nontemporal_load(x + i), y + i);
}

// Eight independent accumulator chains of 16 x 16 x 4 FP64 matrix-core
// products per wavefront (enough to cover the instruction's latency); the
// sum of the accumulators is stored so that nothing is optimised away.
__global__ __launch_bounds__(256) void k_peak_mfma64(int iters, double seed, double* __restrict__ out) {
  const double a = seed + 1e-3 * (threadIdx.x & 63), b = seed - 1e-3 * (threadIdx.x >> 6);
  dbl4_t c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = dbl4_t{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[blockIdx.x * (size_t)blockDim.x + threadIdx.x] = s;
}

// Sixteen independent FP64 FMA chains per lane.
__global__ __launch_bounds__(256) void k_peak_fma64(int iters, double seed, double* __restrict__ out) {
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = seed + 1e-3 * k + 1e-6 * threadIdx.x;
  const double m = 1.0 - 1e-9, c = 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = fma(x[k], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += x[k];
  out[blockIdx.x * (size_t)blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_peak(int kind, hipStream_t st, double* value) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  hipEvent_t a = nullptr, b = nullptr;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  void* x = nullptr;
  void* y = nullptr;
  const int grid = 8 * ncu;  // eight workgroups of four wavefronts per compute unit
  size_t bytes = 0;
  if (kind == 0) bytes = (size_t)1 << 30;  // 1 GiB read + 1 GiB written
  else bytes = (size_t)grid * 256 * sizeof(double);
  e = hipMalloc(&x, bytes);
  if (e == hipSuccess && kind == 0) e = hipMalloc(&y, bytes);
  if (e == hipSuccess && kind == 0) e = hipMemsetAsync(x, 0, bytes, st);
  float ms = 0.0f;
  const int reps = 5;
  const int iters = 4096;
  for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {  // pass 0 warms up
    if ((e = hipEventRecord(a, st)) != hipSuccess) break;
    for (int r = 0; r < reps; ++r) {
      if (kind == 0)
        hipLaunchKernelGGL(k_peak_copy, dim3(4 * grid), dim3(256), 0, st, static_cast<const dv2_t*>(x),
                           static_cast<dv2_t*>(y), bytes / sizeof(dv2_t));
      else if (kind == 1)
        hipLaunchKernelGGL(k_peak_mfma64, dim3(grid), dim3(256), 0, st, iters, 1.0, static_cast<double*>(x));
      else
        hipLaunchKernelGGL(k_peak_fma64, dim3(grid), dim3(256), 0, st, iters, 1.0, static_cast<double*>(x));
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  }
  if (e == hipSuccess) {
    const double s = ms * 1e-3 / reps;
    if (kind == 0) *value = 2.0 * (double)bytes / s / 1e9;                            // GB/s
    else if (kind == 1) *value = (double)grid * 4 * iters * 8 * 16 * 16 * 4 * 2.0 / s / 1e12;  // TFLOP/s
    else *value = (double)grid * 256 * iters * 16 * 2.0 / s / 1e12;                   // TFLOP/s
  }
  (void)hipStreamSynchronize(st);
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return e;
}

}  // namespace eg
