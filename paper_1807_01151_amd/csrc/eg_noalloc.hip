// No-allocation residual norm: the density-residual norm of Section 4 (the
// norm under eq. (cfl)), (1/|Omega|) (int R_rho^2)^(1/2), of a level-p_max
// residual in the orthonormal psi coordinates of the C ABI, where the
// integral is the sum of the squared density coefficients.  Its only
// workspace is a file-scope device array: one partial sum per block of
// NOALLOC_EPB elements, summed by one block in a fixed order (deterministic).
// Every block writes its partial before the final sum reads it, so nothing
// has to be cleared between calls.  All calls on one GPU share that GPU's
// array: calls that overlap on one GPU (other streams or host threads) race.

#include <hip/hip_runtime.h>

#include <mutex>

#include "eg_launch.h"

namespace eg {

namespace {
constexpr int NOALLOC_EPB = 256;          // elements per block of the partial sums
constexpr int NOALLOC_MAX_BLOCKS = 4096;  // static workspace: 4096 partials = 32 KiB
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

// The workspace.  Host code never passes this name to a kernel or a copy:
// on the host it is only a stand-in for the symbol; the per-device address
// comes from hipGetSymbolAddress (noalloc_resolve) and is kept in g_scratch.
static __device__ __align__(256) double scratch[NOALLOC_MAX_BLOCKS];

namespace {
std::mutex g_mu;
double* g_scratch[NOALLOC_MAX_DEVICES] = {};

__device__ __forceinline__ double block_sum_256(double v, double* s_w) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

// part[b] = sum over the density coefficients of elements
// [b EPB, min((b + 1) EPB, ne)) of x^2; r is [ne][V][N] (V N = VN).
__global__ __launch_bounds__(256) void k_dnorm_partial(const double* __restrict__ r, int ne, int VN, int N,
                                                       double* __restrict__ part) {
  __shared__ double s_w[4];
  const int e0 = blockIdx.x * NOALLOC_EPB;
  const int nel = min(NOALLOC_EPB, ne - e0);
  double acc = 0.0;
  for (int t = threadIdx.x; t < nel * N; t += 256) {
    const double x = r[(size_t)(e0 + t / N) * VN + t % N];
    acc += x * x;
  }
  const double s = block_sum_256(acc, s_w);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_dnorm_final(const double* __restrict__ part, int nblk, double omega,
                                                     double* __restrict__ out) {
  __shared__ double s_w[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[i];
  const double s = block_sum_256(acc, s_w);
  if (threadIdx.x == 0) out[0] = sqrt(s) / omega;
}
}  // namespace

int noalloc_max_elems() { return NOALLOC_EPB * NOALLOC_MAX_BLOCKS; }

hipError_t noalloc_resolve(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // resolved with that device current only
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = static_cast<double*>(p);
  return hipSuccess;
}

hipError_t launch_dnorm_noalloc(int device, int ne, int V, int N, double omega, const double* r, double* out,
                                hipStream_t st) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES || ne < 1 || ne > noalloc_max_elems()) return hipErrorInvalidValue;
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    part = g_scratch[device];
  }
  if (!part) return hipErrorNotInitialized;
  const int nblk = (ne + NOALLOC_EPB - 1) / NOALLOC_EPB;
  hipLaunchKernelGGL(k_dnorm_partial, dim3(nblk), dim3(256), 0, st, r, ne, V * N, N, part);
  hipLaunchKernelGGL(k_dnorm_final, dim3(1), dim3(256), 0, st, part, nblk, omega, out);
  return hipGetLastError();
}

}  // namespace eg
