// Measurement helper: the rate at which this device gathers random 4-byte
// values through an adjacency, i.e. the bare access pattern of the neighbour
// scan (the hotspot of the method, Sec. III, Optimizations) without any of
// the method's work.  One pass: coalesced reads of idx, one gather of vals per
// entry, a sum so that nothing is optimised away.  The round kernels are
// compared against this rate for the same graph.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/kcore.h"
#include "kcore_runtime.h"

namespace kcore {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;     // index loads issued before their gathers
constexpr int kProbeBlocksPerCu = 32;

__global__ void k_probe_zero(unsigned long long* out) {
  if (threadIdx.x == 0) *out = 0;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const int32_t* __restrict__ idx, int64_t m,
                                                             const int32_t* __restrict__ vals,
                                                             unsigned long long* out) {
  const int64_t T = (int64_t)gridDim.x * kProbeBlock;
  int64_t j = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  long long acc = 0;
  for (; j + (kProbeUnroll - 1) * T < m; j += kProbeUnroll * T) {
    int32_t c[kProbeUnroll];
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) c[q] = idx[j + q * T];
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) acc += vals[c[q]];
  }
  for (; j < m; j += T) acc += vals[idx[j]];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ long long part[kProbeBlock / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
#pragma unroll
    for (int w = 0; w < kProbeBlock / 64; ++w) t += part[w];
    atomicAdd(out, (unsigned long long)t);
  }
}

}  // namespace
}  // namespace kcore

extern "C" kcore_status kcore_probe_gather(const int32_t* idx, int64_t m, const int32_t* vals, int64_t n,
                                           int64_t* out_sum, void* stream) {
  using namespace kcore;
  if (m < 0 || n < 0 || !out_sum || (m > 0 && (!idx || !vals || n == 0)))
    return fail(KCORE_E_INVALID, "bad probe arguments");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  unsigned long long* out = reinterpret_cast<unsigned long long*>(out_sum);
  hipLaunchKernelGGL(k_probe_zero, dim3(1), dim3(64), 0, st, out);
  if (m > 0)
    hipLaunchKernelGGL(k_probe_gather, dim3(kProbeBlocksPerCu * cus), dim3(kProbeBlock), 0, st, idx, m, vals, out);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "probe launch");
  return KCORE_OK;
}
