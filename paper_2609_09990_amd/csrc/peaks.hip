// Device-ceiling microkernels for roofline reports.  Built with the VGPR form
// of MFMA (accumulators in ordinary VGPRs): in the AGPR form the compiler moves
// the loop-carried accumulators between register files around every MFMA of
// this short loop, which would measure the moves rather than the MFMA rate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace dmrg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// Device ceilings.  mfma_f64_peak: every lane runs `iters` rounds of four
// independent fp64 16x16x4 MFMAs on register operands (no memory traffic in the
// loop), then stores one value so the work is kept.  stream_copy: 16-byte
// non-temporal loads and stores over a whole buffer.
__global__ __launch_bounds__(256) void mfma_f64_peak(double* __restrict__ out, int iters) {
  v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0, a2 = a0, a3 = a0;
  const double x = 1e-3 * (threadIdx.x + 1), y = 1.0 + 1e-6 * blockIdx.x;
  for (int i = 0; i < iters; ++i) {
    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(y, x, a1, 0, 0, 0);
    a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, a2, 0, 0, 0);
    a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(y, y, a3, 0, 0, 0);
  }
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = a0[0] + a1[1] + a2[2] + a3[3];
}

__global__ __launch_bounds__(256) void stream_copy(const v4u32* __restrict__ src, v4u32* __restrict__ dst, long n) {
  // four independent 16-byte loads in flight per lane before the stores
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
    v4u32 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * stride < n) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * stride < n) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
}

}  // namespace

long launch_mfma_f64_peak(double* out, int n_blocks, int iters, hipStream_t s) {
  mfma_f64_peak<<<n_blocks, 256, 0, s>>>(out, iters);
  return (long)n_blocks * 4 * iters * 4 * (2L * 16 * 16 * 4);  // flops: 4 waves x iters x 4 MFMAs
}

void launch_stream_copy(const void* src, void* dst, long bytes, hipStream_t s) {
  const long n = bytes / 16;
  if (n > 0) stream_copy<<<(int)std::min<long>((n + 255) / 256, 8192), 256, 0, s>>>((const v4u32*)src, (v4u32*)dst, n);
}

}  // namespace dmrg
