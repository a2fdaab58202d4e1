// Allocation-free variant of dmrg_block_gemm for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// dmrg_block_gemm stages its tile and item descriptors in device memory it
// allocates per call.  This variant keeps them in one file-scope device array,
// `scratch`, of kScratchBytes, and writes them with a small staging kernel from
// scalar kernel arguments, so the call makes no allocation and no host-to-device
// copy.  The array's device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; host code never
// passes the array's own name to a kernel.  Every call on a device shares that
// device's array: calls that overlap on one device (different streams, or
// threads) race; calls ordered on one stream do not.
#include <hip/hip_runtime.h>

#include <mutex>

#include "capi_guard.hpp"
#include "kernels.hpp"

namespace dmrg {
void hip_check(hipError_t e, const char* what);

namespace {

constexpr int kMaxTiles = 4096;  // 64 x 64 tiles: M, N up to 4096
constexpr size_t kItemOffset = (size_t)kMaxTiles * sizeof(GemmUnit);
constexpr size_t kScratchBytes = 256 * 1024;
static_assert(kItemOffset % 16 == 0, "item descriptor must stay 16-byte aligned");
static_assert(kItemOffset + sizeof(GemmItem) <= kScratchBytes, "scratch too small for the descriptors");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
void* scratch_address() {
  int dev = -1;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  DMRG_REQUIRE(dev >= 0 && dev < kMaxDevices, ST_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    DMRG_REQUIRE(p != nullptr, ST_EHIP, "no device address for the scratch array");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Tile descriptors of an M x N output in 64 x 64 tiles (row-major tile order,
// n_tn tiles per row) and the one item: the same table dmrg_block_gemm uploads.
__global__ void stage_block_gemm(GemmUnit* __restrict__ units, GemmItem* __restrict__ item, int n_units, int n_tn,
                                 void* C, int ldc, int M, int N, const void* A, int lda, const void* B, int ldb,
                                 int K, double coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_units) {
    GemmUnit u;
    u.C = C;
    u.ldc = ldc;
    u.M = M;
    u.N = N;
    u.m0 = (i / n_tn) * 64;
    u.n0 = (i % n_tn) * 64;
    u.ib = 0;
    u.ie = 1;
    u.accumulate = 0;
    u.shape = 0;
    units[i] = u;
  }
  if (i == 0) {
    GemmItem it;
    it.A = A;
    it.B = B;
    it.lda = lda;
    it.ldb = ldb;
    it.K = K;
    it.pad = 0;
    it.coef = coef;
    *item = it;
  }
}

}  // namespace
}  // namespace dmrg

using namespace dmrg;

extern "C" dmrg_status dmrg_block_gemm_noalloc(int precision, int mode, int M, int N, int K, const void* A, int lda,
                                               const void* B, int ldb, void* C, int ldc, double coef,
                                               void* hip_stream) {
  return guard([&] {
    DMRG_REQUIRE(A && B && C, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(M > 0 && N > 0 && K > 0, ST_EINVAL, "sizes must be positive");
    DMRG_REQUIRE(mode >= 0 && mode <= 2 && precision >= 0 && precision <= 2, ST_EINVAL, "bad mode/precision");
    DMRG_REQUIRE(!(precision == 2 && mode == 2), ST_EINVAL, "bf16 has no transposed-A mode");
    DMRG_REQUIRE(lda >= (mode == 2 ? M : K) && ldb >= (mode == 1 ? K : N) && ldc >= N, ST_EINVAL,
                 "leading dimension too small");
    const long n_tm = (M + 63) / 64, n_tn = (N + 63) / 64;
    DMRG_REQUIRE(n_tm * n_tn <= kMaxTiles, ST_EINVAL,
                 "output too large for the allocation-free scratch: at most 4096 tiles of 64 x 64 "
                 "(M, N <= 4096 when square); use dmrg_block_gemm");
    const int n_units = (int)(n_tm * n_tn);
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned char* base = (unsigned char*)scratch_address();
    GemmUnit* units = (GemmUnit*)base;
    GemmItem* item = (GemmItem*)(base + kItemOffset);
    stage_block_gemm<<<(n_units + 255) / 256, 256, 0, st>>>(units, item, n_units, (int)n_tn, C, ldc, M, N, A, lda,
                                                            B, ldb, K, coef);
    hip_check(hipGetLastError(), "stage_block_gemm launch");
    launch_gemm(precision, mode, units, n_units, item, st);
    hip_check(hipGetLastError(), "block gemm launch");
  });
}
