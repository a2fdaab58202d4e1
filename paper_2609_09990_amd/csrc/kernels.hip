// gfx950 kernels for the two-site sigma path.
//
// The workhorse is a grouped block GEMM: every output tile of sigma (or of a
// new environment, or of an intermediate T = X psi) accumulates its block
// products ("items") in a fixed order with MFMA, so results are bitwise
// reproducible (no atomics; split-K partial tiles are summed in order by
// splitk_reduce).  Three shapes:
//  * gemm_wg: one 256-thread workgroup per unit, tiles up to 96 x 64 covering a
//    whole output block, A slices staged through LDS and shared by the four
//    waves, B rows by raw buffer loads, k slices of 32 with one of lookahead
//    (sigma phase B, fp64 / fp32);
//  * w32_tile: one wave per (16 RB) x (16 CB) tile reading operands straight
//    from memory (phase A, environment updates, gradient, fp32 / bf16 forms);
//  * gemm_f64 / gemm_f32 / gemm_bf16: plain 64 x 64 LDS tiles, four waves of
//    32 x 32 (one-off products: two-site forms, overlaps, projections, the MLP,
//    dmrg_block_gemm).
// Plus the Davidson BLAS-1 kernels, the one-workgroup Jacobi eigensolver, the
// diagonal, premix / pairmix and precision conversions.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <stdexcept>

#include "kernels.hpp"

namespace dmrg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 16, LDP = TM + 2;

__device__ inline float to_f(float x) { return x; }
__device__ inline float to_f(double x) { return (float)x; }
__device__ inline float to_f(uint16_t x) { return __uint_as_float(((uint32_t)x) << 16); }
__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }
__device__ inline uint16_t f2bf(float x) {
  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Loads a 64 x 16 A tile (k-major into LDS) and a 16 x 64 B tile, scaling A by coef.
template <int MODE, typename TA, typename TB, typename TS>
__device__ inline void load_tiles(TS (*As)[LDP], TS (*Bs)[LDP], const TA* A, const TB* B, int lda,
                                  int ldb, int K, int k0, int m0, int M, int n0, int N,
                                  double coef, int tid) {
  if (MODE == GEMM_NN || MODE == GEMM_NT) {
    int m = tid >> 2, kq = (tid & 3) * 4;
    int gm = m0 + m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int k = kq + j;
      double v = 0.0;
      if (gm < M && k0 + k < K) v = to_d(A[(long)gm * lda + k0 + k]) * coef;
      As[k][m] = (TS)v;
    }
  } else {
    int k = tid >> 4, mq = (tid & 15) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int m = mq + j;
      double v = 0.0;
      if (m0 + m < M && k0 + k < K) v = to_d(A[(long)(k0 + k) * lda + m0 + m]) * coef;
      As[k][m] = (TS)v;
    }
  }
  if (MODE == GEMM_NN || MODE == GEMM_TN) {
    int k = tid >> 4, nq = (tid & 15) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int n = nq + j;
      TS v = (TS)0;
      if (n0 + n < N && k0 + k < K) v = (TS)to_d(B[(long)(k0 + k) * ldb + n0 + n]);
      Bs[k][n] = v;
    }
  } else {
    int n = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int k = kq + j;
      TS v = (TS)0;
      if (n0 + n < N && k0 + k < K) v = (TS)to_d(B[(long)(n0 + n) * ldb + k0 + k]);
      Bs[k][n] = v;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void gemm_f64(const GemmUnit* __restrict__ units,
                                                const GemmItem* __restrict__ items) {
  __shared__ double As[TK][LDP];
  __shared__ double Bs[TK][LDP];
  const GemmUnit u = units[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = items[it];
    const double* A = (const double*)g.A;
    const double* B = (const double*)g.B;
    for (int k0 = 0; k0 < g.K; k0 += TK) {
      load_tiles<MODE, double, double, double>(As, Bs, A, B, g.lda, g.ldb, g.K, k0, u.m0, u.M,
                                               u.n0, u.N, g.coef, tid);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wr + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wc + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  double* C = (double*)u.C;
  // v_mfma_f64_16x16x4f64 accumulator: lane l, element r holds row l/16 + 4r,
  // column l%16 (measured; the f32/bf16 16x16 ops hold row 4(l/16) + r instead)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gm = u.m0 + wr + 16 * i + (lane >> 4) + 4 * r;
        int gn = u.n0 + wc + 16 * j + (lane & 15);
        if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          double v = acc[i][j][r];
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

template <int MODE, typename TA, typename TB>
__global__ __launch_bounds__(256) void gemm_f32(const GemmUnit* __restrict__ units,
                                                const GemmItem* __restrict__ items) {
  __shared__ float As[TK][LDP];
  __shared__ float Bs[TK][LDP];
  const GemmUnit u = units[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = items[it];
    for (int k0 = 0; k0 < g.K; k0 += TK) {
      load_tiles<MODE, TA, TB, float>(As, Bs, (const TA*)g.A, (const TB*)g.B, g.lda, g.ldb, g.K,
                                      k0, u.m0, u.M, u.n0, u.N, g.coef, tid);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wr + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wc + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  float* C = (float*)u.C;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gm = u.m0 + wr + 16 * i + 4 * (lane >> 4) + r;
        int gn = u.n0 + wc + 16 * j + (lane & 15);
        if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          float v = acc[i][j][r];
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

// bf16 operands, fp32 accumulation: A given as TA (bf16 bits or fp32, rounded to
// bf16 in LDS), B as bf16 bits.  One v_mfma_f32_16x16x16_bf16 per 16-deep k tile.
template <int MODE, typename TA>
__global__ __launch_bounds__(256) void gemm_bf16(const GemmUnit* __restrict__ units,
                                                 const GemmItem* __restrict__ items) {
  __shared__ uint16_t As[TK][LDP];
  __shared__ uint16_t Bs[TK][LDP];
  const GemmUnit u = units[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = items[it];
    const TA* A = (const TA*)g.A;
    const uint16_t* B = (const uint16_t*)g.B;
    const float coef = (float)g.coef;
    for (int k0 = 0; k0 < g.K; k0 += TK) {
      if (MODE == GEMM_NN || MODE == GEMM_NT) {
        int m = tid >> 2, kq = (tid & 3) * 4;
        int gm = u.m0 + m;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int k = kq + j;
          float v = 0.f;
          if (gm < u.M && k0 + k < g.K) v = to_f(A[(long)gm * g.lda + k0 + k]) * coef;
          As[k][m] = f2bf(v);
        }
      } else {
        int k = tid >> 4, mq = (tid & 15) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int m = mq + j;
          float v = 0.f;
          if (u.m0 + m < u.M && k0 + k < g.K) v = to_f(A[(long)(k0 + k) * g.lda + u.m0 + m]) * coef;
          As[k][m] = f2bf(v);
        }
      }
      if (MODE == GEMM_NN || MODE == GEMM_TN) {
        int k = tid >> 4, nq = (tid & 15) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int n = nq + j;
          uint16_t v = 0;
          if (u.n0 + n < u.N && k0 + k < g.K) v = B[(long)(k0 + k) * g.ldb + u.n0 + n];
          Bs[k][n] = v;
        }
      } else {
        int n = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int k = kq + j;
          uint16_t v = 0;
          if (u.n0 + n < u.N && k0 + k < g.K) v = B[(long)(u.n0 + n) * g.ldb + k0 + k];
          Bs[k][n] = v;
        }
      }
      __syncthreads();
      v4s a[2], b[2];
      const int kb = 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) a[i][q] = (short)As[kb + q][wr + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) b[j][q] = (short)Bs[kb + q][wc + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      __syncthreads();
    }
  }
  float* C = (float*)u.C;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gm = u.m0 + wr + 16 * i + 4 * (lane >> 4) + r;
        int gn = u.n0 + wc + 16 * j + (lane & 15);
        if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          float v = acc[i][j][r];
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

// Small-tile fp64 GEMM: one wave owns a 32x32 tile (2x2 MFMA 16x16 blocks) and
// loads its MFMA operands straight from global memory (k step 4, no LDS, no
// barriers), so short-K items cost little padding and waves never wait on each
// other.  Four independent waves per workgroup.  accumulate == 2 writes the
// tile into a 32x32 partial slot (split-K), reduced later in a fixed order.
template <int MODE>
__device__ inline double ld_a(const double* A, int lda, int m, int k) {
  return MODE == GEMM_TN ? A[(long)k * lda + m] : A[(long)m * lda + k];
}
template <int MODE>
__device__ inline double ld_b(const double* B, int ldb, int k, int n) {
  return MODE == GEMM_NT ? B[(long)n * ldb + k] : B[(long)k * ldb + n];
}

// Two consecutive doubles p[k], p[k+1] of a row (zero past K or for a masked
// row); a full pair is one 16-byte load (8-byte aligned).
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef __attribute__((address_space(1))) const d2u gd2u;      // global memory
typedef __attribute__((address_space(1))) const double gdbl;
__device__ inline void ld_pair(const double* p, int k, int K, bool rowv, double* x) {
  if (rowv && k + 1 < K) {
    const d2u v = *(gd2u*)(p + k);
    x[0] = v.x;
    x[1] = v.y;
  } else {
    x[0] = (rowv && k < K) ? *(gdbl*)(p + k) : 0.0;
    x[1] = 0.0;
  }
}

// Raw buffer loads: a resource covers one operand's extent, loads past it return
// zeros (no fault), so masked lanes need no branches.  Word 3 is the gfx9 raw
// buffer format.
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));
typedef unsigned int v3u32 __attribute__((ext_vector_type(3)));
constexpr int kBufWord3 = 0x00020000;
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufWord3);
}
__device__ inline void buf_pair(__amdgpu_buffer_rsrc_t r, int e, double* x) {
  const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(r, e * 8, 0, 0);
  __builtin_memcpy(&x[0], &v, 8);
  __builtin_memcpy(&x[1], reinterpret_cast<const char*>(&v) + 8, 8);
}
__device__ inline double buf_one(__amdgpu_buffer_rsrc_t r, int e) {
  const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0);
  double x;
  __builtin_memcpy(&x, &v, 8);
  return x;
}

// One wave computes a (16 RB) x (16 CB) tile: RB x CB fp64 16x16x4 MFMA blocks.
// BUF: every item is known (checked on the host) to fit the buffer-load path, so
// the kernel holds that path alone; otherwise the plain-load paths.  Keeping the
// two apart lets one set of accumulators serve the whole kernel.
template <int MODE, int RB, int CB, bool BUF>
__device__ inline void w32_tile(const GemmUnit& u, const GemmItem* __restrict__ items, int lane) {
  const int r = lane & 15, kq = lane >> 4;
  int am[RB], bn[CB];
  bool av[RB], bv[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    am[i] = u.m0 + 16 * i + r;
    av[i] = am[i] < u.M;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    bn[j] = u.n0 + 16 * j + r;
    bv[j] = bn[j] < u.N;
  }
  v4d acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  // the next item's descriptor is fetched while the current item computes
  GemmItem gnext;
  if (u.ib < u.ie) gnext = items[u.ib];
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = gnext;
    if (it + 1 < u.ie) gnext = items[it + 1];
    const double* A = (const double*)g.A;
    const double* B = (const double*)g.B;
    const double c = g.coef;
    // elements of A and B the unit can touch (row-major, leading dims lda, ldb)
    const long ea = (long)(u.M - 1) * g.lda + g.K;
    const long eb = MODE == GEMM_NT ? (long)(u.N - 1) * g.ldb + g.K : (long)(g.K - 1) * g.ldb + u.N;
    if constexpr (BUF) {
      // Same k pairing as below, through buffer loads: a masked row starts past
      // the extent (its loads read zeros), a k past K is zeroed by a select.
      const __amdgpu_buffer_rsrc_t ra = buf_rsrc(A, ea * 8), rb = buf_rsrc(B, eb * 8);
      int ao[RB], bo[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) ao[i] = av[i] ? am[i] * g.lda : (int)ea;
#pragma unroll
      for (int j = 0; j < CB; ++j) bo[j] = MODE == GEMM_NT ? (bv[j] ? bn[j] * g.ldb : (int)eb) : bn[j];
      const int kfull = g.K - (g.K & 7) + ((g.K & 7) > 4 ? 8 : 0);  // paired blocks; a tail of <= 4 goes alone
      // raw loads of block k0 (masking applied at use), so block k0+8 can be in
      // flight while block k0 is multiplied
      double ta[RB][2], tb[CB][2];
      auto raw = [&](int k0, double (&xa)[RB][2], double (&xb)[CB][2]) {
        const int kk = k0 + 2 * kq;
#pragma unroll
        for (int i = 0; i < RB; ++i) buf_pair(ra, ao[i] + kk, xa[i]);
        if constexpr (MODE == GEMM_NT) {
#pragma unroll
          for (int j = 0; j < CB; ++j) buf_pair(rb, bo[j] + kk, xb[j]);
        } else {
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            xb[j][0] = buf_one(rb, kk * g.ldb + bo[j]);
            xb[j][1] = buf_one(rb, (kk + 1) * g.ldb + bo[j]);
          }
        }
      };
      if (kfull > 0) raw(0, ta, tb);
      for (int k0 = 0; k0 < kfull; k0 += 8) {
        double na[RB][2], nb[CB][2];
        if (k0 + 8 < kfull) raw(k0 + 8, na, nb);
        const int kk = k0 + 2 * kq;
        const bool k0v = kk < g.K, k1v = kk + 1 < g.K;
        double a[RB][2], b[CB][2];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          a[i][0] = k0v ? ta[i][0] * c : 0.0;
          a[i][1] = k1v ? ta[i][1] * c : 0.0;
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          b[j][0] = ((MODE == GEMM_NT || bv[j]) && k0v) ? tb[j][0] : 0.0;
          b[j][1] = ((MODE == GEMM_NT || bv[j]) && k1v) ? tb[j][1] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][h], b[j][h], acc[i][j], 0, 0, 0);
        if (k0 + 8 < kfull) {
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            ta[i][0] = na[i][0];
            ta[i][1] = na[i][1];
          }
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            tb[j][0] = nb[j][0];
            tb[j][1] = nb[j][1];
          }
        }
      }
      if (kfull < g.K) {  // last 1..4 k: one MFMA step, lane kq takes k = kfull + kq
        const int kk = kfull + kq;
        const bool kv = kk < g.K;
        double a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const double t = buf_one(ra, ao[i] + kk);
          a[i] = kv ? t * c : 0.0;
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const double t = MODE == GEMM_NT ? buf_one(rb, bo[j] + kk) : buf_one(rb, kk * g.ldb + bo[j]);
          b[j] = (kv && (MODE == GEMM_NT || bv[j])) ? t : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else if constexpr (MODE == GEMM_NT || MODE == GEMM_NN) {
      (void)ea;
      (void)eb;
      // A runs along k in memory: lane (r, kq) loads the pair k0+2kq, k0+2kq+1 of
      // its rows with one 16-byte load, and the two MFMA steps of an 8-deep block
      // take the even and the odd k of the pairs (the same k order for B, so the
      // product is unchanged).  In NT mode B runs along k too; in NN mode its rows
      // kk and kk+1 are contiguous in n.
      const double* pa[RB];
      const double* pb[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) pa[i] = A + (long)(av[i] ? am[i] : 0) * g.lda;
#pragma unroll
      for (int j = 0; j < CB; ++j) pb[j] = B + (long)(bv[j] ? bn[j] : 0) * g.ldb;
      for (int k0 = 0; k0 < g.K; k0 += 8) {
        const int kk = k0 + 2 * kq;
        double a[RB][2], b[CB][2];
#pragma unroll
        for (int i = 0; i < RB; ++i) ld_pair(pa[i], kk, g.K, av[i], a[i]);
        if constexpr (MODE == GEMM_NT) {
#pragma unroll
          for (int j = 0; j < CB; ++j) ld_pair(pb[j], kk, g.K, bv[j], b[j]);
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bool kv = kk + h < g.K;
            const gdbl* brow = (const gdbl*)(B + (long)(kv ? kk + h : 0) * g.ldb);
#pragma unroll
            for (int j = 0; j < CB; ++j) b[j][h] = (bv[j] && kv) ? brow[bn[j]] : 0.0;
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const double x = a[i][h] * c;
#pragma unroll
            for (int j = 0; j < CB; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, b[j][h], acc[i][j], 0, 0, 0);
          }
      }
    } else {
      for (int k0 = 0; k0 < g.K; k0 += 4) {
        const int ka = k0 + kq;
        const bool kv = ka < g.K;
        double a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) a[i] = (av[i] && kv) ? ld_a<MODE>(A, g.lda, am[i], ka) * c : 0.0;
#pragma unroll
        for (int j = 0; j < CB; ++j) b[j] = (bv[j] && kv) ? ld_b<MODE>(B, g.ldb, ka, bn[j]) : 0.0;
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  double* C = (double*)u.C;
  // accumulator element q of lane l: row l/16 + 4q, column l%16 (fp64 16x16x4 layout)
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int tr = 16 * i + kq + 4 * q, tc = 16 * j + r;
        int gm = u.m0 + tr, gn = u.n0 + tc;
        double v = acc[i][j][q];
        if (u.accumulate == 2) {
          C[tr * (16 * CB) + tc] = v;  // partial slot, full tile (masked entries are zero)
        } else if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

// TAG only names otherwise identical instantiations, so a profiler can tell
// launches apart (e.g. sigma phases, timed and untimed work).
template <int MODE, int TAG, bool BUF>
__global__ __launch_bounds__(256) void gemm_f64_w32(const GemmUnit* __restrict__ units,
                                                    const GemmItem* __restrict__ items, int n_units) {
  // the wave index is uniform across the wave; saying so keeps the unit and item
  // descriptors (and the buffer resources built from them) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // NN launches (sigma phase A: a factor block feeds every column tile of its
  // unit) give each XCD a contiguous range of units, so a block is fetched into
  // one XCD's L2; workgroups are dispatched to the 8 XCDs round-robin.  NT
  // launches keep the plain order, which measured faster for sigma's long-K
  // products when they ran on this kernel.
  int wg = blockIdx.x;
  if constexpr (MODE == GEMM_NN) {
    const int nb = gridDim.x, q = nb >> 3, rem = nb & 7, x = wg & 7;
    wg = x * q + min(x, rem) + (wg >> 3);
  }
  const int ui = wg * 4 + wave;
  if (ui >= n_units) return;  // whole wave exits; the kernel has no barriers
  const GemmUnit u = units[ui];
  switch (u.shape) {  // 8 * RB + CB: tile (16 RB) x (16 CB)
    case 9: w32_tile<MODE, 1, 1, BUF>(u, items, lane); break;
    case 10: w32_tile<MODE, 1, 2, BUF>(u, items, lane); break;
    case 17: w32_tile<MODE, 2, 1, BUF>(u, items, lane); break;
    case 25: w32_tile<MODE, 3, 1, BUF>(u, items, lane); break;
    case 26: w32_tile<MODE, 3, 2, BUF>(u, items, lane); break;
    case 33: w32_tile<MODE, 4, 1, BUF>(u, items, lane); break;
    case 34: w32_tile<MODE, 4, 2, BUF>(u, items, lane); break;
    default: w32_tile<MODE, 2, 2, BUF>(u, items, lane); break;
  }
}

__device__ inline void buf_pair_f32(__amdgpu_buffer_rsrc_t r, int e, float* x) {
  const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(r, e * 4, 0, 0);
  __builtin_memcpy(&x[0], &v, 4);
  __builtin_memcpy(&x[1], reinterpret_cast<const char*>(&v) + 4, 4);
}
__device__ inline float buf_one_f32(__amdgpu_buffer_rsrc_t r, int e) {
  const unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(r, e * 4, 0, 0);
  float x;
  __builtin_memcpy(&x, &v, 4);
  return x;
}

// Block kernel for long item lists in NT mode (fp64 or fp32): one workgroup per unit,
// whose tile ((16 RB) x (16 CB), up to 96 x 64) covers a whole output block of
// the sizes a sigma meets, so every item's operands are read once per block
// rather than once per one-wave tile.  Wave w computes columns 16w .. 16w + 15
// of all RB row blocks.  A slices (c * A, rows m, k contiguous in memory) are
// staged through LDS, transposed to As[k][m] and shared by the four waves; each
// wave reads its own 16 rows of B straight from memory.  LDS holds A as
// As[m][k], so each lane writes and reads its k pair with one 16-byte LDS op.  Items are walked in
// k slices of 32 with one slice of lookahead: the next slice's loads are issued
// before the current slice's MFMAs, and one barrier per slice hands the LDS
// buffers over.  Requires the buffer-load reach of every item (host-checked).
constexpr int kWgKs = 32;   // k slice
constexpr int kWgPk = 34;   // LDS row pitch (elements) of As[m][k]: 16-byte aligned k pairs; 16
                            // lanes reading rows m..m+15 at one k pair hit 16 distinct 4-bank groups

struct WgStage {
  int it;  // item index, or -1 past the end
  int k0;  // first k of the slice
};

// Element-type specifics of the block kernel: fp64 on v_mfma_f64_16x16x4f64
// (accumulator element q of lane l: row l/16 + 4q), fp32 on
// v_mfma_f32_16x16x4f32 (row 4 (l/16) + q); both take A[row l%16][k l/16] and
// B[k l/16][col l%16] per 4-deep step, so the k pairing is shared.
template <typename T>
struct WgType;
template <>
struct WgType<double> {
  typedef v4d acc_t;
  __device__ static void pair(__amdgpu_buffer_rsrc_t r, int e, double* x) { buf_pair(r, e, x); }
  __device__ static acc_t mfma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int kq, int q) { return kq + 4 * q; }
};
template <>
struct WgType<float> {
  typedef v4f acc_t;
  __device__ static void pair(__amdgpu_buffer_rsrc_t r, int e, float* x) { buf_pair_f32(r, e, x); }
  __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int kq, int q) { return 4 * kq + q; }
};

// Item descriptors are fetched one item ahead with a vector load (lane l < 10
// takes dword l) and moved to scalar registers with readlane when used.  A
// scalar load would share its wait counter with the LDS operations, so every
// LDS wait of the slice would also wait for the descriptor to come from memory.
__device__ inline uint32_t desc_word(const GemmItem* items, int j, int lane) {
  return reinterpret_cast<const uint32_t*>(items + j)[lane < 10 ? lane : 0];
}
__device__ inline GemmItem desc_unpack(uint32_t w) {
  uint32_t d[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) d[i] = __builtin_amdgcn_readlane(w, i);
  GemmItem g;
  __builtin_memcpy(&g, d, sizeof(GemmItem));
  return g;
}

template <typename T, int RB>
__device__ inline void wg_tile(const GemmUnit& u, const GemmItem* __restrict__ items, T (*As)[96][kWgPk]) {
  typedef WgType<T> W;
  typedef typename W::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, kq = lane >> 4;
  const int CB = u.shape & 7;
  const bool active = wave < CB;  // wave-uniform
  const int bn = u.n0 + 16 * wave + r;
  const bool bv = active && bn < u.N;
  acc_t acc[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) acc[i] = acc_t{};
  // A staging: 16 RB rows x 16 k-pairs per slice, RB pair loads per thread
  T sa[RB][2];
  T sb[4][2];  // this lane's B pairs of the slice: k = k0 + 8 pb + 2 kq (+1)
  auto load = [&](const GemmItem& g, int k0, T (&xa)[RB][2], T (&xb)[4][2]) {
    const long ea = (long)(u.M - 1) * g.lda + g.K;
    const long eb = (long)(u.N - 1) * g.ldb + g.K;
    const __amdgpu_buffer_rsrc_t ra = buf_rsrc(g.A, ea * (long)sizeof(T)), rb = buf_rsrc(g.B, eb * (long)sizeof(T));
    // pairs wholly past K are not fetched (their values are never used)
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int idx = tid + 256 * j, m = idx >> 4, kp = idx & 15;
      const int gm = u.m0 + m;
      const int off = gm < u.M ? gm * g.lda : (int)ea;
      if (k0 + 2 * kp < g.K) W::pair(ra, off + k0 + 2 * kp, xa[j]);
    }
    if (active) {
      const int off = bv ? bn * g.ldb : (int)eb;
#pragma unroll
      for (int pb = 0; pb < 4; ++pb)
        if (k0 + 8 * pb < g.K) W::pair(rb, off + k0 + 8 * pb + 2 * kq, xb[pb]);
    }
  };
  auto stash = [&](const GemmItem& g, int k0, const T (&xa)[RB][2], int buf) {
    const T c = (T)g.coef;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int idx = tid + 256 * j, m = idx >> 4, kp = idx & 15;
      const int k = k0 + 2 * kp;
      T* dst = &As[buf][m][2 * kp];
      dst[0] = k < g.K ? xa[j][0] * c : (T)0;
      dst[1] = k + 1 < g.K ? xa[j][1] * c : (T)0;
    }
  };
  auto next = [&](WgStage s, int K) -> WgStage {
    if (s.k0 + kWgKs < K) return {s.it, s.k0 + kWgKs};
    return {s.it + 1 < u.ie ? s.it + 1 : -1, 0};
  };
  WgStage cur{u.ib < u.ie ? u.ib : -1, 0};
  GemmItem g{};     // current item
  uint32_t qw = 0;  // the next item's descriptor (one dword per lane), fetched one item ahead
  int buf = 0;
  if (cur.it >= 0) {
    g = items[cur.it];
    load(g, 0, sa, sb);
    if (cur.it + 1 < u.ie) qw = desc_word(items, cur.it + 1, lane);
    stash(g, 0, sa, 0);
  }
  __syncthreads();
  while (cur.it >= 0) {
    const WgStage nx = next(cur, g.K);
    const bool new_item = nx.it >= 0 && nx.it != cur.it;
    const GemmItem gn = new_item ? desc_unpack(qw) : g;
    T na[RB][2], nb[4][2];
    if (nx.it >= 0) load(gn, nx.k0, na, nb);
    if (new_item && nx.it + 1 < u.ie) qw = desc_word(items, nx.it + 1, lane);
    if (active) {
      // pair blocks of this slice: k = k0 + 8 pb + 2 kq + h, zeroed past K in A
      const int np = (min(kWgKs, g.K - cur.k0) + 7) >> 3;
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) {
        if (pb < np) {
          const int kk = 8 * pb + 2 * kq;
          const bool k0v = cur.k0 + kk < g.K, k1v = cur.k0 + kk + 1 < g.K;
          const T b0 = (bv && k0v) ? sb[pb][0] : (T)0, b1 = (bv && k1v) ? sb[pb][1] : (T)0;
          T a[RB][2];
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const T* src = &As[buf][16 * i + r][kk];
            a[i][0] = src[0];
            a[i][1] = src[1];
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) acc[i] = W::mfma(a[i][0], b0, acc[i]);
#pragma unroll
          for (int i = 0; i < RB; ++i) acc[i] = W::mfma(a[i][1], b1, acc[i]);
        }
      }
    }
    if (nx.it >= 0) stash(gn, nx.k0, na, buf ^ 1);
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      sb[pb][0] = nb[pb][0];
      sb[pb][1] = nb[pb][1];
    }
    __syncthreads();
    buf ^= 1;
    cur = nx;
    g = gn;
  }
  if (!active) return;
  T* C = (T*)u.C;
  const int tn = 16 * CB;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tr = 16 * i + W::row(kq, q), tc = 16 * wave + r;
      const int gm = u.m0 + tr, gn = u.n0 + tc;
      const T v = acc[i][q];
      if (u.accumulate == 2) {
        C[tr * tn + tc] = v;  // partial slot, full tile
      } else if (gm < u.M && gn < u.N) {
        const long idx = (long)gm * u.ldc + gn;
        C[idx] = u.accumulate ? C[idx] + v : v;
      }
    }
}

template <typename T, int TAG>
__global__ __launch_bounds__(256) void gemm_wg(const GemmUnit* __restrict__ units,
                                               const GemmItem* __restrict__ items, int n_units) {
  __shared__ __align__(16) T As[2][96][kWgPk];
  if ((int)blockIdx.x >= n_units) return;
  const GemmUnit u = units[blockIdx.x];
  switch (u.shape >> 3) {  // RB; the tile is (16 RB) x (16 CB), CB = shape & 7
    case 1: wg_tile<T, 1>(u, items, As); break;
    case 2: wg_tile<T, 2>(u, items, As); break;
    case 3: wg_tile<T, 3>(u, items, As); break;
    case 4: wg_tile<T, 4>(u, items, As); break;
    case 5: wg_tile<T, 5>(u, items, As); break;
    default: wg_tile<T, 6>(u, items, As); break;
  }
}

// fp32 operands, fp32 accumulation (the precision form): the same one-wave tiles,
// k pairing and buffer loads as the fp64 kernel, on v_mfma_f32_16x16x4f32, whose
// accumulator element q of lane l is row 4 (l/16) + q, column l%16.
template <int MODE, int RB, int CB, bool BUF>
__device__ inline void w32_tile_f32(const GemmUnit& u, const GemmItem* __restrict__ items, int lane) {
  const int r = lane & 15, kq = lane >> 4;
  int am[RB], bn[CB];
  bool av[RB], bv[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    am[i] = u.m0 + 16 * i + r;
    av[i] = am[i] < u.M;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    bn[j] = u.n0 + 16 * j + r;
    bv[j] = bn[j] < u.N;
  }
  v4f acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  GemmItem gnext;
  if (u.ib < u.ie) gnext = items[u.ib];
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = gnext;
    if (it + 1 < u.ie) gnext = items[it + 1];
    const float* A = (const float*)g.A;
    const float* B = (const float*)g.B;
    const float c = (float)g.coef;
    const long ea = MODE == GEMM_TN ? (long)(g.K - 1) * g.lda + u.M : (long)(u.M - 1) * g.lda + g.K;
    const long eb = MODE == GEMM_NT ? (long)(u.N - 1) * g.ldb + g.K : (long)(g.K - 1) * g.ldb + u.N;
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t ra = buf_rsrc(A, ea * 4), rb = buf_rsrc(B, eb * 4);
      int ao[RB], bo[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) ao[i] = av[i] ? am[i] * g.lda : (int)ea;
#pragma unroll
      for (int j = 0; j < CB; ++j) bo[j] = MODE == GEMM_NT ? (bv[j] ? bn[j] * g.ldb : (int)eb) : bn[j];
      const int kfull = g.K - (g.K & 7) + ((g.K & 7) > 4 ? 8 : 0);
      for (int k0 = 0; k0 < kfull; k0 += 8) {
        const int kk = k0 + 2 * kq;
        const bool k0v = kk < g.K, k1v = kk + 1 < g.K;
        float a[RB][2], b[CB][2];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          float t[2];
          buf_pair_f32(ra, ao[i] + kk, t);
          a[i][0] = k0v ? t[0] * c : 0.f;
          a[i][1] = k1v ? t[1] * c : 0.f;
        }
        if constexpr (MODE == GEMM_NT) {
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            float t[2];
            buf_pair_f32(rb, bo[j] + kk, t);
            b[j][0] = k0v ? t[0] : 0.f;
            b[j][1] = k1v ? t[1] : 0.f;
          }
        } else {
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            const float t0 = buf_one_f32(rb, kk * g.ldb + bo[j]);
            const float t1 = buf_one_f32(rb, (kk + 1) * g.ldb + bo[j]);
            b[j][0] = (bv[j] && k0v) ? t0 : 0.f;
            b[j][1] = (bv[j] && k1v) ? t1 : 0.f;
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][h], b[j][h], acc[i][j], 0, 0, 0);
      }
      if (kfull < g.K) {
        const int kk = kfull + kq;
        const bool kv = kk < g.K;
        float a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const float t = buf_one_f32(ra, ao[i] + kk);
          a[i] = kv ? t * c : 0.f;
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const float t = MODE == GEMM_NT ? buf_one_f32(rb, bo[j] + kk) : buf_one_f32(rb, kk * g.ldb + bo[j]);
          b[j] = (kv && (MODE == GEMM_NT || bv[j])) ? t : 0.f;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
      // any mode, any extent: element loads behind lane masks
      for (int k0 = 0; k0 < g.K; k0 += 4) {
        const int ka = k0 + kq;
        const bool kv = ka < g.K;
        float a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i)
          a[i] = (av[i] && kv)
                     ? (MODE == GEMM_TN ? A[(long)ka * g.lda + am[i]] : A[(long)am[i] * g.lda + ka]) * c
                     : 0.f;
#pragma unroll
        for (int j = 0; j < CB; ++j)
          b[j] = (bv[j] && kv) ? (MODE == GEMM_NT ? B[(long)bn[j] * g.ldb + ka] : B[(long)ka * g.ldb + bn[j]])
                               : 0.f;
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  float* C = (float*)u.C;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int tr = 16 * i + 4 * kq + q, tc = 16 * j + r;
        int gm = u.m0 + tr, gn = u.n0 + tc;
        float v = acc[i][j][q];
        if (u.accumulate == 2) {
          C[tr * (16 * CB) + tc] = v;
        } else if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

template <int MODE, bool BUF>
__global__ __launch_bounds__(256) void gemm_f32_w32(const GemmUnit* __restrict__ units,
                                                    const GemmItem* __restrict__ items, int n_units) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ui = blockIdx.x * 4 + wave;
  if (ui >= n_units) return;
  const GemmUnit u = units[ui];
  switch (u.shape) {
    case 9: w32_tile_f32<MODE, 1, 1, BUF>(u, items, lane); break;
    case 10: w32_tile_f32<MODE, 1, 2, BUF>(u, items, lane); break;
    case 17: w32_tile_f32<MODE, 2, 1, BUF>(u, items, lane); break;
    case 25: w32_tile_f32<MODE, 3, 1, BUF>(u, items, lane); break;
    case 26: w32_tile_f32<MODE, 3, 2, BUF>(u, items, lane); break;
    case 33: w32_tile_f32<MODE, 4, 1, BUF>(u, items, lane); break;
    case 34: w32_tile_f32<MODE, 4, 2, BUF>(u, items, lane); break;
    default: w32_tile_f32<MODE, 2, 2, BUF>(u, items, lane); break;
  }
}

// bf16 operands, fp32 accumulation on v_mfma_f32_16x16x16bf16_1k: lane (r, kq)
// supplies A[row r][4 kq .. 4 kq + 3] and B[4 kq .. 4 kq + 3][col r] of each
// 16-deep k step; its accumulator layout is the fp32 one.  A is bf16 bits
// (AF32 = false) or fp32 rounded to bf16 after the item coefficient (AF32 =
// true); B is bf16 bits.  Same one-wave tiles and buffer loads as above.
// Four consecutive bf16 elements from element offset e, which may be odd.  Wide
// buffer loads need dword-aligned addresses, so three dwords are read from the
// even element at or below e and shifted down by 16 bits when e is odd.
__device__ inline void bf16_quad(__amdgpu_buffer_rsrc_t r, int e, uint16_t (&hb)[4]) {
  const v3u32 v = __builtin_amdgcn_raw_buffer_load_b96(r, (e & ~1) * 2, 0, 0);
  const uint32_t sh = (e & 1) * 16;
  const uint32_t w0 = __builtin_amdgcn_alignbit(v[1], v[0], sh), w1 = __builtin_amdgcn_alignbit(v[2], v[1], sh);
  hb[0] = (uint16_t)w0;
  hb[1] = (uint16_t)(w0 >> 16);
  hb[2] = (uint16_t)w1;
  hb[3] = (uint16_t)(w1 >> 16);
}

template <bool AF32>
__device__ inline void a_quad(__amdgpu_buffer_rsrc_t r, int e, float c, int kk, int K, v4s& out) {
  float x[4];
  if constexpr (AF32) {
    const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(r, e * 4, 0, 0);
    __builtin_memcpy(x, &v, 16);
  } else {
    uint16_t hb[4];
    bf16_quad(r, e, hb);
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = __uint_as_float(((uint32_t)hb[q]) << 16);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = (short)(kk + q < K ? f2bf(x[q] * c) : 0);
}
__device__ inline void b_quad_rows(__amdgpu_buffer_rsrc_t r, int e, int kk, int K, v4s& out) {
  uint16_t hb[4];
  bf16_quad(r, e, hb);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = (short)(kk + q < K ? hb[q] : 0);
}
__device__ inline uint16_t buf_bf16(__amdgpu_buffer_rsrc_t r, int e) {
  const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, e * 2, 0, 0);
  return (uint16_t)v;
}

template <int MODE, bool AF32, int RB, int CB, bool BUF>
__device__ inline void w32_tile_bf16(const GemmUnit& u, const GemmItem* __restrict__ items, int lane) {
  const int r = lane & 15, kq = lane >> 4;
  int am[RB], bn[CB];
  bool av[RB], bv[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    am[i] = u.m0 + 16 * i + r;
    av[i] = am[i] < u.M;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    bn[j] = u.n0 + 16 * j + r;
    bv[j] = bn[j] < u.N;
  }
  v4f acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  constexpr int ea_sz = AF32 ? 4 : 2;
  GemmItem gnext;
  if (u.ib < u.ie) gnext = items[u.ib];
  for (int it = u.ib; it < u.ie; ++it) {
    const GemmItem g = gnext;
    if (it + 1 < u.ie) gnext = items[it + 1];
    const float c = (float)g.coef;
    const long ea = MODE == GEMM_TN ? (long)(g.K - 1) * g.lda + u.M : (long)(u.M - 1) * g.lda + g.K;
    const long eb = MODE == GEMM_NT ? (long)(u.N - 1) * g.ldb + g.K : (long)(g.K - 1) * g.ldb + u.N;
    if constexpr (BUF) {
      // bf16 operands may start at an odd element: the descriptors start at the
      // dword boundary below, and element offsets count from there, so that the
      // parity test in bf16_quad sees the true address parity.  The range check
      // of buffer loads works on whole dwords, so the extents are rounded up to
      // the dword holding the last element (same dword, no wider access).
      const int a_sh = AF32 ? 0 : (int)(((uintptr_t)g.A >> 1) & 1), b_sh = (int)(((uintptr_t)g.B >> 1) & 1);
      const __amdgpu_buffer_rsrc_t ra =
          buf_rsrc((const char*)g.A - 2 * a_sh, ((ea + a_sh) * ea_sz + 3) & ~3L);
      const __amdgpu_buffer_rsrc_t rb = buf_rsrc((const char*)g.B - 2 * b_sh, ((eb + b_sh) * 2 + 3) & ~3L);
      int ao[RB], bo[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) ao[i] = (av[i] ? am[i] * g.lda : (int)ea) + a_sh;
#pragma unroll
      for (int j = 0; j < CB; ++j) bo[j] = (MODE == GEMM_NT ? (bv[j] ? bn[j] * g.ldb : (int)eb) : bn[j]) + b_sh;
      for (int k0 = 0; k0 < g.K; k0 += 16) {
        const int kk = k0 + 4 * kq;
        v4s a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) a_quad<AF32>(ra, ao[i] + kk, c, kk, g.K, a[i]);
        if constexpr (MODE == GEMM_NT) {
#pragma unroll
          for (int j = 0; j < CB; ++j) b_quad_rows(rb, bo[j] + kk, kk, g.K, b[j]);
        } else {
#pragma unroll
          for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const uint16_t v = buf_bf16(rb, (kk + q) * g.ldb + bo[j]);
              b[j][q] = (short)((bv[j] && kk + q < g.K) ? v : 0);
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
      // any mode, any extent: element loads behind lane masks
      for (int k0 = 0; k0 < g.K; k0 += 16) {
        const int kk = k0 + 4 * kq;
        v4s a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = kk + q;
            float x = 0.f;
            if (av[i] && k < g.K) {
              const long e = MODE == GEMM_TN ? (long)k * g.lda + am[i] : (long)am[i] * g.lda + k;
              x = AF32 ? ((const float*)g.A)[e] : to_f(((const uint16_t*)g.A)[e]);
            }
            a[i][q] = (short)f2bf(x * c);
          }
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = kk + q;
            uint16_t v = 0;
            if (bv[j] && k < g.K)
              v = ((const uint16_t*)g.B)[MODE == GEMM_NT ? (long)bn[j] * g.ldb + k : (long)k * g.ldb + bn[j]];
            b[j][q] = (short)v;
          }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  float* C = (float*)u.C;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int tr = 16 * i + 4 * kq + q, tc = 16 * j + r;
        int gm = u.m0 + tr, gn = u.n0 + tc;
        float v = acc[i][j][q];
        if (u.accumulate == 2) {
          C[tr * (16 * CB) + tc] = v;
        } else if (gm < u.M && gn < u.N) {
          long idx = (long)gm * u.ldc + gn;
          C[idx] = u.accumulate ? C[idx] + v : v;
        }
      }
}

template <int MODE, bool AF32, bool BUF>
__global__ __launch_bounds__(256) void gemm_bf16_w32(const GemmUnit* __restrict__ units,
                                                     const GemmItem* __restrict__ items, int n_units) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ui = blockIdx.x * 4 + wave;
  if (ui >= n_units) return;
  const GemmUnit u = units[ui];
  switch (u.shape) {
    case 9: w32_tile_bf16<MODE, AF32, 1, 1, BUF>(u, items, lane); break;
    case 10: w32_tile_bf16<MODE, AF32, 1, 2, BUF>(u, items, lane); break;
    case 17: w32_tile_bf16<MODE, AF32, 2, 1, BUF>(u, items, lane); break;
    case 25: w32_tile_bf16<MODE, AF32, 3, 1, BUF>(u, items, lane); break;
    case 26: w32_tile_bf16<MODE, AF32, 3, 2, BUF>(u, items, lane); break;
    case 33: w32_tile_bf16<MODE, AF32, 4, 1, BUF>(u, items, lane); break;
    case 34: w32_tile_bf16<MODE, AF32, 4, 2, BUF>(u, items, lane); break;
    default: w32_tile_bf16<MODE, AF32, 2, 2, BUF>(u, items, lane); break;
  }
}

__global__ void splitk_reduce_f32(const SplitTile* __restrict__ tiles, const float* __restrict__ slots) {
  // workgroup (tile, chunk of 256 elements): one element per thread
  const SplitTile t = tiles[blockIdx.x];
  const int e = blockIdx.y * blockDim.x + threadIdx.x;
  if (e >= t.tm * t.tn) return;
  const int tr = e / t.tn, tc = e - tr * t.tn;
  const int gm = t.m0 + tr, gn = t.n0 + tc;
  if (gm >= t.M || gn >= t.N) return;
  float acc = 0.f;
  const long step = (long)t.tm * t.tn;
  for (int s = 0; s < t.ns; ++s) acc += slots[t.s0 + s * step + e];
  float* c = (float*)t.C + (long)gm * t.ldc + gn;
  *c = t.acc ? *c + acc : acc;
}

// Split-K reduction: out tile = (out tile if acc) + sum of its partial slots in order.
__global__ void splitk_reduce(const SplitTile* __restrict__ tiles, const double* __restrict__ slots) {
  // workgroup (tile, chunk of 256 elements): one element per thread
  const SplitTile t = tiles[blockIdx.x];
  const int e = blockIdx.y * blockDim.x + threadIdx.x;
  if (e >= t.tm * t.tn) return;
  const int tr = e / t.tn, tc = e - tr * t.tn;
  const int gm = t.m0 + tr, gn = t.n0 + tc;
  if (gm >= t.M || gn >= t.N) return;
  double acc = 0.0;
  const long step = (long)t.tm * t.tn;
  for (int s = 0; s < t.ns; ++s) acc += slots[t.s0 + s * step + e];
  double* c = (double*)t.C + (long)gm * t.ldc + gn;
  *c = t.acc ? *c + acc : acc;
}

__global__ void premix_kernel(double* __restrict__ out, const double* const* __restrict__ srcs,
                              const int* __restrict__ ptr, const double* __restrict__ coef,
                              long nnz) {
  const int f = blockIdx.y;
  const int b = ptr[f], e = ptr[f + 1];
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < nnz;
       j += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = b; i < e; ++i) acc += coef[i] * srcs[i][j];
    out[(long)f * nnz + j] = acc;
  }
}

// out[out_off[g] + j] = sum_{i in [ptr[g], ptr[g+1])} coef[i] * srcs[i][j], j < nnz[g];
// one workgroup per group, sources summed in order.
__global__ void pairmix_kernel(double* __restrict__ out, const double* const* __restrict__ srcs,
                               const int* __restrict__ ptr, const double* __restrict__ coef,
                               const long* __restrict__ out_off, const int* __restrict__ nnz) {
  const int g = blockIdx.x;
  const int b = ptr[g], e = ptr[g + 1], n = nnz[g];
  double* o = out + out_off[g];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double acc = 0.0;
    for (int i = b; i < e; ++i) acc += coef[i] * srcs[i][j];
    o[j] = acc;
  }
}

__global__ void fill_kernel(double* x, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void copy_blocks_kernel(const int64_t* __restrict__ desc, const double* __restrict__ src,
                                   double* __restrict__ dst) {
  const int64_t* d = desc + 9 * blockIdx.x;
  const long so = d[0], srs = d[1], scs = d[2], dof = d[3], drs = d[4], dcs = d[5];
  const int rows = (int)d[6], cols = (int)d[7];
  const double sc = __longlong_as_double((long long)d[8]);
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
    int r = e / cols, c = e % cols;
    dst[dof + (long)r * drs + (long)c * dcs] = sc * src[so + (long)r * srs + (long)c * scs];
  }
}

__global__ void axpy_dev_kernel(double* __restrict__ y, const double* __restrict__ x,
                                const double* __restrict__ a, double sign, long n) {
  const double s = sign * a[0];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] += s * x[i];
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void fill_f32_kernel(float* x, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = 0.f;
}

__global__ void dots_partial(const double* __restrict__ V, long ldv, const double* __restrict__ x,
                             long n, long chunk, double* __restrict__ partial) {
  const int c = blockIdx.x, i = blockIdx.y;
  const long b = (long)c * chunk, e = min(n, b + chunk);
  const double* v = V + (long)i * ldv;
  double acc = 0.0;
  for (long j = b + threadIdx.x; j < e; j += blockDim.x) acc += v[j] * x[j];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)i * gridDim.x + c] = red[0];
}

__global__ void dots_final(const double* __restrict__ partial, int nchunk, double* __restrict__ out) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double acc = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += blockDim.x) acc += partial[(long)i * nchunk + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

__global__ void gemv_kernel(const double* __restrict__ V, long ldv, int k,
                            const double* __restrict__ coef, double alpha, double* __restrict__ out,
                            double beta, long n) {
  __shared__ double cs[128];
  for (int i = threadIdx.x; i < k; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += cs[i] * V[(long)i * ldv + j];
    out[j] = (beta == 0.0 ? 0.0 : beta * out[j]) + alpha * acc;
  }
}

__global__ void scale_by_norm_kernel(double* x, long n, const double* nrm2) {
  const double s = 1.0 / sqrt(nrm2[0]);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] *= s;
}

__global__ void precond_diag_kernel(const double* __restrict__ r, const double* __restrict__ d,
                                    const double* __restrict__ theta, double* __restrict__ out, long n) {
  const double th = theta[0];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double den = th - d[i];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    out[i] = r[i] / den;
  }
}

// Low-precision copy entries recomputed from fp64 with a shift:
// dst[idx[i]] = round(src[idx[i]] - w[i] * s) (fp32 or bf16 by `bf16`).
__global__ void shift_entries_kernel(const double* __restrict__ src, void* __restrict__ dst, int bf16,
                                     const long* __restrict__ idx, const double* __restrict__ w, long n, double s) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long e = idx[i];
    const float v = (float)(src[e] - w[i] * s);
    if (bf16) ((uint16_t*)dst)[e] = f2bf(v);
    else ((float*)dst)[e] = v;
  }
}

__global__ void axpy_ratio_kernel(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ num,
                                  const double* __restrict__ den, double sign, long n) {
  const double a = sign * num[0] / den[0];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

__global__ void xpby_ratio_kernel(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ num,
                                  const double* __restrict__ den, long n) {
  const double b = num[0] / den[0];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = z[i] + b * p[i];
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, double a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

// d[i] += sum_{j<k} V[j ldv + i]^2 (diagonal of a rank-k update V V^T).
__global__ void add_squares_kernel(double* __restrict__ d, const double* __restrict__ V, long ldv, int k, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double acc = d[i];
    for (int j = 0; j < k; ++j) {
      const double v = V[(long)j * ldv + i];
      acc = fma(v, v, acc);
    }
    d[i] = acc;
  }
}

// Symmetric eigensolver for k <= 64 in one workgroup: cyclic Jacobi with the
// round-robin (circle) pairing, so each round rotates the n/2 disjoint pairs
// (p, q) together (n = k rounded up to even; a pair holding the padding index
// is not rotated).  A pair is rotated when its coupling is significant against
// its diagonal entries.  A round maps each 2 x 2 block of A (rows of pair a,
// columns of pair b) to R_a^T A_ab R_b and each block of V to V_ab R_b; every
// thread derives the angles of its blocks' two pairs from the round's input A
// and writes the other copy of A and V, so a round has one barrier.  Per
// element this is the arithmetic of rotating all rows, then all columns.  The
// iteration ends when no pair is significant (a sweep would rotate nothing) or
// the off-diagonal part is at the rounding level.
__device__ inline void jacobi_pair(int round, int t, int n, int& p, int& q) {
  if (t == 0) {
    p = round % (n - 1);
    q = n - 1;
  } else {
    p = (round + t) % (n - 1);
    q = (round - t + (n - 1)) % (n - 1);
  }
  if (p > q) {
    const int x = p;
    p = q;
    q = x;
  }
}
__device__ inline bool jacobi_significant(double apq, double app, double aqq) {
  return fabs(apq) > 1e-300 && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq));
}
// rotation of pair (p, q), p < q < k: c = 1, s = 0 when the coupling is not significant
__device__ inline void jacobi_angle(const double (*A)[65], int p, int q, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
  if (jacobi_significant(apq, app, aqq)) {
    const double theta = (aqq - app) / (2.0 * apq);
    const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    c = 1.0 / sqrt(tt * tt + 1.0);
    s = tt * c;
  }
}

__global__ __launch_bounds__(256) void jacobi_eig_kernel(const double* __restrict__ G, int ldg, int k,
                                                         double* __restrict__ evals,
                                                         double* __restrict__ evecs) {
  __shared__ double A[2][64][65];
  __shared__ double V[2][64][65];
  __shared__ double red[3][256];
  __shared__ int order[64];
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += blockDim.x) {  // lower triangle holds the matrix
    const int i = e / k, j = e % k;
    A[0][i][j] = i >= j ? G[(long)i * ldg + j] : G[(long)j * ldg + i];
    V[0][i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n = k + (k & 1);
  const int half = n / 2;
  int cur = 0;
  for (int sweep = 0; sweep < 40 && k > 1; ++sweep) {
    double off = 0.0, dg = 0.0, sig = 0.0;
    for (int e = t; e < k * k; e += blockDim.x) {
      const int i = e / k, j = e % k;
      const double a = A[cur][i][j];
      if (i != j) off += a * a;
      else dg += a * a;
      if (i < j && jacobi_significant(a, A[cur][i][i], A[cur][j][j])) sig += 1.0;
    }
    red[0][t] = off;
    red[1][t] = dg;
    red[2][t] = sig;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) {
        red[0][t] += red[0][t + s];
        red[1][t] += red[1][t + s];
        red[2][t] += red[2][t + s];
      }
      __syncthreads();
    }
    const double offsum = red[0][0], dgsum = red[1][0], nsig = red[2][0];
    __syncthreads();  // red is written again by the next sweep's check
    if (nsig == 0.0 || offsum <= 1e-32 * (dgsum > 1e-300 ? dgsum : 1e-300)) break;  // uniform
    for (int round = 0; round < n - 1; ++round) {
      const double(*Ai)[65] = A[cur];
      const double(*Vi)[65] = V[cur];
      double(*Ao)[65] = A[cur ^ 1];
      double(*Vo)[65] = V[cur ^ 1];
      for (int e = t; e < half * half; e += blockDim.x) {
        const int a = e / half, b = e % half;
        int pa, qa, pb, qb;
        jacobi_pair(round, a, n, pa, qa);
        jacobi_pair(round, b, n, pb, qb);
        const bool va = qa < k, vb = qb < k;  // false: the pair holds the padding index
        double ca = 1.0, sa = 0.0, cb = 1.0, sb = 0.0;
        if (va) jacobi_angle(Ai, pa, qa, ca, sa);
        if (vb) jacobi_angle(Ai, pb, qb, cb, sb);
        double x00 = Ai[pa][pb], x01 = vb ? Ai[pa][qb] : 0.0;
        double x10 = va ? Ai[qa][pb] : 0.0, x11 = (va && vb) ? Ai[qa][qb] : 0.0;
        double w00 = Vi[pa][pb], w01 = vb ? Vi[pa][qb] : 0.0;
        double w10 = va ? Vi[qa][pb] : 0.0, w11 = (va && vb) ? Vi[qa][qb] : 0.0;
        if (va) {  // rows p_a, q_a
          const double y00 = ca * x00 - sa * x10, y10 = sa * x00 + ca * x10;
          const double y01 = ca * x01 - sa * x11, y11 = sa * x01 + ca * x11;
          x00 = y00;
          x10 = y10;
          x01 = y01;
          x11 = y11;
        }
        if (vb) {  // columns p_b, q_b of A and of V
          const double y00 = cb * x00 - sb * x01, y01 = sb * x00 + cb * x01;
          const double y10 = cb * x10 - sb * x11, y11 = sb * x10 + cb * x11;
          x00 = y00;
          x01 = y01;
          x10 = y10;
          x11 = y11;
          const double z00 = cb * w00 - sb * w01, z01 = sb * w00 + cb * w01;
          const double z10 = cb * w10 - sb * w11, z11 = sb * w10 + cb * w11;
          w00 = z00;
          w01 = z01;
          w10 = z10;
          w11 = z11;
        }
        Ao[pa][pb] = x00;
        Vo[pa][pb] = w00;
        if (vb) {
          Ao[pa][qb] = x01;
          Vo[pa][qb] = w01;
        }
        if (va) {
          Ao[qa][pb] = x10;
          Vo[qa][pb] = w10;
        }
        if (va && vb) {
          Ao[qa][qb] = x11;
          Vo[qa][qb] = w11;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  // ascending order of the eigenvalues, equal ones by index (a NaN counts as
  // +inf, so the ranks are a permutation): each thread ranks one value against
  // all k (independent LDS reads instead of a serial sort on one thread)
  for (int j = t; j < k; j += blockDim.x) {
    const double dj = A[cur][j][j], kj = dj == dj ? dj : INFINITY;
    int rank = 0;
    for (int i = 0; i < k; ++i) {
      const double di = A[cur][i][i], ki = di == di ? di : INFINITY;
      rank += (ki < kj || (ki == kj && i < j)) ? 1 : 0;
    }
    order[rank] = j;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    int j = e / k, i = e % k;  // eigenvector j, component i
    evecs[(long)j * k + i] = V[cur][i][order[j]];
  }
  for (int j = t; j < k; j += blockDim.x) evals[j] = A[cur][order[j]][order[j]];
}

// Subspace rotation in place: V[:, i] = sum_j V[:, j] Y[i * k + j] for i < keep
// (columns of V are vectors of length n, stride ldv; Y holds k-vectors one after
// another).  Rows are independent: each thread reads all k entries of its row
// before writing the keep new ones, so the update is safe in place.
constexpr int kRotMax = 16;
__global__ __launch_bounds__(256) void subspace_rotate_kernel(double* __restrict__ V, long ldv, int k,
                                                              const double* __restrict__ Y, int keep, long n) {
  __shared__ double Ys[64 * kRotMax];
  for (int e = threadIdx.x; e < 64 * kRotMax; e += blockDim.x) {
    const int j = e / kRotMax, i = e % kRotMax;
    Ys[e] = (j < k && i < keep) ? Y[(long)i * k + j] : 0.0;
  }
  __syncthreads();
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (long)gridDim.x * blockDim.x) {
    double acc[kRotMax];
#pragma unroll
    for (int i = 0; i < kRotMax; ++i) acc[i] = 0.0;
    for (int j = 0; j < k; ++j) {
      const double v = V[(long)j * ldv + r];
#pragma unroll
      for (int i = 0; i < kRotMax; ++i) acc[i] += v * Ys[j * kRotMax + i];
    }
#pragma unroll
    for (int i = 0; i < kRotMax; ++i)
      if (i < keep) V[(long)i * ldv + r] = acc[i];
  }
}

__global__ void f64_to_f32_kernel(const double* x, float* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void f64_to_bf16_kernel(const double* x, uint16_t* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = f2bf((float)x[i]);
}
__global__ void f32_to_f64_kernel(const float* x, double* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void diag_kernel(double* __restrict__ out, const DiagBlock* __restrict__ blocks,
                            const DiagTerm* __restrict__ terms) {
  const DiagBlock b = blocks[blockIdx.x];
  for (int e = threadIdx.x; e < b.rows * b.cols; e += blockDim.x) {
    int i = e / b.cols, j = e % b.cols;
    double acc = 0.0;
    for (int tt = b.t0; tt < b.t1; ++tt) {
      const DiagTerm& d = terms[tt];
      acc += d.w * d.x[i] * d.y[j];
    }
    out[b.out_off + (long)i * b.ld + j] = acc;
  }
}

// desc: src_off, ld, n, dst_off
__global__ void extract_diag_kernel(const int64_t* __restrict__ desc, const double* __restrict__ src,
                                    double* __restrict__ dst) {
  const int64_t* d = desc + 4 * blockIdx.x;
  for (int i = threadIdx.x; i < (int)d[2]; i += blockDim.x) dst[d[3] + i] = src[d[0] + (long)i * (d[1] + 1)];
}

inline int grid_for(long n, int bs = 256, int cap = 4096) {
  long g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

void launch_gemm_w32(int mode, int tag, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                     hipStream_t s) {
  if (n_units <= 0) return;
  dim3 grid((n_units + 3) / 4), block(256);
  if (!buf || mode == GEMM_TN) {
    if (mode == GEMM_NN) gemm_f64_w32<GEMM_NN, 0, false><<<grid, block, 0, s>>>(units, items, n_units);
    else if (mode == GEMM_NT) gemm_f64_w32<GEMM_NT, 0, false><<<grid, block, 0, s>>>(units, items, n_units);
    else gemm_f64_w32<GEMM_TN, 0, false><<<grid, block, 0, s>>>(units, items, n_units);
    return;
  }
#define DMRG_W32_LAUNCH(T)                                                                            \
  if (mode == GEMM_NN) gemm_f64_w32<GEMM_NN, T, true><<<grid, block, 0, s>>>(units, items, n_units); \
  else gemm_f64_w32<GEMM_NT, T, true><<<grid, block, 0, s>>>(units, items, n_units);
  switch (tag) {
    case 1: DMRG_W32_LAUNCH(1) break;
    case 2: DMRG_W32_LAUNCH(2) break;
    case 3: DMRG_W32_LAUNCH(3) break;
    case 4: DMRG_W32_LAUNCH(4) break;
    default: DMRG_W32_LAUNCH(0) break;
  }
#undef DMRG_W32_LAUNCH
}

void launch_gemm_wg(int prec, int tag, const GemmUnit* units, int n_units, const GemmItem* items, hipStream_t s) {
  if (n_units <= 0) return;
  // unit b on workgroup b: consecutive units (which share operands) run at the
  // same time on the 8 XCDs in turn; giving each XCD a contiguous eighth of the
  // list instead measured 1.3x slower for sigma phase B (5.5 -> 7.2 ms), and
  // runs of 2..32 consecutive units per XCD (list order kept at that grain) no
  // different (5.37-5.41 ms at CAS(20,20), M = 1024; results bitwise equal)
  const int grid = n_units;
  if (prec == PREC_F32) {
    gemm_wg<float, 0><<<grid, 256, 0, s>>>(units, items, n_units);
    return;
  }
  switch (tag) {
    case 1: gemm_wg<double, 1><<<grid, 256, 0, s>>>(units, items, n_units); break;
    case 2: gemm_wg<double, 2><<<grid, 256, 0, s>>>(units, items, n_units); break;
    case 3: gemm_wg<double, 3><<<grid, 256, 0, s>>>(units, items, n_units); break;
    case 4: gemm_wg<double, 4><<<grid, 256, 0, s>>>(units, items, n_units); break;
    case 5: gemm_wg<double, 5><<<grid, 256, 0, s>>>(units, items, n_units); break;
    default: gemm_wg<double, 0><<<grid, 256, 0, s>>>(units, items, n_units); break;
  }
}

// tiles are at most 96 x 64 = 24 chunks of 256 elements
constexpr int kReduceChunks = 24;

void launch_splitk_reduce(const SplitTile* tiles, int n, const double* slots, hipStream_t s) {
  if (n > 0) splitk_reduce<<<dim3(n, kReduceChunks), 256, 0, s>>>(tiles, slots);
}

void launch_gemm_w32_f32(int mode, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                         hipStream_t s) {
  if (n_units <= 0) return;
  dim3 grid((n_units + 3) / 4), block(256);
  if (buf && mode == GEMM_NN) gemm_f32_w32<GEMM_NN, true><<<grid, block, 0, s>>>(units, items, n_units);
  else if (buf && mode == GEMM_NT) gemm_f32_w32<GEMM_NT, true><<<grid, block, 0, s>>>(units, items, n_units);
  else if (mode == GEMM_NN) gemm_f32_w32<GEMM_NN, false><<<grid, block, 0, s>>>(units, items, n_units);
  else if (mode == GEMM_NT) gemm_f32_w32<GEMM_NT, false><<<grid, block, 0, s>>>(units, items, n_units);
  else gemm_f32_w32<GEMM_TN, false><<<grid, block, 0, s>>>(units, items, n_units);
}

void launch_gemm_w32_bf16(int mode, bool a_f32, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                          hipStream_t s) {
  if (n_units <= 0) return;
  dim3 grid((n_units + 3) / 4), block(256);
#define DMRG_BF_LAUNCH(AF)                                                                                 \
  if (buf && mode == GEMM_NN) gemm_bf16_w32<GEMM_NN, AF, true><<<grid, block, 0, s>>>(units, items, n_units);      \
  else if (buf && mode == GEMM_NT) gemm_bf16_w32<GEMM_NT, AF, true><<<grid, block, 0, s>>>(units, items, n_units); \
  else if (mode == GEMM_NN) gemm_bf16_w32<GEMM_NN, AF, false><<<grid, block, 0, s>>>(units, items, n_units);       \
  else if (mode == GEMM_NT) gemm_bf16_w32<GEMM_NT, AF, false><<<grid, block, 0, s>>>(units, items, n_units);       \
  else gemm_bf16_w32<GEMM_TN, AF, false><<<grid, block, 0, s>>>(units, items, n_units);
  if (a_f32) {
    DMRG_BF_LAUNCH(true)
  } else {
    DMRG_BF_LAUNCH(false)
  }
#undef DMRG_BF_LAUNCH
}

void launch_splitk_reduce_f32(const SplitTile* tiles, int n, const float* slots, hipStream_t s) {
  if (n > 0) splitk_reduce_f32<<<dim3(n, kReduceChunks), 256, 0, s>>>(tiles, slots);
}

void launch_gemm(int prec, int mode, const GemmUnit* units, int n_units, const GemmItem* items,
                 hipStream_t s) {
  if (n_units <= 0) return;
  dim3 grid(n_units), block(256);
  if (prec == PREC_F64) {
    if (mode == GEMM_NN) gemm_f64<GEMM_NN><<<grid, block, 0, s>>>(units, items);
    else if (mode == GEMM_NT) gemm_f64<GEMM_NT><<<grid, block, 0, s>>>(units, items);
    else gemm_f64<GEMM_TN><<<grid, block, 0, s>>>(units, items);
  } else if (prec == PREC_F32) {
    if (mode == GEMM_NN) gemm_f32<GEMM_NN, float, float><<<grid, block, 0, s>>>(units, items);
    else if (mode == GEMM_NT) gemm_f32<GEMM_NT, float, float><<<grid, block, 0, s>>>(units, items);
    else gemm_f32<GEMM_TN, float, float><<<grid, block, 0, s>>>(units, items);
  } else if (prec == PREC_BF16) {  // A: bf16, B: bf16
    if (mode == GEMM_NN) gemm_bf16<GEMM_NN, uint16_t><<<grid, block, 0, s>>>(units, items);
    else gemm_bf16<GEMM_NT, uint16_t><<<grid, block, 0, s>>>(units, items);
  } else {  // A: fp32 rounded to bf16 on load, B: bf16
    if (mode == GEMM_NN) gemm_bf16<GEMM_NN, float><<<grid, block, 0, s>>>(units, items);
    else gemm_bf16<GEMM_NT, float><<<grid, block, 0, s>>>(units, items);
  }
}

void launch_premix(double* out, const double* const* srcs, const int* ptr, const double* coef,
                   int n_out, long nnz, hipStream_t s) {
  if (n_out <= 0 || nnz <= 0) return;
  dim3 grid(grid_for(nnz, 256, 64), n_out);
  premix_kernel<<<grid, 256, 0, s>>>(out, srcs, ptr, coef, nnz);
}

void launch_pairmix(double* out, const double* const* srcs, const int* ptr, const double* coef, const long* out_off,
                    const int* nnz, int n_groups, hipStream_t s) {
  if (n_groups > 0) pairmix_kernel<<<n_groups, 256, 0, s>>>(out, srcs, ptr, coef, out_off, nnz);
}

void launch_fill(double* x, long n, double v, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<<<grid_for(n), 256, 0, s>>>(x, n, v);
}

void launch_copy_blocks(const int64_t* desc, int n_blocks, const double* src, double* dst,
                        hipStream_t s) {
  if (n_blocks <= 0) return;
  copy_blocks_kernel<<<n_blocks, 256, 0, s>>>(desc, src, dst);
}

void launch_axpy_dev(double* y, const double* x, const double* a, double sign, long n, hipStream_t s) {
  if (n > 0) axpy_dev_kernel<<<grid_for(n), 256, 0, s>>>(y, x, a, sign, n);
}

void launch_copy(double* dst, const double* src, long n, hipStream_t s) {
  if (n > 0) copy_kernel<<<grid_for(n), 256, 0, s>>>(dst, src, n);
}

void launch_fill_f32(float* x, long n, hipStream_t s) {
  if (n > 0) fill_f32_kernel<<<grid_for(n), 256, 0, s>>>(x, n);
}

void launch_dots(const double* V, long ldv, int k, const double* x, long n, double* partial,
                 double* out, hipStream_t s) {
  if (k <= 0) return;
  long chunk = 8192;
  int nchunk = (int)((n + chunk - 1) / chunk);
  if (nchunk > 512) {
    nchunk = 512;
    chunk = (n + nchunk - 1) / nchunk;
  }
  if (nchunk < 1) nchunk = 1;
  dots_partial<<<dim3(nchunk, k), 256, 0, s>>>(V, ldv, x, n, chunk, partial);
  dots_final<<<k, 256, 0, s>>>(partial, nchunk, out);
}

void launch_gemv(const double* V, long ldv, int k, const double* coef, double alpha, double* out,
                 double beta, long n, hipStream_t s) {
  gemv_kernel<<<grid_for(n), 256, 0, s>>>(V, ldv, k, coef, alpha, out, beta, n);
}

void launch_scale_by_norm(double* x, long n, const double* nrm2, hipStream_t s) {
  scale_by_norm_kernel<<<grid_for(n), 256, 0, s>>>(x, n, nrm2);
}

void launch_precond_diag(const double* r, const double* diag, const double* theta, double* out,
                         long n, hipStream_t s) {
  precond_diag_kernel<<<grid_for(n), 256, 0, s>>>(r, diag, theta, out, n);
}

void launch_shift_entries(const double* src, void* dst, bool bf16, const long* idx, const double* w, long n,
                          double shift, hipStream_t s) {
  if (n > 0) shift_entries_kernel<<<grid_for(n), 256, 0, s>>>(src, dst, bf16 ? 1 : 0, idx, w, n, shift);
}

void launch_axpy_ratio(double* y, const double* x, const double* num, const double* den, double sign, long n,
                       hipStream_t s) {
  if (n > 0) axpy_ratio_kernel<<<grid_for(n), 256, 0, s>>>(y, x, num, den, sign, n);
}

void launch_xpby_ratio(double* p, const double* z, const double* num, const double* den, long n, hipStream_t s) {
  if (n > 0) xpby_ratio_kernel<<<grid_for(n), 256, 0, s>>>(p, z, num, den, n);
}

void launch_axpy(double* y, const double* x, double a, long n, hipStream_t s) {
  if (n > 0) axpy_kernel<<<grid_for(n), 256, 0, s>>>(y, x, a, n);
}

void launch_add_squares(double* d, const double* V, long ldv, int k, long n, hipStream_t s) {
  if (n > 0 && k > 0) add_squares_kernel<<<grid_for(n), 256, 0, s>>>(d, V, ldv, k, n);
}

void launch_subspace_rotate(double* V, long ldv, int k, const double* Y, int keep, long n, hipStream_t s) {
  if (n <= 0 || keep <= 0) return;
  if (k > 64 || keep > kRotMax || keep > k) throw std::runtime_error("subspace rotation: k <= 64, keep <= 16 and <= k");
  subspace_rotate_kernel<<<grid_for(n), 256, 0, s>>>(V, ldv, k, Y, keep, n);
}

void launch_jacobi_eig(const double* G, int ldg, int k, double* evals, double* evecs,
                       hipStream_t s) {
  if (k > 64) throw std::runtime_error("subspace eigensolver: k <= 64");
  if (k > 0) jacobi_eig_kernel<<<1, 256, 0, s>>>(G, ldg, k, evals, evecs);
}

void launch_f64_to_f32(const double* x, float* y, long n, hipStream_t s) {
  if (n > 0) f64_to_f32_kernel<<<grid_for(n), 256, 0, s>>>(x, y, n);
}
void launch_f64_to_bf16(const double* x, uint16_t* y, long n, hipStream_t s) {
  if (n > 0) f64_to_bf16_kernel<<<grid_for(n), 256, 0, s>>>(x, y, n);
}
void launch_f32_to_f64(const float* x, double* y, long n, hipStream_t s) {
  if (n > 0) f32_to_f64_kernel<<<grid_for(n), 256, 0, s>>>(x, y, n);
}

void launch_diag(double* out, const DiagBlock* blocks, int n_blocks, const DiagTerm* terms,
                 hipStream_t s) {
  if (n_blocks > 0) diag_kernel<<<n_blocks, 256, 0, s>>>(out, blocks, terms);
}

void launch_extract_diag(const int64_t* desc, int n, const double* src, double* dst,
                         hipStream_t s) {
  if (n > 0) extract_diag_kernel<<<n, 64, 0, s>>>(desc, src, dst);
}

}  // namespace dmrg
