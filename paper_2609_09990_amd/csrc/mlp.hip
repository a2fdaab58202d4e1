// Learned Davidson preconditioner on gfx950: network kernels (forward, cosine
// loss, backward, Adam), per-amplitude feature kernels and the gathering of
// training triples.  Element-wise kernels and deterministic column reductions
// (fixed chunks, partials summed in order); the hidden layer's GEMMs run on the
// block-GEMM engine (see mlp_net.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstring>

#include "mlp.hpp"

namespace dmrg {

namespace {

constexpr int kThreads = 256;

inline int grid_of(long n) {
  long g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum (or min) over the 256 threads of a block, same order on every call.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}
__device__ inline double block_min(double v, double* sh) {
  v = wave_min(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  return r;
}

__global__ void layer1_kernel(const float* __restrict__ X, long n, int nin, const float* __restrict__ W1,
                              const float* __restrict__ b1, int width, float* __restrict__ a1,
                              uint16_t* __restrict__ a1b) {
  const long total = n * width;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / width;
    const int j = (int)(e - i * width);
    float z = b1[j];
    for (int f = 0; f < nin; ++f) z = fmaf(X[i * nin + f], W1[j * nin + f], z);
    z = fmaxf(z, 0.f);
    if (a1) a1[e] = z;
    if (a1b) a1b[e] = bf16_rne(z);
  }
}

// One wave per row.
__global__ void layer3_kernel(float* __restrict__ z2, long n, int width, const float* __restrict__ b2,
                              const float* __restrict__ W3, const float* __restrict__ b3, float* __restrict__ y,
                              int store) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  float* zr = z2 + row * width;
  double acc = 0.0;
  for (int j = lane; j < width; j += 64) {
    float a = fmaxf(zr[j] + b2[j], 0.f);
    acc += (double)a * W3[j];
    if (store) zr[j] = a;
  }
  acc = wave_sum(acc);
  if (lane == 0) y[row] = (float)(acc + b3[0]);
}

// Fused bf16 inference of the width-256 network, y = W3 relu(W2 relu(W1 x + b1)
// + b2) + b3, without writing activations to memory.  Persistent workgroups of
// 8 waves (one per CU: W2 in bf16, 256 x 256, is staged once in LDS with a row
// pitch of 260) walk 32-row tiles: the tile's inputs are staged in LDS; layer 1
// (thread t: columns 4 (t % 64).. whose W1 rows it keeps in registers, rows
// 4 (t / 64)..) writes bf16 to LDS, the rounding the layered path applies;
// layer 2 runs on v_mfma_f32_16x16x16 bf16 (wave w: rows 16 (w & 1).., columns
// 64 (w >> 1)..: 4 tiles of 16 x 16); layer 3 is a dot product with W3 reduced
// over lanes and the four column quarters.
constexpr int kInfW = 256, kInfRows = 32, kInfPitch = kInfW + 4, kInfThreads = 512, kInfMaxIn = 16;
typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kInfThreads) void mlp_infer_bf16_kernel(
    const float* __restrict__ X, long n, int nin, const float* __restrict__ W1, const float* __restrict__ b1,
    const uint16_t* __restrict__ W2b, const float* __restrict__ b2, const float* __restrict__ W3,
    const float* __restrict__ b3, float* __restrict__ y) {
  __shared__ __align__(16) uint16_t W2s[kInfW * kInfPitch];
  __shared__ __align__(16) uint16_t A1s[kInfRows * kInfPitch];
  __shared__ float Xs[kInfRows * kInfMaxIn];
  __shared__ float part[4][kInfRows];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kInfW * kInfW / 4; e += kInfThreads) {  // 4 bf16 (8 bytes) per step
    const int j = e / (kInfW / 4), i4 = (e % (kInfW / 4)) * 4;
    *reinterpret_cast<uint2*>(W2s + j * kInfPitch + i4) = *reinterpret_cast<const uint2*>(W2b + (long)j * kInfW + i4);
  }
  // layer-1 role of this thread: columns c0..c0+3, rows r0..r0+3 of every tile
  const int c0 = 4 * (tid & 63), r0 = 4 * (tid >> 6);
  float w1[4][kInfMaxIn], bb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bb[c] = b1[c0 + c];
#pragma unroll
    for (int f = 0; f < kInfMaxIn; ++f) w1[c][f] = f < nin ? W1[(c0 + c) * nin + f] : 0.f;
  }
  const int rb = wave & 1, cb = (wave >> 1) * 64;
  const long ntiles = (n + kInfRows - 1) / kInfRows;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long row0 = tile * kInfRows;
    __syncthreads();  // W2s staged / the previous tile's Xs, A1s and part[] read
    for (int e = tid; e < kInfRows * kInfMaxIn; e += kInfThreads) {
      const int r = e / kInfMaxIn, f = e % kInfMaxIn;
      Xs[e] = (f < nin && row0 + r < n) ? X[(row0 + r) * nin + f] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int r = r0 + rr;
      float z[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) z[c] = bb[c];
#pragma unroll
      for (int f = 0; f < kInfMaxIn; ++f) {
        const float xf = Xs[r * kInfMaxIn + f];
#pragma unroll
        for (int c = 0; c < 4; ++c) z[c] = fmaf(xf, w1[c][f], z[c]);
      }
      uint2 pk;
      pk.x = (uint32_t)bf16_rne(fmaxf(z[0], 0.f)) | ((uint32_t)bf16_rne(fmaxf(z[1], 0.f)) << 16);
      pk.y = (uint32_t)bf16_rne(fmaxf(z[2], 0.f)) | ((uint32_t)bf16_rne(fmaxf(z[3], 0.f)) << 16);
      *reinterpret_cast<uint2*>(A1s + r * kInfPitch + c0) = pk;
    }
    __syncthreads();
    v4f_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (v4f_t){0.f, 0.f, 0.f, 0.f};
    const int ar = rb * 16 + (lane & 15);
#pragma unroll 4
    for (int k0 = 0; k0 < kInfW; k0 += 16) {
      const int kk = k0 + 4 * (lane >> 4);
      const uint2 av = *reinterpret_cast<const uint2*>(A1s + ar * kInfPitch + kk);
      v4s_t a;
      a[0] = (short)(av.x & 0xffff);
      a[1] = (short)(av.x >> 16);
      a[2] = (short)(av.y & 0xffff);
      a[3] = (short)(av.y >> 16);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = cb + 16 * t + (lane & 15);  // B[k][col j] = W2[j][k]
        const uint2 bv = *reinterpret_cast<const uint2*>(W2s + j * kInfPitch + kk);
        v4s_t b;
        b[0] = (short)(bv.x & 0xffff);
        b[1] = (short)(bv.x >> 16);
        b[2] = (short)(bv.y & 0xffff);
        b[3] = (short)(bv.y >> 16);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
    // layer 3: element q of acc[t] is row 4 (lane >> 4) + q, column cb + 16 t + (lane & 15)
    float sq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = cb + 16 * t + (lane & 15);
      const float bj = b2[j], wj = W3[j];
#pragma unroll
      for (int q = 0; q < 4; ++q) sq[q] = fmaf(fmaxf(acc[t][q] + bj, 0.f), wj, sq[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) sq[q] += __shfl_xor(sq[q], m);
    if ((lane & 15) == 0)
#pragma unroll
      for (int q = 0; q < 4; ++q) part[wave >> 1][rb * 16 + 4 * (lane >> 4) + q] = sq[q];
    __syncthreads();
    if (tid < kInfRows && row0 + tid < n)
      y[row0 + tid] = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + b3[0];
  }
}

__global__ void seg_stats_kernel(const float* __restrict__ y, const float* __restrict__ t, int seglen,
                                 double* __restrict__ stats) {
  __shared__ double sh[4];
  const long base = (long)blockIdx.x * seglen;
  double yt = 0, yy = 0, tt = 0;
  for (int i = threadIdx.x; i < seglen; i += blockDim.x) {
    double a = y[base + i], b = t[base + i];
    yt += a * b;
    yy += a * a;
    tt += b * b;
  }
  yt = block_sum(yt, sh);
  yy = block_sum(yy, sh);
  tt = block_sum(tt, sh);
  if (threadIdx.x == 0) {
    stats[3 * blockIdx.x] = yt;
    stats[3 * blockIdx.x + 1] = yy;
    stats[3 * blockIdx.x + 2] = tt;
  }
}

__global__ void cos_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                const double* __restrict__ stats, int nseg, int seglen, float* __restrict__ dy) {
  const long total = (long)nseg * seglen;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long sgi = e / seglen;
    const double yt = stats[3 * sgi], yy = stats[3 * sgi + 1], tt = stats[3 * sgi + 2];
    double g = 0.0;
    if (yy > 0.0 && tt > 0.0) {
      const double ny = sqrt(yy), nt = sqrt(tt), c = yt / (ny * nt);
      g = -(t[e] / (ny * nt) - c * y[e] / yy) / nseg;
    }
    dy[e] = (float)g;
  }
}

__global__ void colsum_partial_kernel(const float* __restrict__ A, long rows, int cols, const float* __restrict__ w,
                                      int wstride, long chunk, double* __restrict__ partial) {
  const long r0 = (long)blockIdx.x * chunk;
  const long r1 = r0 + chunk < rows ? r0 + chunk : rows;
  for (int j = threadIdx.x; j < cols; j += blockDim.x) {
    double acc = 0.0;
    for (long i = r0; i < r1; ++i) acc += (double)A[i * cols + j] * (w ? (double)w[i * wstride] : 1.0);
    partial[(long)blockIdx.x * cols + j] = acc;
  }
}

__global__ void sum_partials_kernel(const double* __restrict__ partial, int nchunks, long cols,
                                    float* __restrict__ out, int ostride) {
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += partial[(long)c * cols + j];
    out[j * ostride] = (float)acc;
  }
}

__global__ void sum_partials_f32_kernel(const float* __restrict__ partial, int nchunks, long cols,
                                        float* __restrict__ out) {
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += partial[(long)c * cols + j];
    out[j] = (float)acc;
  }
}

__global__ void back3_kernel(float* __restrict__ a2, const float* __restrict__ dy, const float* __restrict__ W3,
                             long n, int width) {
  const long total = n * width;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / width;
    const int j = (int)(e - i * width);
    a2[e] = a2[e] > 0.f ? dy[i] * W3[j] : 0.f;
  }
}

__global__ void relu_mask_kernel(float* __restrict__ x, const float* __restrict__ mask, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!(mask[i] > 0.f)) x[i] = 0.f;
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
  }
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = bf16_rne(x[i]);
}

// one block per feature block: s_b = mean |d - theta|, then mean and min of (d - theta)/s_b
__global__ void feat_stats_kernel(const double* __restrict__ d, const double* __restrict__ theta,
                                  const int64_t* __restrict__ blocks, double* __restrict__ stats) {
  __shared__ double sh[4];
  const int64_t* b = blocks + 4 * blockIdx.x;
  const long off = b[0], ld = b[1];
  const int rows = (int)b[2], cols = (int)b[3];
  const long size = (long)rows * cols;
  const double th = theta[0];
  double sa = 0.0;
  for (long e = threadIdx.x; e < size; e += blockDim.x) {
    const long i = e / cols, j = e - i * cols;
    sa += fabs(d[off + i * ld + j] - th);
  }
  sa = block_sum(sa, sh);
  double s = sa / (double)size;
  if (!(s > 1e-300)) s = 1e-300;
  double su = 0.0, mn = INFINITY;
  for (long e = threadIdx.x; e < size; e += blockDim.x) {
    const long i = e / cols, j = e - i * cols;
    const double u = (d[off + i * ld + j] - th) / s;
    su += u;
    mn = fmin(mn, u);
  }
  su = block_sum(su, sh);
  mn = block_min(mn, sh);
  if (threadIdx.x == 0) {
    stats[4 * blockIdx.x] = s;
    stats[4 * blockIdx.x + 1] = su / (double)size;
    stats[4 * blockIdx.x + 2] = mn;
    stats[4 * blockIdx.x + 3] = log((double)size) / 10.0;
  }
}

__global__ void feat_fill_kernel(const double* __restrict__ r, const double* __restrict__ d,
                                 const double* __restrict__ theta, const double* __restrict__ t,
                                 const int64_t* __restrict__ blocks, const double* __restrict__ stats,
                                 const double* __restrict__ nrr, const double* __restrict__ ntt, long n, float kpos,
                                 float* __restrict__ X) {
  const int64_t* b = blocks + 4 * blockIdx.x;
  const long off = b[0], ld = b[1];
  const int rows = (int)b[2], cols = (int)b[3];
  const long size = (long)rows * cols;
  const double th = theta[0];
  const double s = stats[4 * blockIdx.x], mu = stats[4 * blockIdx.x + 1], mn = stats[4 * blockIdx.x + 2],
               lsz = stats[4 * blockIdx.x + 3];
  const double sq = sqrt((double)n);
  const double fr = nrr[0] > 0.0 ? sq / sqrt(nrr[0]) : 0.0;
  const double ft = ntt[0] > 0.0 ? sq / sqrt(ntt[0]) : 0.0;
  for (long e = threadIdx.x; e < size; e += blockDim.x) {
    const long i = e / cols, j = e - i * cols;
    const long p = off + i * ld + j;
    const double ev = d[p] - th;
    double inv = ev == 0.0 ? 10.0 : s / ev;
    inv = fmin(fmax(inv, -10.0), 10.0);
    float* x = X + p * 8;
    x[0] = (float)(r[p] * fr);
    x[1] = (float)(ev / s);
    x[2] = (float)inv;
    x[3] = (float)(t[p] * ft);
    x[4] = (float)mu;
    x[5] = (float)mn;
    x[6] = (float)lsz;
    x[7] = kpos;
  }
}

__global__ void gather_rows_kernel(const float* __restrict__ X, int nf, const int64_t* __restrict__ idx, int m,
                                   float* __restrict__ out) {
  const long total = (long)m * nf;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long j = e / nf;
    const int f = (int)(e - j * nf);
    out[e] = X[idx[j] * nf + f];
  }
}

__global__ void triple_target_kernel(const double* __restrict__ psi_i, const double* __restrict__ psi_star,
                                     const double* __restrict__ cdev, const int64_t* __restrict__ idx, int m,
                                     float* __restrict__ out) {
  const double c = cdev[0];
  const double sg = c >= 0.0 ? 1.0 : -1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const long p = idx[j];
    out[j] = (float)(sg * psi_star[p] - fabs(c) * psi_i[p]);
  }
}

}  // namespace

void launch_mlp_layer1(const float* X, long n, int nin, const float* W1, const float* b1, int width, float* a1,
                       uint16_t* a1b, hipStream_t s) {
  if (n > 0) layer1_kernel<<<grid_of(n * width), kThreads, 0, s>>>(X, n, nin, W1, b1, width, a1, a1b);
}
void launch_mlp_layer3(float* z2, long n, int width, const float* b2, const float* W3, const float* b3, float* y,
                       bool store, hipStream_t s) {
  if (n > 0) layer3_kernel<<<(int)((n + 3) / 4), kThreads, 0, s>>>(z2, n, width, b2, W3, b3, y, store ? 1 : 0);
}
bool launch_mlp_infer_bf16(const float* X, long n, int nin, const float* W1, const float* b1, int width,
                           const uint16_t* W2b, const float* b2, const float* W3, const float* b3, float* y,
                           hipStream_t s) {
  if (width != kInfW || nin < 1 || nin > kInfMaxIn) return false;
  if (n <= 0) return true;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const long ntiles = (n + kInfRows - 1) / kInfRows;
  const int grid = (int)std::min<long>(ntiles, std::max(cus, 1));
  mlp_infer_bf16_kernel<<<grid, kInfThreads, 0, s>>>(X, n, nin, W1, b1, W2b, b2, W3, b3, y);
  return true;
}
void launch_seg_stats(const float* y, const float* t, int nseg, int seglen, double* stats, hipStream_t s) {
  if (nseg > 0) seg_stats_kernel<<<nseg, kThreads, 0, s>>>(y, t, seglen, stats);
}
void launch_cos_grad(const float* y, const float* t, const double* stats, int nseg, int seglen, float* dy,
                     hipStream_t s) {
  long n = (long)nseg * seglen;
  if (n > 0) cos_grad_kernel<<<grid_of(n), kThreads, 0, s>>>(y, t, stats, nseg, seglen, dy);
}
void launch_colsum_partial(const float* A, long rows, int cols, const float* w, int wstride, long chunk,
                           double* partial, hipStream_t s) {
  int nch = (int)((rows + chunk - 1) / chunk);
  if (nch > 0) colsum_partial_kernel<<<nch, kThreads, 0, s>>>(A, rows, cols, w, wstride, chunk, partial);
}
void launch_sum_partials(const double* partial, int nchunks, long cols, float* out, int ostride, hipStream_t s) {
  if (cols > 0) sum_partials_kernel<<<grid_of(cols), kThreads, 0, s>>>(partial, nchunks, cols, out, ostride);
}
void launch_sum_partials_f32(const float* partial, int nchunks, long cols, float* out, hipStream_t s) {
  if (cols > 0) sum_partials_f32_kernel<<<grid_of(cols), kThreads, 0, s>>>(partial, nchunks, cols, out);
}
void launch_mlp_back3(float* a2, const float* dy, const float* W3, long n, int width, hipStream_t s) {
  if (n > 0) back3_kernel<<<grid_of(n * width), kThreads, 0, s>>>(a2, dy, W3, n, width);
}
void launch_relu_mask(float* x, const float* mask, long n, hipStream_t s) {
  if (n > 0) relu_mask_kernel<<<grid_of(n), kThreads, 0, s>>>(x, mask, n);
}
void launch_adam(float* w, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s) {
  if (n > 0) adam_kernel<<<grid_of(n), kThreads, 0, s>>>(w, m, v, g, n, lr, b1, b2, eps, c1, c2);
}
void launch_f32_to_bf16_rne(const float* x, uint16_t* y, long n, hipStream_t s) {
  if (n > 0) f32_to_bf16_kernel<<<grid_of(n), kThreads, 0, s>>>(x, y, n);
}
void launch_feat_stats(const double* d, const double* theta, const int64_t* blocks, int nb, double* stats,
                       hipStream_t s) {
  if (nb > 0) feat_stats_kernel<<<nb, kThreads, 0, s>>>(d, theta, blocks, stats);
}
void launch_feat_fill(const double* r, const double* d, const double* theta, const double* t,
                      const int64_t* blocks, int nb, const double* stats, const double* nrr, const double* ntt,
                      long n, float kpos, float* X, hipStream_t s) {
  if (nb > 0) feat_fill_kernel<<<nb, kThreads, 0, s>>>(r, d, theta, t, blocks, stats, nrr, ntt, n, kpos, X);
}
void launch_gather_rows(const float* X, int nf, const int64_t* idx, int m, float* out, hipStream_t s) {
  if (m > 0) gather_rows_kernel<<<grid_of((long)m * nf), kThreads, 0, s>>>(X, nf, idx, m, out);
}
void launch_triple_target(const double* psi_i, const double* psi_star, const double* cdev, const int64_t* idx,
                          int m, float* out, hipStream_t s) {
  if (m > 0) triple_target_kernel<<<grid_of(m), kThreads, 0, s>>>(psi_i, psi_star, cdev, idx, m, out);
}

}  // namespace dmrg
