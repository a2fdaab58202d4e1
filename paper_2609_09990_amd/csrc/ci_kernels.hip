// Determinant-space kernels (device CI pipeline, Sec. III): the scatter of an
// MPS's prefix x suffix amplitudes into the CI matrix, the excited copies
// E_rs c of a CI vector, and the assembly of the one- and two-body (transition)
// density matrices from their products.  All three are bandwidth-bound element
// loops; the contraction between them runs on the fp64 MFMA block kernel.
#include "ci.hpp"

namespace dmrg {
namespace {

inline int grid_cap(long n, int cap = 4096) {
  long g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

__global__ void ci_scatter_kernel(const double* __restrict__ amp, const CiSector* __restrict__ secs,
                                  const int* __restrict__ pa, const int* __restrict__ pb,
                                  const double* __restrict__ ps, const int* __restrict__ sa,
                                  const int* __restrict__ sb, const double* __restrict__ ss,
                                  double* __restrict__ c, long nb) {
  const CiSector S = secs[blockIdx.y];
  const long n = (long)S.n_pre * S.n_suf;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long a = S.pre_off + i / S.n_suf, b = S.suf_off + i % S.n_suf;
    c[(long)(pa[a] + sa[b]) * nb + (pb[a] + sb[b])] = ps[a] * ss[b] * amp[S.amp_off + i];
  }
}

// blockIdx.y: row x of the copies, blockIdx.z: (source vector v, chunk g) as
// v nch + g; threads over the chunk.  Consecutive threads take consecutive beta
// strings of one alpha string, so the alpha-excitation reads are row gathers of
// c and the beta ones stay in a row.
__global__ void ci_excite_kernel(const double* __restrict__ c0, long cstride, long na, long nb, int n2,
                                 const int* __restrict__ ta, const int* __restrict__ tb, double* __restrict__ T,
                                 long vstride, long nch, long cl, long gstride, long d0, long dend) {
  const int x = blockIdx.y;
  const long v = blockIdx.z / nch, g = blockIdx.z - v * nch;
  const double* __restrict__ c = c0 + v * cstride;
  double* out = T + v * vstride + g * gstride + (long)x * cl;
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < cl; j += (long)gridDim.x * blockDim.x) {
    const long d = d0 + g * cl + j;
    if (d >= dend) break;
    const long ia = d / nb, ib = d - ia * nb;
    double v;
    if (x == n2) {
      v = c[d];
    } else {
      v = 0.0;
      const int xa = ta[(long)x * na + ia];
      if (xa != 0) v += (xa > 0 ? 1.0 : -1.0) * c[(long)(abs(xa) - 1) * nb + ib];
      const int xb = tb[(long)x * nb + ib];
      if (xb != 0) v += (xb > 0 ? 1.0 : -1.0) * c[ia * nb + (abs(xb) - 1)];
    }
    out[j] = v;
  }
}

__global__ void rdm_assemble_kernel(const double* __restrict__ G, int ldg, int n, double scale,
                                    double* __restrict__ gamma, double* __restrict__ Gam) {
  const long n2 = (long)n * n, n4 = n2 * n2;
  const double* id = G + n2 * ldg;  // the row of the unexcited bra
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 + n4; i += (long)gridDim.x * blockDim.x) {
    if (i < n2) {
      gamma[i] = scale * id[i];
      continue;
    }
    const long x = i - n2;
    const int s = (int)(x % n), r = (int)(x / n % n), q = (int)(x / n2 % n), p = (int)(x / (n2 * n));
    double v = G[(long)(q * n + p) * ldg + r * n + s];
    if (q == r) v -= id[p * n + s];
    Gam[x] = scale * v;
  }
}

// Offsets of the 9 blocks of a two-orbital density matrix in its 36 entries,
// block b = 3 k_alpha + k_beta (electrons of each spin on the pair), sizes
// 1, 2, 1 states for k = 0, 1, 2 of each spin.
__constant__ int kOrbOff[9] = {0, 1, 5, 6, 10, 26, 30, 31, 35};

// One workgroup: determinants of a grid-stride range for one pair.  A thread
// takes the environments (configurations of the other orbitals) whose
// representative determinant it holds (one electron of a spin on the pair sits
// on i), gathers the <= 4 amplitudes of that environment, and adds their outer
// product to its own LDS row; rows are summed in a fixed order at the end.
__global__ __launch_bounds__(256) void orb_pairs_kernel(const double* __restrict__ c, const uint32_t* __restrict__ sa,
                                                        const uint32_t* __restrict__ sb, const int* __restrict__ rank_a,
                                                        const int* __restrict__ rank_b, long nb, long ndet,
                                                        const int* __restrict__ pairs, double* __restrict__ partial) {
  __shared__ double acc[256][37];
  const int tid = threadIdx.x;
  const int i = pairs[2 * blockIdx.y], j = pairs[2 * blockIdx.y + 1];
  const uint32_t mi = 1u << i, mj = 1u << j;
  for (int e = 0; e < 36; ++e) acc[tid][e] = 0.0;
  for (long d = (long)blockIdx.x * 256 + tid; d < ndet; d += (long)gridDim.x * 256) {
    const long ia = d / nb, ib = d - ia * nb;
    const uint32_t a = sa[ia], b = sb[ib];
    const int ai = a >> i & 1, aj = a >> j & 1, bi = b >> i & 1, bj = b >> j & 1;
    const int ka = ai + aj, kb = bi + bj;
    if ((ka == 1 && !ai) || (kb == 1 && !bi)) continue;  // not the environment's representative
    const uint32_t ea = a & ~(mi | mj), eb = b & ~(mi | mj);
    uint32_t A[2], B[2];
    const int nA = ka == 1 ? 2 : 1, nB = kb == 1 ? 2 : 1;
    A[0] = ka == 0 ? 0u : (ka == 1 ? mi : (mi | mj));
    A[1] = mj;
    B[0] = kb == 0 ? 0u : (kb == 1 ? mi : (mi | mj));
    B[1] = mj;
    const int na_env = __popc(ea);
    double v[4];
    int q = 0;
    for (int pa = 0; pa < nA; ++pa)
      for (int pb = 0; pb < nB; ++pb) {
        const uint32_t a2 = ea | A[pa], b2 = eb | B[pb];
        const long idx = (long)rank_a[a2] * nb + rank_b[b2];
        // local creators moved in front of the environment's (alpha-first order)
        const int par = (int)(a2 >> i & 1) * __popc(ea & (mi - 1)) + (int)(a2 >> j & 1) * __popc(ea & (mj - 1)) +
                        (int)(b2 >> i & 1) * (na_env + __popc(eb & (mi - 1))) +
                        (int)(b2 >> j & 1) * (na_env + __popc(eb & (mj - 1)));
        v[q++] = (par & 1 ? -1.0 : 1.0) * c[idx];
      }
    const int off = kOrbOff[3 * ka + kb];
    for (int p = 0; p < q; ++p)
      for (int r = 0; r < q; ++r) acc[tid][off + p * q + r] += v[p] * v[r];
  }
  __syncthreads();
  if (tid < 36) {
    double s = 0.0;
    for (int t = 0; t < 256; ++t) s += acc[t][tid];
    partial[((long)blockIdx.y * gridDim.x + blockIdx.x) * 36 + tid] = s;
  }
}

__global__ void orb_sum_kernel(const double* __restrict__ partial, int npairs, int nblk, double* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= npairs * 36) return;
  const int p = x / 36, e = x % 36;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((long)p * nblk + b) * 36 + e];
  out[x] = s;
}

void launch_orb_pairs(const double* c, const uint32_t* sa, const uint32_t* sb, const int* rank_a, const int* rank_b,
                      long nb, long ndet, const int* pairs, int npairs, int nblk, double* partial, hipStream_t s) {
  if (npairs > 0) orb_pairs_kernel<<<dim3(nblk, npairs), 256, 0, s>>>(c, sa, sb, rank_a, rank_b, nb, ndet, pairs, partial);
}

void launch_orb_sum(const double* partial, int npairs, int nblk, double* out, hipStream_t s) {
  if (npairs > 0) orb_sum_kernel<<<(npairs * 36 + 255) / 256, 256, 0, s>>>(partial, npairs, nblk, out);
}

void launch_ci_scatter(const double* amp, const CiSector* secs, int n_secs, const int* pa, const int* pb,
                       const double* ps, const int* sa, const int* sb, const double* ss, double* c, long nb,
                       hipStream_t s) {
  if (n_secs <= 0) return;
  ci_scatter_kernel<<<dim3(256, n_secs), 256, 0, s>>>(amp, secs, pa, pb, ps, sa, sb, ss, c, nb);
}

void launch_ci_excite(const double* c, long na, long nb, int n2, const int* ta, const int* tb, double* T, long cl,
                      long d0, long dend, hipStream_t s, long gstride, int nvec, long cstride, long vstride) {
  const long nch = (dend - d0 + cl - 1) / cl;
  if (nch <= 0 || nvec <= 0) return;
  if (gstride <= 0) gstride = (long)(n2 + 1) * cl;
  ci_excite_kernel<<<dim3(grid_cap(cl, 64), n2 + 1, (unsigned)(nch * nvec)), 256, 0, s>>>(
      c, cstride, na, nb, n2, ta, tb, T, vstride, nch, cl, gstride, d0, dend);
}

// out[d] = scale * sum_{x < n2} (E_x U_x)[d], U_x the rows of U (row-major, ldu).
__global__ void ci_apply_sum_kernel(const double* __restrict__ U, long ldu, long na, long nb, int n2,
                                    const int* __restrict__ ta, const int* __restrict__ tb, double scale,
                                    double* __restrict__ out, long ndet) {
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < ndet; d += (long)gridDim.x * blockDim.x) {
    const long ia = d / nb, ib = d - ia * nb;
    double v = 0.0;
    for (int x = 0; x < n2; ++x) {
      const double* u = U + (long)x * ldu;
      const int xa = ta[(long)x * na + ia];
      if (xa != 0) v += (xa > 0 ? 1.0 : -1.0) * u[(long)(abs(xa) - 1) * nb + ib];
      const int xb = tb[(long)x * nb + ib];
      if (xb != 0) v += (xb > 0 ? 1.0 : -1.0) * u[ia * nb + (abs(xb) - 1)];
    }
    out[d] = scale * v;
  }
}

void launch_ci_apply_sum(const double* U, long ldu, long na, long nb, int n2, const int* ta, const int* tb,
                         double scale, double* out, long ndet, hipStream_t s) {
  if (ndet > 0) ci_apply_sum_kernel<<<grid_cap(ndet), 256, 0, s>>>(U, ldu, na, nb, n2, ta, tb, scale, out, ndet);
}

// Gamma3[((((p n + q) n + r) n + s) n + t) n + u] = scale G[(q n + p) ldg + (t n + u) rows + r n + s]
__global__ void rdm3_assemble_kernel(const double* __restrict__ G, long ldg, int n, int rows, double scale,
                                     double* __restrict__ out) {
  const long n2 = (long)n * n, n6 = n2 * n2 * n2;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long)gridDim.x * blockDim.x) {
    const int u = (int)(i % n), t = (int)(i / n % n), s = (int)(i / n2 % n), r = (int)(i / (n2 * n) % n);
    const int q = (int)(i / (n2 * n2) % n), p = (int)(i / (n2 * n2 * n));
    out[i] = scale * G[(long)(q * n + p) * ldg + (long)(t * n + u) * rows + r * n + s];
  }
}

void launch_rdm3_assemble(const double* G, long ldg, int n, int rows, double scale, double* out, hipStream_t s) {
  const long n2 = (long)n * n;
  rdm3_assemble_kernel<<<grid_cap(n2 * n2 * n2), 256, 0, s>>>(G, ldg, n, rows, scale, out);
}

void launch_rdm_assemble(const double* G, int ldg, int n, double scale, double* gamma, double* Gamma,
                         hipStream_t s) {
  const long n2 = (long)n * n;
  rdm_assemble_kernel<<<grid_cap(n2 + n2 * n2), 256, 0, s>>>(G, ldg, n, scale, gamma, Gamma);
}

}  // namespace dmrg
