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

// blockIdx.y: row x of the copies, blockIdx.z: chunk g; threads over the chunk.
// Consecutive threads take consecutive beta strings of one alpha string, so the
// alpha-excitation reads are row gathers of c and the beta ones stay in a row.
__global__ void ci_excite_kernel(const double* __restrict__ c, long na, long nb, int n2,
                                 const int* __restrict__ ta, const int* __restrict__ tb, double* __restrict__ T,
                                 long cl, long d0, long dend) {
  const int x = blockIdx.y;
  const long g = blockIdx.z;
  const long rows = n2 + 1;
  double* out = T + (g * rows + x) * cl;
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

void launch_ci_scatter(const double* amp, const CiSector* secs, int n_secs, const int* pa, const int* pb,
                       const double* ps, const int* sa, const int* sb, const double* ss, double* c, long nb,
                       hipStream_t s) {
  if (n_secs <= 0) return;
  ci_scatter_kernel<<<dim3(256, n_secs), 256, 0, s>>>(amp, secs, pa, pb, ps, sa, sb, ss, c, nb);
}

void launch_ci_excite(const double* c, long na, long nb, int n2, const int* ta, const int* tb, double* T, long cl,
                      long d0, long dend, hipStream_t s) {
  const long nch = (dend - d0 + cl - 1) / cl;
  if (nch <= 0) return;
  ci_excite_kernel<<<dim3(grid_cap(cl, 64), n2 + 1, (unsigned)nch), 256, 0, s>>>(c, na, nb, n2, ta, tb, T, cl, d0,
                                                                                 dend);
}

void launch_rdm_assemble(const double* G, int ldg, int n, double scale, double* gamma, double* Gamma,
                         hipStream_t s) {
  const long n2 = (long)n * n;
  rdm_assemble_kernel<<<grid_cap(n2 + n2 * n2), 256, 0, s>>>(G, ldg, n, scale, gamma, Gamma);
}

}  // namespace dmrg
