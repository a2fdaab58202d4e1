// Determinant-space (CI) view of a state and its reduced density matrices: the
// device CI pipeline of the paper's Sec. III (colexicographic string ranks,
// determinant-string enumeration, one- and two-body density matrices formed on
// the device), used here for the 1-/2-RDMs and transition RDMs of MPS states.
//
// Conventions (shared with the integrals of Sec. II.A):
// * E_pq = sum_sigma a+_{p sigma} a_{q sigma}; a determinant is
//   (prod_{p in I_a} a+_{p alpha})(prod_{p in I_b} a+_{p beta})|0>, creators in
//   ascending orbital order, all alpha before all beta;
// * strings are ranked colexicographically, rank = sum_t C(o_t, t + 1) over the
//   sorted occupied orbitals o_0 < o_1 < ...;
// * a CI vector is the row-major matrix c[I_a][I_b] (N_a x N_b).
// The MPS site basis orders spin orbitals 0a, 0b, 1a, 1b, ... (s = n_a + 2 n_b),
// so a site-product amplitude enters c with the sign of moving every alpha
// creator in front of the beta creators of lower orbitals:
// (-1)^{sum over alpha-occupied p of the number of beta electrons below p}.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmrg {

// One middle-cut sector of the MPS-to-CI scatter: its prefix x suffix
// amplitude matrix (row-major, n_pre x n_suf, at amp_off) and its rows of the
// prefix / suffix rank and sign tables.
struct CiSector {
  long amp_off;
  long pre_off, suf_off;
  int n_pre, n_suf;
};

// c[(pa + sa) * nb + (pb + sb)] = ps * ss * amp, over every sector's pairs.
void launch_ci_scatter(const double* amp, const CiSector* secs, int n_secs, const int* pa, const int* pb,
                       const double* ps, const int* sa, const int* sb, const double* ss, double* c, long nb,
                       hipStream_t s);

// Excited copies of a CI vector for determinants [d0, dend), in chunks of cl:
// T[(g * rows + x) * cl + j] = (E_rs c)[d] for x = r n + s < n2 and c[d] for
// x = n2 (rows = n2 + 1), d = d0 + g cl + j.  ta[x * na + J] (tb likewise) is
// +-(I + 1) when E_rs |I> = +-|J> within one spin's strings, 0 when no I.
// gstride: elements between consecutive chunks (<= 0: (n2 + 1) cl).  nvec source
// vectors c + v cstride in one launch, written from T + v vstride.
void launch_ci_excite(const double* c, long na, long nb, int n2, const int* ta, const int* tb, double* T, long cl,
                      long d0, long dend, hipStream_t s, long gstride = 0, int nvec = 1, long cstride = 0,
                      long vstride = 0);
// out[d] = scale * sum_{x < n2} (E_x U_x)[d] over the rows U_x = U + x ldu.
void launch_ci_apply_sum(const double* U, long ldu, long na, long nb, int n2, const int* ta, const int* tb,
                         double scale, double* out, long ndet, hipStream_t s);
// Gamma3[p q r s t u] = scale G[(q n + p) ldg + (t n + u) rows + r n + s].
void launch_rdm3_assemble(const double* G, long ldg, int n, int rows, double scale, double* out, hipStream_t s);

// gamma[pq] = scale G[n2][pq]; Gamma[pqrs] = scale (G[qp][rs] - d_qr G[n2][ps])
// with G the (n2 + 1) x (n2 + 1) product of the excited copies (row-major, ldg).
void launch_rdm_assemble(const double* G, int ldg, int n, double scale, double* gamma, double* Gamma,
                         hipStream_t s);

// Two-orbital density matrices of a CI vector (unnormalised), for every pair
// (pairs[2 p], pairs[2 p + 1]), i < j: with the pair's spin orbitals moved to the
// front in the order (i alpha, j alpha, i beta, j beta), rho = sum over the
// configurations of the other orbitals of v v^T.  Only the 36 entries of the 9
// blocks of equal pair (N_alpha, N_beta) can be non-zero; partial[(p * nblk + b)
// * 36 + e] receives workgroup b's sums (nblk = grid size per pair), and
// launch_orb_sum adds them in order into out[p * 36 + e].  sa / sb: the strings
// by rank; rank_a / rank_b: the rank of every n-bit mask (-1 if not a string).
void launch_orb_pairs(const double* c, const uint32_t* sa, const uint32_t* sb, const int* rank_a, const int* rank_b,
                      long nb, long ndet, const int* pairs, int npairs, int nblk, double* partial, hipStream_t s);
void launch_orb_sum(const double* partial, int npairs, int nblk, double* out, hipStream_t s);

}  // namespace dmrg
