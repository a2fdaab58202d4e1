// Determinant-space view of MPS states and their (transition) 1-/2-RDMs (the
// device CI pipeline of Sec. III; conventions in ci.hpp).
//
// MPS -> CI.  The chain is cut at c = L/2.  Left of the cut every prefix of
// physical states (s_0 .. s_{c-1}) that reaches a sector q of bond c carries the
// row vector A_0[s_0] ... A_{c-1}[s_{c-1}]; right of it every suffix carries
// A_c[s_c] ... A_{L-1}[s_{L-1}].  Both families grow one site at a time as block
// GEMMs (all prefixes of one sector times one site block), and the amplitudes
// of sector q are the product P_q S_q^T of its prefix and suffix matrices, one
// GEMM per sector.  A determinant's string ranks split into a prefix part and a
// suffix part (the suffix's ranks counted after the prefix's electrons, fixed by
// q), and so does its sign, so a scatter kernel places every amplitude.
//
// RDMs.  With the excited copies T_x = E_rs |c> (x = r n + s) and T_{n^2} = |c>,
//   <bra| E_pq |ket> = <bra | T^ket_{pq}>,
//   <bra| E_pq E_rs |ket> = <E_qp bra | E_rs ket> = <T^bra_{qp} | T^ket_{rs}>,
// so one product G = T^bra (T^ket)^T of (n^2 + 1) rows over all determinants
// gives gamma, Gamma' = <E_pq E_rs> - d_qr gamma_ps and <bra|ket>.  The
// determinants are taken in passes whose copies fit a fixed budget; G is a
// split-K sum on the fp64 MFMA block kernel, partial tiles reduced in a fixed
// order (deterministic), passes added in order.
#include <algorithm>
#include <cmath>

#include "ci.hpp"
#include "solver.hpp"

namespace dmrg {
namespace {

long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

int popc(uint32_t x) { return __builtin_popcount(x); }

// Colexicographic rank contribution of the occupied orbitals of `bits`, the
// first of them being electron number t0 of its spin.
long colex_part(uint32_t bits, int t0) {
  long r = 0;
  int t = t0;
  for (int o = 0; o < 32; ++o)
    if (bits >> o & 1u) r += binom(o, ++t);
  return r;
}

std::vector<uint32_t> colex_strings(int n, int k) {
  std::vector<uint32_t> out(binom(n, k));
  for (uint32_t m = 0; m < (1u << n); ++m)
    if (popc(m) == k) out[colex_part(m, 0)] = m;
  return out;
}

// tab[x * N + J] = +-(I + 1) when E_rs |I> = +-|J> (x = r n + s), else 0:
// a_s removes s from I with (-1)^(electrons below s), a+_r inserts r into what
// is left with (-1)^(electrons below r).
std::vector<int> excitation_table(int n, const std::vector<uint32_t>& strs) {
  const long N = (long)strs.size();
  std::vector<int> t((long)n * n * N, 0);
  for (long J = 0; J < N; ++J) {
    const uint32_t j = strs[J];
    for (int r = 0; r < n; ++r) {
      if (!(j >> r & 1u)) continue;
      for (int s = 0; s < n; ++s) {
        if (s != r && (j >> s & 1u)) continue;
        const uint32_t i = (j & ~(1u << r)) | (1u << s);
        const uint32_t i1 = i & ~(1u << s);
        const int par = popc(i & ((1u << s) - 1)) + popc(i1 & ((1u << r) - 1));
        const int I = (int)colex_part(i, 0) + 1;
        t[((long)r * n + s) * N + J] = (par & 1) ? -I : I;
      }
    }
  }
  return t;
}

void tiles64(std::vector<GemmUnit>& units, double* C, int ldc, int M, int N, int ib, int ie) {
  for (int m0 = 0; m0 < M; m0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) units.push_back({C, ldc, M, N, m0, n0, ib, ie, 0});
}

// one generic-kernel GEMM launch over 64 x 64 tiles (items and units uploaded here)
void gemm_tiles(int mode, const std::vector<GemmItem>& items, const std::vector<GemmUnit>& units, hipStream_t st);

template <class T>
void upload(DevMem& d, const std::vector<T>& v, hipStream_t st) {
  d.reserve(std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) hip_check(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "ci upload");
}

// rank of every n-bit mask among the strings with k bits, -1 for the others
std::vector<int> rank_table(int n, int k) {
  std::vector<int> r((size_t)1 << n, -1);
  for (uint32_t m = 0; m < (1u << n); ++m)
    if (popc(m) == k) r[m] = (int)colex_part(m, 0);
  return r;
}

// Eigenvalues (ascending) and, if V, eigenvectors (columns of the row-major
// n x n V) of a symmetric matrix by cyclic Jacobi rotations (small n only).
void jacobi_eigh(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>* V) {
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double th = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = cs * qkp - sn * qkq;
          Q[(size_t)k * n + q] = sn * qkp + cs * qkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)idx[i] * n + idx[i]];
  if (V) {
    V->assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) (*V)[(size_t)k * n + i] = Q[(size_t)k * n + idx[i]];
  }
}

double entropy_of(const std::vector<double>& rho, int n) {
  std::vector<double> w;
  jacobi_eigh(rho, n, w, nullptr);
  double s = 0;
  for (double x : w)
    if (x > 1e-300) s -= x * std::log(x);
  return s;
}

void gemm_tiles(int mode, const std::vector<GemmItem>& items, const std::vector<GemmUnit>& units, hipStream_t st) {
  if (units.empty()) return;
  DevMem di, du;
  upload(di, items, st);
  upload(du, units, st);
  launch_gemm(PREC_F64, mode, du.as<GemmUnit>(), (int)units.size(), di.as<GemmItem>(), st);
  hip_check(hipStreamSynchronize(st), "ci gemm");
}

// Split-K product G (M x N, row-major, ldg = N) [+]= sum over chunks g of
// A_g (M x K_g) B_g^T (N x K_g) on the fp64 MFMA block kernel: A_g = A + g
// astride, B_g = B + g bstride, both with leading dimension cl; about 2048
// workgroups, partial tiles reduced in a fixed order; acc adds to G.
void splitk_nt(const double* A, long astride, const double* B, long bstride, long cl, int M, int N,
               const std::vector<int>& K, double* G, bool acc, hipStream_t st) {
  struct Tile {
    int m0, n0, tm, tn;
  };
  std::vector<Tile> tl;
  for (int m0 = 0; m0 < M; m0 += 96)
    for (int n0 = 0; n0 < N; n0 += 64)
      tl.push_back({m0, n0, std::min(96, (M - m0 + 15) / 16 * 16), std::min(64, (N - n0 + 15) / 16 * 16)});
  const long nt = (long)tl.size(), nch = (long)K.size();
  std::vector<GemmItem> items;
  for (long g = 0; g < nch; ++g) {
    DMRG_REQUIRE(buffer_reach_ok(GEMM_NT, M, N, K[g], (int)cl, (int)cl, 8, 8), ST_EINVAL,
                 "determinant chunk beyond the block kernel reach");
    items.push_back({A + g * astride, B + g * bstride, (int)cl, (int)cl, K[g], 0, 1.0});
  }
  const long ng = std::max<long>(1, std::min<long>(nch, 2048 / std::max<long>(nt, 1)));
  std::vector<SplitTile> tiles;
  std::vector<GemmUnit> units;
  long so = 0;
  for (const Tile& t : tl) {
    tiles.push_back({G, so, N, M, N, t.m0, t.n0, (int)ng, t.tm, t.tn, acc ? 1 : 0, 0});
    so += ng * t.tm * t.tn;
  }
  DevMem slots, ditems, dunits, dtiles;
  slots.reserve((size_t)so * 8);
  for (long gi = 0; gi < ng; ++gi) {
    const int ib = (int)(nch * gi / ng), ie = (int)(nch * (gi + 1) / ng);
    for (long t = 0; t < nt; ++t) {
      const SplitTile& s = tiles[t];
      units.push_back({slots.as<double>() + s.s0 + gi * s.tm * s.tn, s.tn, M, N, s.m0, s.n0, ib, ie, 2,
                       8 * (s.tm / 16) + s.tn / 16});
    }
  }
  upload(ditems, items, st);
  upload(dunits, units, st);
  upload(dtiles, tiles, st);
  launch_gemm_wg(PREC_F64, 5, dunits.as<GemmUnit>(), (int)units.size(), ditems.as<GemmItem>(), st);
  launch_splitk_reduce(dtiles.as<SplitTile>(), (int)nt, slots.as<double>(), st);
  hip_check(hipStreamSynchronize(st), "split-K product");
}

}  // namespace

long ci_dimension(int n, int na, int nb) { return binom(n, na) * binom(n, nb); }

// V c with V = 1/2 sum_pqrs (pq|rs) E_pq E_rs and (pq|rs) = sum_Q B^Q_pq B^Q_rs,
// streamed through the factors: T_rs = E_rs c, W_Q = sum_rs B^Q_rs T_rs,
// U_pq = sum_Q B^Q_pq W_Q, V c = 1/2 sum_pq E_pq U_pq (two GEMMs and two
// gather kernels; (pq|rs) is never formed).
void ci_apply_v(int n, int na, int nb, int nq, const double* Bh, hipStream_t st, const double* c, double* out) {
  DMRG_REQUIRE(n >= 1 && n <= 16 && nq >= 0, ST_EINVAL, "the two-electron operator on CI vectors needs 1..16 orbitals");
  const std::vector<uint32_t> sa = colex_strings(n, na), sb = colex_strings(n, nb);
  const long NA = (long)sa.size(), NB = (long)sb.size(), N = NA * NB;
  const int n2 = n * n;
  if (nq == 0) {
    launch_fill(out, N, 0.0, st);
    hip_check(hipStreamSynchronize(st), "apply V");
    return;
  }
  DevMem ta, tb, T, W, U, Bd;
  upload(ta, excitation_table(n, sa), st);
  upload(tb, excitation_table(n, sb), st);
  T.reserve((size_t)(n2 + 1) * N * 8);
  W.reserve((size_t)nq * N * 8);
  U.reserve((size_t)n2 * N * 8);
  Bd.reserve((size_t)nq * n2 * 8);
  hip_check(hipMemcpyAsync(Bd.p, Bh, (size_t)nq * n2 * 8, hipMemcpyHostToDevice, st), "B");
  launch_ci_excite(c, NA, NB, n2, ta.as<int>(), tb.as<int>(), T.as<double>(), N, 0, N, st);
  std::vector<GemmItem> items{{Bd.as<double>(), T.as<double>(), n2, (int)N, n2, 0, 1.0}};
  std::vector<GemmUnit> units;
  tiles64(units, W.as<double>(), (int)N, nq, (int)N, 0, 1);
  gemm_tiles(GEMM_NN, items, units, st);  // W = B T (nq x N)
  items = {{Bd.as<double>(), W.as<double>(), n2, (int)N, nq, 0, 1.0}};
  units.clear();
  tiles64(units, U.as<double>(), (int)N, n2, (int)N, 0, 1);
  gemm_tiles(GEMM_TN, items, units, st);  // U = B^T W (n^2 x N)
  launch_ci_apply_sum(U.as<double>(), N, NA, NB, n2, ta.as<int>(), tb.as<int>(), 0.5, out, N, st);
  hip_check(hipStreamSynchronize(st), "apply V");
}

// Gamma3[pqrstu] = scale <bra|E_pq E_rs E_tu|ket> = scale <E_qp bra | E_rs E_tu ket>:
// the copies E_tu ket are kept whole, E_rs of each is formed per pass of
// determinants, and one split-K product of (n^2 + 1) bra rows with n^2 (n^2 + 1)
// ket rows per pass accumulates G.
void ci_rdm3(int n, int na, int nb, hipStream_t st, const double* bra, const double* ket, double scale, double* out) {
  DMRG_REQUIRE(n >= 1 && n <= 12, ST_EINVAL, "the three-body density from CI vectors needs 1..12 orbitals");
  const std::vector<uint32_t> sa = colex_strings(n, na), sb = colex_strings(n, nb);
  const long NA = (long)sa.size(), NB = (long)sb.size(), N = NA * NB;
  const int n2 = n * n, rows = n2 + 1, nbr = n2 * rows;
  constexpr long CL = 4096;
  DevMem ta, tb, Tk, T1, T2, G, d3;
  upload(ta, excitation_table(n, sa), st);
  upload(tb, excitation_table(n, sb), st);
  Tk.reserve((size_t)rows * N * 8);
  launch_ci_excite(ket, NA, NB, n2, ta.as<int>(), tb.as<int>(), Tk.as<double>(), N, 0, N, st);  // [x][N]
  const long per_pass = std::max<long>(1, (4L << 30) / ((long)nbr * CL * 8)) * CL;
  const long pass = std::min(per_pass, (N + CL - 1) / CL * CL);
  T1.reserve((size_t)rows * pass * 8);
  T2.reserve((size_t)nbr * pass * 8);
  G.reserve((size_t)rows * nbr * 8);
  for (long d0 = 0; d0 < N; d0 += pass) {
    const long dend = std::min(N, d0 + pass), nch = (dend - d0 + CL - 1) / CL;
    launch_ci_excite(bra, NA, NB, n2, ta.as<int>(), tb.as<int>(), T1.as<double>(), CL, d0, dend, st);
    // chunk g of E_rs (E_x ket) at T2 + g nbr CL + x rows CL, every x in one launch
    launch_ci_excite(Tk.as<double>(), NA, NB, n2, ta.as<int>(), tb.as<int>(), T2.as<double>(), CL, d0, dend, st,
                     (long)nbr * CL, n2, N, (long)rows * CL);
    std::vector<int> K;
    for (long g = 0; g < nch; ++g) K.push_back((int)std::min(CL, dend - d0 - g * CL));
    splitk_nt(T1.as<double>(), rows * CL, T2.as<double>(), (long)nbr * CL, CL, rows, nbr, K, G.as<double>(), d0 > 0,
              st);
  }
  const long n6 = (long)n2 * n2 * n2;
  d3.reserve((size_t)n6 * 8);
  launch_rdm3_assemble(G.as<double>(), nbr, n, rows, scale, d3.as<double>(), st);
  hip_check(hipMemcpyAsync(out, d3.p, (size_t)n6 * 8, hipMemcpyDeviceToHost, st), "rdm3 out");
  hip_check(hipStreamSynchronize(st), "rdm3");
}

void orbital_rdm2(int n, int na, int nb, hipStream_t st, const double* c, std::vector<double>& rho) {
  DMRG_REQUIRE(n >= 2 && n <= 16, ST_EINVAL, "orbital density matrices from CI vectors need 2..16 orbitals");
  const std::vector<uint32_t> sa = colex_strings(n, na), sb = colex_strings(n, nb);
  const long NB = (long)sb.size(), N = (long)sa.size() * NB;
  std::vector<int> pairs;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      pairs.push_back(i);
      pairs.push_back(j);
    }
  const int np = (int)pairs.size() / 2;
  const int nblk = (int)std::max<long>(1, std::min<long>((N + 255) / 256, (2048 + np - 1) / np));
  DevMem dsa, dsb, dra, drb, dpairs, part, out;
  upload(dsa, sa, st);
  upload(dsb, sb, st);
  upload(dra, rank_table(n, na), st);
  upload(drb, rank_table(n, nb), st);
  upload(dpairs, pairs, st);
  part.reserve((size_t)np * nblk * 36 * 8);
  out.reserve((size_t)np * 36 * 8);
  launch_orb_pairs(c, dsa.as<uint32_t>(), dsb.as<uint32_t>(), dra.as<int>(), drb.as<int>(), NB, N, dpairs.as<int>(), np,
                   nblk, part.as<double>(), st);
  launch_orb_sum(part.as<double>(), np, nblk, out.as<double>(), st);
  std::vector<double> e((size_t)np * 36);
  hip_check(hipMemcpyAsync(e.data(), out.p, e.size() * 8, hipMemcpyDeviceToHost, st), "orbital rdm");
  hip_check(hipStreamSynchronize(st), "orbital rdm");
  // expand the 36 entries of each pair: block (k_alpha, k_beta), states
  // (alpha configuration, beta configuration) in the kernel's order
  rho.assign((size_t)np * 256, 0.0);
  static const int kOff[9] = {0, 1, 5, 6, 10, 26, 30, 31, 35};
  for (int p = 0; p < np; ++p) {
    double* R = rho.data() + (size_t)p * 256;
    double tr = 0;
    for (int ka = 0; ka < 3; ++ka)
      for (int kb = 0; kb < 3; ++kb) {
        const int nA = ka == 1 ? 2 : 1, nB = kb == 1 ? 2 : 1, q = nA * nB;
        int L[4];
        for (int pa = 0; pa < nA; ++pa)
          for (int pb = 0; pb < nB; ++pb) {
            const int ai = ka == 2 || (ka == 1 && pa == 0), aj = ka == 2 || (ka == 1 && pa == 1);
            const int bi = kb == 2 || (kb == 1 && pb == 0), bj = kb == 2 || (kb == 1 && pb == 1);
            L[pa * nB + pb] = (ai + 2 * bi) + 4 * (aj + 2 * bj);
          }
        for (int x = 0; x < q; ++x)
          for (int y = 0; y < q; ++y) R[L[x] * 16 + L[y]] = e[(size_t)p * 36 + kOff[3 * ka + kb] + x * q + y];
        for (int x = 0; x < q; ++x) tr += R[L[x] * 16 + L[x]];
      }
    DMRG_REQUIRE(tr > 0, ST_EINVAL, "zero CI vector");
    for (int x = 0; x < 256; ++x) R[x] /= tr;
  }
}

void mutual_information(int n, int na, int nb, hipStream_t st, const double* c, double* s1, double* I) {
  std::vector<double> rho;
  orbital_rdm2(n, na, nb, st, c, rho);
  mutual_information_of(n, rho, s1, I);
}

void mutual_information_of(int n, const std::vector<double>& rho, double* s1, double* I) {
  std::vector<double> s2((size_t)n * n, 0.0);
  std::vector<double> one(n, -1.0);
  int p = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j, ++p) {
      const std::vector<double> R(rho.begin() + (size_t)p * 256, rho.begin() + (size_t)(p + 1) * 256);
      s2[(size_t)i * n + j] = entropy_of(R, 16);
      if (one[i] < 0 || one[j] < 0) {  // one-orbital matrices: diagonal partial traces
        double di[4] = {0, 0, 0, 0}, dj[4] = {0, 0, 0, 0};
        for (int L = 0; L < 16; ++L) {
          di[L % 4] += R[L * 16 + L];
          dj[L / 4] += R[L * 16 + L];
        }
        auto h = [](const double* d) {
          double s = 0;
          for (int t = 0; t < 4; ++t)
            if (d[t] > 1e-300) s -= d[t] * std::log(d[t]);
          return s;
        };
        if (one[i] < 0) one[i] = h(di);
        if (one[j] < 0) one[j] = h(dj);
      }
    }
  for (int i = 0; i < n; ++i) {
    s1[i] = one[i];
    I[(size_t)i * n + i] = 0;
    for (int j = i + 1; j < n; ++j)
      I[(size_t)i * n + j] = I[(size_t)j * n + i] = 0.5 * (one[i] + one[j] - s2[(size_t)i * n + j]);
  }
}

void fiedler_order(int n, const double* I, int* order, double* fiedler) {
  DMRG_REQUIRE(n >= 2 && n <= 64, ST_EINVAL, "ordering needs 2..64 orbitals");
  std::vector<double> Lap((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double d = 0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        Lap[(size_t)i * n + j] = -I[(size_t)i * n + j];
        d += I[(size_t)i * n + j];
      }
    Lap[(size_t)i * n + i] = d;
  }
  std::vector<double> w, V;
  jacobi_eigh(Lap, n, w, &V);
  std::vector<double> v(n);
  int big = 0;
  for (int i = 0; i < n; ++i) {
    v[i] = V[(size_t)i * n + 1];
    if (std::fabs(v[i]) > std::fabs(v[big])) big = i;
  }
  if (v[big] < 0)
    for (double& x : v) x = -x;
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return v[a] < v[b]; });
  for (int i = 0; i < n; ++i) {
    order[i] = idx[i];
    if (fiedler) fiedler[i] = v[i];
  }
}

void Solver::mps_to_ci(int state, double* c) {
  DMRG_REQUIRE(state >= 0 && state <= (int)defl_.size(), ST_EINVAL, "state must be 0 (this MPS) or a held state");
  const std::vector<Bond>& B = state == 0 ? bonds_ : defl_[state - 1].bonds;
  const std::vector<SiteTensor>& S = state == 0 ? mps_ : defl_[state - 1].sites;
  const int L = prob_->n;
  DMRG_REQUIRE((int)S.size() == L && (int)B.size() == L + 1, ST_ESTATE, "no MPS");
  DMRG_REQUIRE(L <= 24, ST_EINVAL, "the CI vector is built for at most 24 orbitals");
  const long Nb = binom(L, prob_->n_beta);
  DMRG_REQUIRE(ci_dimension(L, prob_->n_alpha, prob_->n_beta) < (1L << 31), ST_EINVAL, "CI space too large");
  DMRG_REQUIRE(B[0].sec.size() == 1 && B[0].sec[0].dim == 1 && B[L].sec.size() == 1 && B[L].sec[0].dim == 1,
               ST_ESTATE, "boundary bonds must hold one state");
  const int cut = L / 2;
  struct Str {
    uint32_t a, b;
  };
  struct Part {
    int src, dst;
    long r0;
    const double* blk;
    int ldb;
  };
  const double one = 1.0;
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  // prefixes: sites 0 .. cut-1, one matrix (prefixes x sector dim) per sector
  std::vector<std::vector<Str>> pre(1, std::vector<Str>{{0u, 0u}});
  std::vector<long> poff(1, 0);
  DevMem P, Pn;
  P.reserve(8);
  hip_check(hipMemcpyAsync(P.p, &one, 8, hipMemcpyHostToDevice, st), "ci");
  for (int k = 0; k < cut; ++k) {
    const Bond& bl = B[k];
    const Bond& br = B[k + 1];
    const SiteTensor& A = S[k];
    std::vector<std::vector<Str>> npre(br.sec.size());
    std::vector<Part> parts;
    for (size_t i = 0; i < bl.sec.size(); ++i) {
      if (pre[i].empty() || A.lay.slab_of_left[i] < 0) continue;
      const Slab& sb = A.lay.slabs[A.lay.slab_of_left[i]];
      for (int s = 0; s < 4; ++s) {
        const int j = br.find(bl.sec[i].q + site_qn(s));
        const int bi = j < 0 ? -1 : sb.block_of(s, j);
        if (bi < 0) continue;
        parts.push_back({(int)i, j, (long)npre[j].size(), A.buf.as<double>() + sb.off + sb.blocks[bi].col0, sb.width});
        for (const Str& p : pre[i]) npre[j].push_back({p.a | (uint32_t)(s & 1) << k, p.b | (uint32_t)(s >> 1) << k});
      }
    }
    std::vector<long> noff(br.sec.size(), 0);
    long tot = 0;
    for (size_t j = 0; j < br.sec.size(); ++j) {
      noff[j] = tot;
      tot += (long)npre[j].size() * br.sec[j].dim;
    }
    Pn.reserve(std::max<long>(tot, 1) * 8);
    items.clear();
    units.clear();
    for (const Part& pt : parts) {
      const int di = bl.sec[pt.src].dim, dj = br.sec[pt.dst].dim;
      const int ib = (int)items.size();
      items.push_back({P.as<double>() + poff[pt.src], pt.blk, di, pt.ldb, di, 0, 1.0});
      tiles64(units, Pn.as<double>() + noff[pt.dst] + pt.r0 * dj, dj, (int)pre[pt.src].size(), dj, ib, ib + 1);
    }
    gemm_once(GEMM_NN, items, units);
    std::swap(P, Pn);
    pre.swap(npre);
    poff.swap(noff);
  }
  // suffixes: sites cut .. L-1, one matrix (suffixes x sector dim) per sector
  std::vector<std::vector<Str>> suf(1, std::vector<Str>{{0u, 0u}});
  std::vector<long> soff(1, 0);
  DevMem Sm, Sn;
  Sm.reserve(8);
  hip_check(hipMemcpyAsync(Sm.p, &one, 8, hipMemcpyHostToDevice, st), "ci");
  for (int k = L - 1; k >= cut; --k) {
    const Bond& bl = B[k];
    const Bond& br = B[k + 1];
    const SiteTensor& A = S[k];
    std::vector<std::vector<Str>> nsuf(bl.sec.size());
    std::vector<Part> parts;
    for (size_t j = 0; j < br.sec.size(); ++j) {
      if (suf[j].empty()) continue;
      for (int s = 0; s < 4; ++s) {
        const int i = bl.find(br.sec[j].q - site_qn(s));
        if (i < 0 || A.lay.slab_of_left[i] < 0) continue;
        const Slab& sb = A.lay.slabs[A.lay.slab_of_left[i]];
        const int bi = sb.block_of(s, (int)j);
        if (bi < 0) continue;
        parts.push_back({(int)j, i, (long)nsuf[i].size(), A.buf.as<double>() + sb.off + sb.blocks[bi].col0, sb.width});
        for (const Str& x : suf[j]) nsuf[i].push_back({x.a | (uint32_t)(s & 1) << k, x.b | (uint32_t)(s >> 1) << k});
      }
    }
    std::vector<long> noff(bl.sec.size(), 0);
    long tot = 0;
    for (size_t i = 0; i < bl.sec.size(); ++i) {
      noff[i] = tot;
      tot += (long)nsuf[i].size() * bl.sec[i].dim;
    }
    Sn.reserve(std::max<long>(tot, 1) * 8);
    items.clear();
    units.clear();
    for (const Part& pt : parts) {
      const int dj = br.sec[pt.src].dim, di = bl.sec[pt.dst].dim;
      const int ib = (int)items.size();
      items.push_back({Sm.as<double>() + soff[pt.src], pt.blk, dj, pt.ldb, dj, 0, 1.0});
      tiles64(units, Sn.as<double>() + noff[pt.dst] + pt.r0 * di, di, (int)suf[pt.src].size(), di, ib, ib + 1);
    }
    gemm_once(GEMM_NT, items, units);
    std::swap(Sm, Sn);
    suf.swap(nsuf);
    soff.swap(noff);
  }
  // amplitudes per sector of the cut, rank and sign tables, scatter
  const Bond& bc = B[cut];
  std::vector<CiSector> secs;
  std::vector<int> pa, pb, sa, sb;
  std::vector<double> ps, ss;
  long amp = 0;
  items.clear();
  units.clear();
  std::vector<std::pair<size_t, long>> amp_at;
  for (size_t i = 0; i < bc.sec.size(); ++i) {
    const long np = (long)pre[i].size(), ns = (long)suf[i].size();
    if (np == 0 || ns == 0) continue;
    const QN q = bc.sec[i].q;
    const int a0 = (q.n + q.sz) / 2, b0 = (q.n - q.sz) / 2;
    secs.push_back({amp, (long)pa.size(), (long)sa.size(), (int)np, (int)ns});
    for (const Str& p : pre[i]) {
      int par = 0;
      for (int o = 0; o < cut; ++o)
        if (p.a >> o & 1u) par += popc(p.b & ((1u << o) - 1));
      pa.push_back((int)colex_part(p.a, 0));
      pb.push_back((int)colex_part(p.b, 0));
      ps.push_back(par & 1 ? -1.0 : 1.0);
    }
    for (const Str& x : suf[i]) {
      int par = popc(x.a) * b0;
      for (int o = cut; o < L; ++o)
        if (x.a >> o & 1u) par += popc(x.b & ((1u << o) - 1));
      sa.push_back((int)colex_part(x.a, a0));
      sb.push_back((int)colex_part(x.b, b0));
      ss.push_back(par & 1 ? -1.0 : 1.0);
    }
    amp_at.push_back({i, amp});
    amp += np * ns;
  }
  DevMem Amp;
  Amp.reserve(std::max<long>(amp, 1) * 8);
  for (const auto& [i, off] : amp_at) {
    const int d = bc.sec[i].dim, np = (int)pre[i].size(), ns = (int)suf[i].size();
    const int ib = (int)items.size();
    items.push_back({P.as<double>() + poff[i], Sm.as<double>() + soff[i], d, d, d, 0, 1.0});
    tiles64(units, Amp.as<double>() + off, ns, np, ns, ib, ib + 1);
  }
  gemm_once(GEMM_NT, items, units);
  DevMem dsec, dpa, dpb, dps, dsa, dsb, dss;
  upload(dsec, secs, st);
  upload(dpa, pa, st);
  upload(dpb, pb, st);
  upload(dps, ps, st);
  upload(dsa, sa, st);
  upload(dsb, sb, st);
  upload(dss, ss, st);
  launch_fill(c, ci_dimension(L, prob_->n_alpha, prob_->n_beta), 0.0, st);
  launch_ci_scatter(Amp.as<double>(), dsec.as<CiSector>(), (int)secs.size(), dpa.as<int>(), dpb.as<int>(),
                    dps.as<double>(), dsa.as<int>(), dsb.as<int>(), dss.as<double>(), c, Nb, st);
  hip_check(hipStreamSynchronize(st), "mps_to_ci");
}

void ci_rdm12(int n, int na, int nb, hipStream_t st, const double* bra, const double* ket, double scale,
              double* gamma, double* Gamma, double* overlap) {
  DMRG_REQUIRE(n >= 1 && n <= 16, ST_EINVAL, "RDMs from CI vectors need 1..16 orbitals");
  const std::vector<uint32_t> sa = colex_strings(n, na), sb = colex_strings(n, nb);
  const long NA = (long)sa.size(), NB = (long)sb.size(), N = NA * NB;
  const int n2 = n * n, rows = n2 + 1;
  DevMem ta, tb;
  upload(ta, excitation_table(n, sa), st);
  upload(tb, excitation_table(n, sb), st);
  constexpr long CL = 8192;  // determinants per split-K item
  const long per_pass = std::max<long>(1, (512L << 20) / ((long)rows * CL * 8)) * CL;
  const long pass = std::min(per_pass, (N + CL - 1) / CL * CL);
  const bool same = bra == ket;
  DevMem Tb, Tk, G, dg, dG;
  Tb.reserve((size_t)rows * pass * 8);
  if (!same) Tk.reserve((size_t)rows * pass * 8);
  const double* TK = same ? Tb.as<double>() : Tk.as<double>();
  G.reserve((size_t)rows * rows * 8);
  for (long d0 = 0; d0 < N; d0 += pass) {
    const long dend = std::min(N, d0 + pass), nch = (dend - d0 + CL - 1) / CL;
    launch_ci_excite(bra, NA, NB, n2, ta.as<int>(), tb.as<int>(), Tb.as<double>(), CL, d0, dend, st);
    if (!same) launch_ci_excite(ket, NA, NB, n2, ta.as<int>(), tb.as<int>(), Tk.as<double>(), CL, d0, dend, st);
    std::vector<int> K;
    for (long g = 0; g < nch; ++g) K.push_back((int)std::min(CL, dend - d0 - g * CL));
    splitk_nt(Tb.as<double>(), rows * CL, TK, rows * CL, CL, rows, rows, K, G.as<double>(), d0 > 0, st);
  }
  dg.reserve((size_t)n2 * 8);
  dG.reserve((size_t)n2 * n2 * 8);
  launch_rdm_assemble(G.as<double>(), rows, n, scale, dg.as<double>(), dG.as<double>(), st);
  if (gamma) hip_check(hipMemcpyAsync(gamma, dg.p, (size_t)n2 * 8, hipMemcpyDeviceToHost, st), "rdm out");
  if (Gamma) hip_check(hipMemcpyAsync(Gamma, dG.p, (size_t)n2 * n2 * 8, hipMemcpyDeviceToHost, st), "rdm out");
  if (overlap)
    hip_check(hipMemcpyAsync(overlap, G.as<double>() + (long)n2 * rows + n2, 8, hipMemcpyDeviceToHost, st), "rdm out");
  hip_check(hipStreamSynchronize(st), "rdm");
}

}  // namespace dmrg
