// Matrix-product operator of the active-space Hamiltonian with Cholesky channels.
//
// H = sum_pq h_pq E_pq + 1/2 sum_pqru (pq|ru) sum_{x,y} a+_{p x} a+_{r y} a_{u y} a_{q x}
// (x, y spins; normal ordered) with (pq|ru) = sum_Q B^Q_pq B^Q_ru (the paper's
// factorised two-electron tensor, Sec. II.A).  The MPO is the two-site sweep's
// operator (Sec. II.H: the dense d^L operator is never formed).
//
// Channels at a cut with A = sites < c and B = sites >= c:
//   I  : nothing applied on A yet (right side carries the full H_B)
//   H  : everything applied on A (left side carries H_A)
//   N1 : exactly one ladder operator on A (normal on the left), keyed by it
//   C1 : exactly one ladder operator left on B, keyed by it (complementary left)
//   Q  : Cholesky density channel: left side sum_{pq in A} B^Q_pq E_pq, right
//        side sum_{rs in B} B^Q_rs E_rs -- every Coulomb-separable term
//        (pq on one side, rs on the other) runs through these N_Q channels.
//   PN : two operators on A, keyed by them (cuts c <= L/2)
//   PC : two operators left on B, keyed by them (cuts c > L/2)
// Jordan-Wigner strings are folded into the 4x4 site operators (site states
// s = n_alpha + 2 n_beta, spin orbitals ordered 0a,0b,1a,1b,...).
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace dmrg {

using Mat4 = std::array<double, 16>;  // row-major [s][s']

enum ChanKind : int { CK_I = 0, CK_H = 1, CK_N1 = 2, CK_C1 = 3, CK_Q = 4, CK_PN = 5, CK_PC = 6 };

struct MPOEntry {
  int a;      // channel at cut k
  int b;      // channel at cut k+1
  double c;   // coefficient
  int op;     // index into MPO::ops
};

// Gradient provenance: d(entry coefficient)/d(parameter) = f.
enum ParamKind : int { PK_H = 0, PK_G = 1, PK_B = 2 };
struct Prov {
  int entry;
  int kind;
  int i[4];
  double f;
};

struct Channel {
  uint64_t key;
  int kind;
  QN dq;  // change of the block quantum number produced by the channel's left operator
};

struct MPO {
  int L = 0, nq = 0, cmid = 0;
  std::vector<std::vector<Channel>> chans;  // per cut 0..L
  std::vector<std::vector<MPOEntry>> W;     // per site 0..L-1 (cut k -> cut k+1)
  std::vector<std::vector<Prov>> prov;      // per site
  std::vector<Mat4> ops;
  std::vector<int> chan_I, chan_H;          // per cut (-1 when absent)
  int dim(int cut) const { return (int)chans[cut].size(); }
};

// Builds the MPO from h (n*n row-major) and B (nq*n*n row-major).  Host only.
MPO build_mpo(int L, int nq, const double* h, const double* B);

// MPO of S_- S_+ = (sum_p s-_p)(sum_q s+_q), s+_p = a+_{p alpha} a_{p beta},
// s-_p = a+_{p beta} a_{p alpha}: the spin diagnostic of Sec. II.F, since
// <S^2> = <S_- S_+> + S_z (S_z + 1).  A sum-then-product operator of bond
// dimension 4 (channels I, s+ placed, s- placed, H); the on-site operators are
// even, so no Jordan-Wigner strings cross sites.  Host only.
MPO build_spin_mpo(int L);

// MPO whose entries carry the two-orbital operators of every pair i < j:
// channel (i, t, s) opens at site i with |t><s| and runs through the sites
// between with the identity (|t><s| even) or the parity diag(1, -1, -1, 1) (odd:
// the Jordan-Wigner string), and closes at site j with every |t_j><s_j| that
// conserves N and S_z.  Each closing entry belongs to one term, so the
// derivative of <Psi|O|Psi> by its coefficient is the expectation value
// <(|t><s|)_i P (|t_j><s_j|)_j>.  `closings` lists them: (site j, entry index
// in W[j], i, t, s, t_j, s_j).  Host only.
struct PairClosing {
  int j, entry, i, t, s, tj, sj;
};
MPO build_pair_mpo(int L, std::vector<PairClosing>& closings);

}  // namespace dmrg
