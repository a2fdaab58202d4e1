// Cholesky-channel MPO builder (host).  See mpo.hpp for the channel families.
//
// Construction: every Hamiltonian term is a product of ladder operators.  Sorted
// into site order (spin orbital 2*site+spin, stable), a term sits at each cut in
// exactly one channel (routing below).  Channels keyed by what is on the left
// (I, N1, PN) are "left-keyed", those keyed by what remains on the right (C1, PC,
// H) are "right-keyed"; a term's path crosses from left- to right-keyed exactly
// once, and that transition carries the term's coefficient.  All other
// transitions are shared by many terms and carry coefficient 1 (or B^Q for the
// Cholesky channels), so they are generated once per channel.
//
// Coulomb-separable two-electron terms ((pq| on one side of some cut, |rs) on the
// other) are not enumerated: the product of the Q-entry coefficient B^Q_pq and
// the Q-exit coefficient B^Q_rs, summed over the N_Q channels, reproduces
// (pq|rs) E_pq E_rs for all of them.
#include "mpo.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

namespace dmrg {
namespace {

struct Ladder {
  int site, spin, dag;  // spin 0 alpha / 1 beta; dag 1 = creation
};

inline int so_key(const Ladder& o) { return 2 * o.site + o.spin; }
inline int enc(const Ladder& o) { return o.site * 4 + o.spin * 2 + o.dag; }
inline QN ladder_dq(const Ladder& o) {
  int dn = o.dag ? 1 : -1;
  return {dn, (o.spin == 0 ? 1 : -1) * dn};
}

inline uint64_t key0(int kind) { return (uint64_t)kind << 56; }
inline uint64_t key1(int kind, const Ladder& o) { return ((uint64_t)kind << 56) | (uint64_t)enc(o); }
inline uint64_t key2(int kind, const Ladder& o1, const Ladder& o2) {
  return ((uint64_t)kind << 56) | ((uint64_t)enc(o1) << 20) | (uint64_t)enc(o2);
}
inline uint64_t keyQ(int q) { return ((uint64_t)CK_Q << 56) | (uint64_t)q; }
inline int key_kind(uint64_t k) { return (int)(k >> 56); }
inline Ladder dec(int e) { return {e >> 2, (e >> 1) & 1, e & 1}; }

QN key_dq(uint64_t k) {
  int kind = key_kind(k);
  switch (kind) {
    case CK_N1: return ladder_dq(dec((int)(k & 0xFFFFF)));
    case CK_C1: return -ladder_dq(dec((int)(k & 0xFFFFF)));
    case CK_PN: return ladder_dq(dec((int)((k >> 20) & 0xFFFFF))) + ladder_dq(dec((int)(k & 0xFFFFF)));
    case CK_PC: return -(ladder_dq(dec((int)((k >> 20) & 0xFFFFF))) + ladder_dq(dec((int)(k & 0xFFFFF))));
    default: return {0, 0};
  }
}

using Mat2 = std::array<double, 4>;
const Mat2 kI2 = {1, 0, 0, 1}, kF2 = {1, 0, 0, -1}, kCre = {0, 0, 1, 0}, kAnn = {0, 1, 0, 0};
Mat2 mul2(const Mat2& a, const Mat2& b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2],
          a[2] * b[1] + a[3] * b[3]};
}

// Site operator of the ladder operators at one site (listed in sorted, product
// order) when `n_after` operators of the term act on later sites.  With the
// Jordan-Wigner map a_j = (prod_{i<j} F_i) c_j, the strings of all operators
// combine into F_m^{r(m)} on spin orbital m (r(m) = operators on later spin
// orbitals), multiplied to the right of the ladder operators on m.
Mat4 local_op(const std::vector<Ladder>& ops, int n_after) {
  Mat2 m[2] = {kI2, kI2};
  int cnt[2] = {0, 0};
  for (const auto& o : ops) {
    m[o.spin] = mul2(m[o.spin], o.dag ? kCre : kAnn);
    cnt[o.spin]++;
  }
  int r[2] = {n_after + cnt[1], n_after};
  for (int s = 0; s < 2; ++s)
    if (r[s] & 1) m[s] = mul2(m[s], kF2);
  Mat4 out{};
  for (int s = 0; s < 4; ++s)
    for (int t = 0; t < 4; ++t)
      out[s * 4 + t] = m[0][(s & 1) * 2 + (t & 1)] * m[1][(s >> 1) * 2 + (t >> 1)];
  return out;
}

Mat4 add4(const Mat4& a, const Mat4& b) {
  Mat4 o;
  for (int i = 0; i < 16; ++i) o[i] = a[i] + b[i];
  return o;
}

bool is_zero(const Mat4& a) {
  for (double x : a)
    if (x != 0.0) return false;
  return true;
}

struct Builder {
  int L, nq, cmid;
  const double* h;
  const double* B;
  std::vector<double> g;
  std::vector<std::unordered_map<uint64_t, int>> chan_id;  // per cut
  std::vector<std::vector<uint64_t>> chan_key;
  struct EKey {
    int a, b, op;
    bool operator<(const EKey& o) const {
      return a != o.a ? a < o.a : (b != o.b ? b < o.b : op < o.op);
    }
  };
  std::vector<std::map<EKey, int>> entry_index;  // per site
  std::vector<std::vector<MPOEntry>> W;
  std::vector<std::vector<Prov>> prov;
  std::map<Mat4, int> op_id;
  std::vector<Mat4> ops;

  double Bq(int q, int p, int r) const { return B[((size_t)q * L + p) * L + r]; }

  int intern(const Mat4& m) {
    auto it = op_id.find(m);
    if (it != op_id.end()) return it->second;
    int id = (int)ops.size();
    ops.push_back(m);
    op_id.emplace(m, id);
    return id;
  }
  int chan(int cut, uint64_t key) {
    auto& mp = chan_id[cut];
    auto it = mp.find(key);
    if (it != mp.end()) return it->second;
    int id = (int)chan_key[cut].size();
    chan_key[cut].push_back(key);
    mp.emplace(key, id);
    return id;
  }
  // Adds (or accumulates into) W_site[a -> b] with site operator m.
  int add(int site, uint64_t ka, uint64_t kb, double c, const Mat4& m) {
    if (is_zero(m)) return -1;
    int a = chan(site, ka), b = chan(site + 1, kb), op = intern(m);
    EKey ek{a, b, op};
    auto& idx = entry_index[site];
    auto it = idx.find(ek);
    if (it != idx.end()) {
      W[site][it->second].c += c;
      return it->second;
    }
    int e = (int)W[site].size();
    W[site].push_back({a, b, c, op});
    idx.emplace(ek, e);
    return e;
  }
  void add_prov(int site, int e, int kind, int i0, int i1, int i2, int i3, double f) {
    if (e < 0) return;
    prov[site].push_back({e, kind, {i0, i1, i2, i3}, f});
  }

  std::vector<Ladder> ops_at(int site) const {
    std::vector<Ladder> v;
    for (int sp = 0; sp < 2; ++sp)
      for (int d = 0; d < 2; ++d) v.push_back({site, sp, d});
    return v;
  }

  void structural(int k) {
    const uint64_t I = key0(CK_I), H = key0(CK_H);
    const Mat4 id = local_op({}, 0);
    const Mat4 F = local_op({}, 1);
    add(k, I, I, 1.0, id);
    add(k, H, H, 1.0, id);
    auto here = ops_at(k);
    // I -> N1 (operator on site k), N1 propagation, C1 propagation / closing
    for (auto& o : here) add(k, I, key1(CK_N1, o), 1.0, local_op({o}, 1));
    for (int p = 0; p < k; ++p)
      for (auto& o : ops_at(p)) add(k, key1(CK_N1, o), key1(CK_N1, o), 1.0, F);
    for (int q = k; q < L; ++q)
      for (auto& o : ops_at(q)) {
        if (q > k) add(k, key1(CK_C1, o), key1(CK_C1, o), 1.0, F);
        else add(k, key1(CK_C1, o), H, 1.0, local_op({o}, 0));
      }
    // normal-left pair channels
    if (k + 1 <= cmid) {
      for (int p1 = 0; p1 < k; ++p1)
        for (int p2 = p1; p2 < k; ++p2)
          for (auto& o1 : ops_at(p1))
            for (auto& o2 : ops_at(p2)) {
              if (!pair_ok(o1, o2)) continue;
              add(k, key2(CK_PN, o1, o2), key2(CK_PN, o1, o2), 1.0, id);
            }
      for (int p1 = 0; p1 < k; ++p1)
        for (auto& o1 : ops_at(p1))
          for (auto& o2 : here) add(k, key1(CK_N1, o1), key2(CK_PN, o1, o2), 1.0, local_op({o2}, 2));
      for (auto& o1 : here)
        for (auto& o2 : here) {
          if (!pair_ok(o1, o2)) continue;
          add(k, I, key2(CK_PN, o1, o2), 1.0, local_op({o1, o2}, 2));
        }
    }
    // complementary-left pair channels
    if (k > cmid) {
      for (int q1 = k; q1 < L; ++q1)
        for (int q2 = q1; q2 < L; ++q2)
          for (auto& o3 : ops_at(q1))
            for (auto& o4 : ops_at(q2)) {
              if (!pair_ok(o3, o4)) continue;
              uint64_t kp = key2(CK_PC, o3, o4);
              if (q1 > k) add(k, kp, kp, 1.0, id);
              else if (q2 > k) add(k, kp, key1(CK_C1, o4), 1.0, local_op({o3}, 1));
              else add(k, kp, H, 1.0, local_op({o3, o4}, 0));
            }
    }
    // Cholesky density channels
    if (nq > 0) {
      Mat4 Ekk_in = add4(local_op({{k, 0, 1}, {k, 0, 0}}, 2), local_op({{k, 1, 1}, {k, 1, 0}}, 2));
      Mat4 Ekk_out = add4(local_op({{k, 0, 1}, {k, 0, 0}}, 0), local_op({{k, 1, 1}, {k, 1, 0}}, 0));
      for (int q = 0; q < nq; ++q) {
        uint64_t kq = keyQ(q);
        if (k + 1 <= L - 1) {
          int e = add(k, I, kq, Bq(q, k, k), Ekk_in);
          add_prov(k, e, PK_B, q, k, k, 0, 1.0);
          for (int p = 0; p < k; ++p)
            for (int sp = 0; sp < 2; ++sp) {
              e = add(k, key1(CK_N1, {p, sp, 1}), kq, Bq(q, p, k), local_op({{k, sp, 0}}, 2));
              add_prov(k, e, PK_B, q, p, k, 0, 1.0);
              e = add(k, key1(CK_N1, {p, sp, 0}), kq, -Bq(q, k, p), local_op({{k, sp, 1}}, 2));
              add_prov(k, e, PK_B, q, k, p, 0, -1.0);
            }
          if (k >= 1) add(k, kq, kq, 1.0, id);
        }
        if (k >= 1) {
          int e = add(k, kq, H, Bq(q, k, k), Ekk_out);
          add_prov(k, e, PK_B, q, k, k, 0, 1.0);
          for (int s = k + 1; s < L; ++s)
            for (int sp = 0; sp < 2; ++sp) {
              e = add(k, kq, key1(CK_C1, {s, sp, 0}), Bq(q, k, s), local_op({{k, sp, 1}}, 1));
              add_prov(k, e, PK_B, q, k, s, 0, 1.0);
              e = add(k, kq, key1(CK_C1, {s, sp, 1}), -Bq(q, s, k), local_op({{k, sp, 0}}, 1));
              add_prov(k, e, PK_B, q, s, k, 0, -1.0);
            }
        }
      }
    }
  }

  // A pair key is two operators in sorted order; on one spin orbital both
  // product orders (n and 1-n) are distinct keys, equal operators vanish.
  static bool pair_ok(const Ladder& o1, const Ladder& o2) {
    int k1 = so_key(o1), k2 = so_key(o2);
    if (k1 > k2) return false;
    if (k1 == k2 && o1.dag == o2.dag) return false;
    return true;
  }

  uint64_t route(const std::vector<Ladder>& s, int cut) const {
    int n = (int)s.size(), nl = 0;
    for (auto& o : s) nl += o.site < cut;
    if (nl == 0) return key0(CK_I);
    if (nl == n) return key0(CK_H);
    if (nl == 1) return key1(CK_N1, s[0]);
    if (n - nl == 1) return key1(CK_C1, s[n - 1]);
    return cut <= cmid ? key2(CK_PN, s[0], s[1]) : key2(CK_PC, s[2], s[3]);
  }
  static bool left_keyed(uint64_t k) {
    int kd = key_kind(k);
    return kd == CK_I || kd == CK_N1 || kd == CK_PN;
  }

  // Adds one enumerated term: coefficient c times the operator product `ops`.
  void add_term(double c, std::vector<Ladder> ops, int pkind, int i0, int i1, int i2, int i3,
                double pf) {
    // stable sort into spin-orbital order, counting swaps of distinct orbitals
    int n = (int)ops.size();
    double sign = 1.0;
    for (int i = 1; i < n; ++i)
      for (int j = i; j > 0 && so_key(ops[j - 1]) > so_key(ops[j]); --j) {
        std::swap(ops[j - 1], ops[j]);
        sign = -sign;
      }
    for (int cut = 0; cut < L; ++cut) {
      uint64_t a = route(ops, cut), b = route(ops, cut + 1);
      if (!(left_keyed(a) && !left_keyed(b))) continue;
      std::vector<Ladder> here;
      int after = 0;
      for (auto& o : ops) {
        if (o.site == cut) here.push_back(o);
        else if (o.site > cut) ++after;
      }
      int e = add(cut, a, b, c * sign, local_op(here, after));
      add_prov(cut, e, pkind, i0, i1, i2, i3, pf * sign);
      return;
    }
  }

  void enumerate() {
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int sp = 0; sp < 2; ++sp)
          add_term(h[p * L + q], {{p, sp, 1}, {q, sp, 0}}, PK_H, p, q, 0, 0, 1.0);
    if (nq == 0) return;
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s) {
            bool sep = std::max(p, q) < std::min(r, s) || std::max(r, s) < std::min(p, q);
            if (sep) continue;
            double c = 0.5 * g[(((size_t)p * L + q) * L + r) * L + s];
            for (int x = 0; x < 2; ++x)
              for (int y = 0; y < 2; ++y) {
                if (p == r && x == y) continue;  // a+ a+ on one spin orbital
                if (q == s && x == y) continue;
                add_term(c, {{p, x, 1}, {r, y, 1}, {s, y, 0}, {q, x, 0}}, PK_G, p, q, r, s, 0.5);
              }
          }
  }
};

}  // namespace

MPO build_mpo(int L, int nq, const double* h, const double* B) {
  DMRG_REQUIRE(L >= 2 && L <= 64, ST_EINVAL, "n_orb must be in [2, 64]");
  Builder b;
  b.L = L;
  b.nq = nq;
  b.cmid = L / 2;
  b.h = h;
  b.B = B;
  b.g.assign((size_t)L * L * L * L, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int p = 0; p < L * L; ++p) {
      double x = B[(size_t)q * L * L + p];
      if (x == 0.0) continue;
      for (int r = 0; r < L * L; ++r) b.g[(size_t)p * L * L + r] += x * B[(size_t)q * L * L + r];
    }
  b.chan_id.resize(L + 1);
  b.chan_key.resize(L + 1);
  b.entry_index.resize(L);
  b.W.resize(L);
  b.prov.resize(L);
  for (int k = 0; k < L; ++k) b.structural(k);
  b.enumerate();

  // prune channels not on a path from I(cut 0) to H(cut L)
  std::vector<std::vector<char>> fwd(L + 1), bwd(L + 1);
  for (int c = 0; c <= L; ++c) {
    fwd[c].assign(b.chan_key[c].size(), 0);
    bwd[c].assign(b.chan_key[c].size(), 0);
  }
  {
    auto it = b.chan_id[0].find(key0(CK_I));
    DMRG_REQUIRE(it != b.chan_id[0].end(), ST_EINVAL, "MPO has no identity channel");
    fwd[0][it->second] = 1;
    auto ih = b.chan_id[L].find(key0(CK_H));
    DMRG_REQUIRE(ih != b.chan_id[L].end(), ST_EINVAL, "MPO has no closing channel");
    bwd[L][ih->second] = 1;
  }
  // An entry whose coefficient is an integral stays even when that integral is
  // exactly zero: it adds nothing to H but carries dE/d(integral).
  std::vector<std::vector<char>> live(L);
  for (int k = 0; k < L; ++k) {
    live[k].assign(b.W[k].size(), 0);
    for (size_t i = 0; i < b.W[k].size(); ++i) live[k][i] = b.W[k][i].c != 0.0;
    for (auto& p : b.prov[k]) live[k][p.entry] = 1;
  }
  for (int k = 0; k < L; ++k)
    for (size_t i = 0; i < b.W[k].size(); ++i)
      if (fwd[k][b.W[k][i].a] && live[k][i]) fwd[k + 1][b.W[k][i].b] = 1;
  for (int k = L - 1; k >= 0; --k)
    for (size_t i = 0; i < b.W[k].size(); ++i)
      if (bwd[k + 1][b.W[k][i].b] && live[k][i]) bwd[k][b.W[k][i].a] = 1;

  MPO m;
  m.L = L;
  m.nq = nq;
  m.cmid = b.cmid;
  m.ops = b.ops;
  m.chans.resize(L + 1);
  m.chan_I.assign(L + 1, -1);
  m.chan_H.assign(L + 1, -1);
  std::vector<std::vector<int>> remap(L + 1);
  for (int c = 0; c <= L; ++c) {
    std::vector<std::pair<std::pair<QN, uint64_t>, int>> live;
    for (size_t i = 0; i < b.chan_key[c].size(); ++i)
      if (fwd[c][i] && bwd[c][i]) live.push_back({{key_dq(b.chan_key[c][i]), b.chan_key[c][i]}, (int)i});
    std::sort(live.begin(), live.end(), [](const auto& x, const auto& y) {
      if (x.first.first != y.first.first) return x.first.first < y.first.first;
      return x.first.second < y.first.second;
    });
    remap[c].assign(b.chan_key[c].size(), -1);
    for (size_t j = 0; j < live.size(); ++j) {
      uint64_t key = live[j].first.second;
      remap[c][live[j].second] = (int)j;
      m.chans[c].push_back({key, key_kind(key), live[j].first.first});
      if (key_kind(key) == CK_I) m.chan_I[c] = (int)j;
      if (key_kind(key) == CK_H) m.chan_H[c] = (int)j;
    }
  }
  m.W.resize(L);
  m.prov.resize(L);
  for (int k = 0; k < L; ++k) {
    std::vector<int> emap(b.W[k].size(), -1);
    for (size_t i = 0; i < b.W[k].size(); ++i) {
      const auto& e = b.W[k][i];
      int a = remap[k][e.a], bb = remap[k + 1][e.b];
      if (a < 0 || bb < 0 || !live[k][i]) continue;
      emap[i] = (int)m.W[k].size();
      m.W[k].push_back({a, bb, e.c, e.op});
    }
    for (auto& p : b.prov[k])
      if (emap[p.entry] >= 0) {
        Prov q = p;
        q.entry = emap[p.entry];
        m.prov[k].push_back(q);
      }
  }
  return m;
}

MPO build_spin_mpo(int L) {
  DMRG_REQUIRE(L >= 2 && L <= 64, ST_EINVAL, "n_orb must be in [2, 64]");
  // site states s = n_alpha + 2 n_beta, matrices [s][s']
  Mat4 id{}, sp{}, sm{}, smsp{};
  for (int s = 0; s < 4; ++s) id[s * 4 + s] = 1.0;
  sp[1 * 4 + 2] = 1.0;    // |beta> -> |alpha>; |alpha beta> -> 0 (Pauli)
  sm[2 * 4 + 1] = 1.0;    // |alpha> -> |beta>
  smsp[2 * 4 + 2] = 1.0;  // s- s+ = n_beta (1 - n_alpha)
  MPO m;
  m.L = L;
  m.nq = 0;
  m.cmid = L / 2;
  m.ops = {id, sp, sm, smsp};
  enum { OP_ID = 0, OP_SP = 1, OP_SM = 2, OP_SMSP = 3 };
  // channels of an inner cut in (dq, key) order: s- placed, I, H, s+ placed
  const uint64_t kM = key1(CK_N1, Ladder{0, 1, 1}), kP = key1(CK_N1, Ladder{0, 0, 1});
  m.chans.resize(L + 1);
  m.chan_I.assign(L + 1, -1);
  m.chan_H.assign(L + 1, -1);
  std::vector<std::array<int, 4>> idx(L + 1, {-1, -1, -1, -1});  // I, H, P, M per cut
  for (int c = 0; c <= L; ++c) {
    const bool inner = c > 0 && c < L;
    if (inner) {
      idx[c][3] = (int)m.chans[c].size();
      m.chans[c].push_back({kM, CK_N1, {0, -2}});
    }
    if (c < L) {
      idx[c][0] = (int)m.chans[c].size();
      m.chans[c].push_back({key0(CK_I), CK_I, {0, 0}});
    }
    if (c > 0) {
      idx[c][1] = (int)m.chans[c].size();
      m.chans[c].push_back({key0(CK_H), CK_H, {0, 0}});
    }
    if (inner) {
      idx[c][2] = (int)m.chans[c].size();
      m.chans[c].push_back({kP, CK_N1, {0, 2}});
    }
    m.chan_I[c] = idx[c][0];
    m.chan_H[c] = idx[c][1];
  }
  m.W.resize(L);
  m.prov.resize(L);
  for (int k = 0; k < L; ++k) {
    const auto& a = idx[k];
    const auto& b = idx[k + 1];
    auto add = [&](int ca, int cb, int op) {
      if (ca >= 0 && cb >= 0) m.W[k].push_back({ca, cb, 1.0, op});
    };
    add(a[0], b[0], OP_ID);    // nothing yet
    add(a[0], b[2], OP_SP);    // s+ on this site, s- to come
    add(a[0], b[3], OP_SM);    // s- on this site, s+ to come
    add(a[0], b[1], OP_SMSP);  // both on this site
    add(a[2], b[2], OP_ID);
    add(a[2], b[1], OP_SM);
    add(a[3], b[3], OP_ID);
    add(a[3], b[1], OP_SP);
    add(a[1], b[1], OP_ID);    // done
  }
  return m;
}

MPO build_pair_mpo(int L, std::vector<PairClosing>& closings) {
  DMRG_REQUIRE(L >= 2 && L <= 64, ST_EINVAL, "n_orb must be in [2, 64]");
  MPO m;
  m.L = L;
  m.nq = 0;
  m.cmid = L / 2;
  // ops: 0 identity, 1 parity, 2 + 4 t + s: |t><s|
  Mat4 id{}, par{};
  for (int u = 0; u < 4; ++u) {
    id[u * 4 + u] = 1.0;
    par[u * 4 + u] = (u == 1 || u == 2) ? -1.0 : 1.0;
  }
  m.ops = {id, par};
  for (int t = 0; t < 4; ++t)
    for (int s = 0; s < 4; ++s) {
      Mat4 o{};
      o[t * 4 + s] = 1.0;
      m.ops.push_back(o);
    }
  auto odd = [](int t, int s) { return (__builtin_popcount(t) + __builtin_popcount(s)) & 1; };
  // channels per cut, sorted by (dq, key): I (cuts 0..L-1), H (cuts 1..L), and
  // (i, t, s) for i < c <= L-1
  const uint64_t kI = key0(CK_I), kH = key0(CK_H);
  auto kO = [](int i, int t, int s) { return ((uint64_t)CK_N1 << 56) | ((uint64_t)i << 8) | (uint64_t)(4 * t + s); };
  m.chans.resize(L + 1);
  m.chan_I.assign(L + 1, -1);
  m.chan_H.assign(L + 1, -1);
  std::vector<std::map<uint64_t, int>> idx(L + 1);
  for (int c = 0; c <= L; ++c) {
    std::vector<std::pair<std::pair<QN, uint64_t>, int>> live;  // ((dq, key), kind)
    if (c < L) live.push_back({{QN{0, 0}, kI}, CK_I});
    if (c > 0) live.push_back({{QN{0, 0}, kH}, CK_H});
    if (c < L)
      for (int i = 0; i < c; ++i)
        for (int t = 0; t < 4; ++t)
          for (int s = 0; s < 4; ++s) live.push_back({{site_qn(t) - site_qn(s), kO(i, t, s)}, CK_N1});
    std::sort(live.begin(), live.end(), [](const auto& x, const auto& y) {
      if (x.first.first != y.first.first) return x.first.first < y.first.first;
      return x.first.second < y.first.second;
    });
    for (size_t j = 0; j < live.size(); ++j) {
      idx[c][live[j].first.second] = (int)j;
      m.chans[c].push_back({live[j].first.second, live[j].second, live[j].first.first});
      if (live[j].second == CK_I) m.chan_I[c] = (int)j;
      if (live[j].second == CK_H) m.chan_H[c] = (int)j;
    }
  }
  m.W.resize(L);
  m.prov.resize(L);
  closings.clear();
  for (int k = 0; k < L; ++k) {
    auto at = [&](int c, uint64_t key) {
      auto it = idx[c].find(key);
      return it == idx[c].end() ? -1 : it->second;
    };
    auto add = [&](int a, int b, double c, int op) {
      if (a >= 0 && b >= 0) m.W[k].push_back({a, b, c, op});
    };
    add(at(k, kI), at(k + 1, kI), 1.0, 0);
    if (k == 0) add(at(0, kI), at(1, kH), 0.0, 0);  // keeps H at cut 1 (the norm's right channel)
    for (int t = 0; t < 4; ++t)
      for (int s = 0; s < 4; ++s) add(at(k, kI), at(k + 1, kO(k, t, s)), 1.0, 2 + 4 * t + s);
    for (int i = 0; i < k; ++i)
      for (int t = 0; t < 4; ++t)
        for (int s = 0; s < 4; ++s) {
          const int a = at(k, kO(i, t, s));
          add(a, at(k + 1, kO(i, t, s)), 1.0, odd(t, s) ? 1 : 0);
          const QN d = site_qn(s) - site_qn(t);  // what the closing operator must change
          for (int tj = 0; tj < 4; ++tj)
            for (int sj = 0; sj < 4; ++sj) {
              if (site_qn(tj) - site_qn(sj) != d) continue;
              closings.push_back({k, (int)m.W[k].size(), i, t, s, tj, sj});
              add(a, at(k + 1, kH), 1.0, 2 + 4 * tj + sj);
            }
        }
    if (k > 0) add(at(k, kH), at(k + 1, kH), 1.0, 0);
  }
  return m;
}

}  // namespace dmrg
