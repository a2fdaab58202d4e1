// Excited states by penalty deflation, and the spin diagnostic (Sec. II.F).
//
// Lower converged states Phi_j (MPS of the same active space and sector) stay
// on the device.  The state being optimised, Psi, meets each of them through
// overlap environments: at cut c, OL_j[c] = <left basis of Psi at c | part of
// Phi_j on the sites before c> and OR_j[c] the same on the sites from c on,
// block-diagonal by quantum number (dim_Psi x dim_Phi per common sector).  At
// the two-site step k the projection of Phi_j into the step's space is
//   phi_j[a s1 s2 b] = sum OL_j[k][a a'] Phi_k[a' s1 m] Phi_{k+1}[m s2 b'] OR_j[k+2][b b'],
// i.e. P Phi_j for the projector P on the step's orthonormal two-site basis, so
// the projected penalty operator P (H + sum_j w_j |Phi_j><Phi_j|) P is exactly
// H_eff + sum_j w_j |phi_j><phi_j| (Phi_j normalised): a rank-n update of the
// sigma product in fp64.
//
// The dual penalty lambda S_z^2 + mu (N - N_el)^2 of the paper vanishes on every
// state of the (N_el, S_z) sector; the solver's quantum-number blocks never leave
// that sector, so the penalty is identically zero here and is not formed.
#include <cmath>

#include "mpo.hpp"
#include "solver.hpp"

namespace dmrg {
namespace {

// Block offsets of a block-diagonal matrix between bonds a (rows) and b
// (columns): per sector of a, the element offset of its dim_a x dim_b block, or
// -1 where b lacks the sector.
std::vector<long> ovl_layout(const Bond& a, const Bond& b, long& size) {
  std::vector<long> off(a.sec.size(), -1);
  size = 0;
  for (size_t i = 0; i < a.sec.size(); ++i) {
    const int j = b.find(a.sec[i].q);
    if (j < 0) continue;
    off[i] = size;
    size += (long)a.sec[i].dim * b.sec[j].dim;
  }
  return off;
}

void tiles(std::vector<GemmUnit>& units, double* C, int ldc, int M, int N, int ib, int ie) {
  for (int m0 = 0; m0 < M; m0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) units.push_back({C, ldc, M, N, m0, n0, ib, ie, 0});
}

}  // namespace

// in: overlap at cut `site` (rows: bra bond, columns: ket bond); out: cut site+1.
// out[q'] = sum_{q, s} bra(q, s, q')^T in[q] ket(q, s, q').
void Solver::ovl_update_left(const MPSView& bra, const MPSView& ket, int site, const double* in, double* out) {
  const Bond& ba = (*bra.bonds)[site];
  const Bond& bb = (*bra.bonds)[site + 1];
  const Bond& ka = (*ket.bonds)[site];
  const Bond& kb = (*ket.bonds)[site + 1];
  const SiteTensor& A = (*bra.sites)[site];
  const SiteTensor& K = (*ket.sites)[site];
  long s_in = 0, s_out = 0;
  const std::vector<long> oin = ovl_layout(ba, ka, s_in);
  const std::vector<long> oout = ovl_layout(bb, kb, s_out);
  struct Part {
    int out_sec;        // bra sector at cut site+1
    const double* bra;  // bra block (rows: bra sector at cut site)
    int lda, rows;
    long t_off;
    int cols;           // ket sector dim at cut site+1
  };
  struct First {
    const double* in;
    int ldi;
    const double* ket;
    int ldk;
  };
  std::vector<Part> parts;
  std::vector<First> firsts;
  long tsize = 0;
  for (size_t i = 0; i < ba.sec.size(); ++i) {
    if (oin[i] < 0) continue;
    const int j = ka.find(ba.sec[i].q);
    const int sa = A.lay.slab_of_left[i], sk = K.lay.slab_of_left[j];
    if (sa < 0 || sk < 0) continue;
    const Slab& SA = A.lay.slabs[sa];
    const Slab& SK = K.lay.slabs[sk];
    for (const auto& kbk : SK.blocks) {
      const int rb = bb.find(kb.sec[kbk.ri].q);
      if (rb < 0) continue;
      const int ab = SA.block_of(kbk.phys, rb);
      if (ab < 0) continue;
      parts.push_back({rb, A.buf.as<double>() + SA.off + SA.blocks[ab].col0, SA.width, ba.sec[i].dim, tsize, kbk.mr});
      firsts.push_back({in + oin[i], ka.sec[j].dim, K.buf.as<double>() + SK.off + kbk.col0, SK.width});
      tsize += (long)ba.sec[i].dim * kbk.mr;
    }
  }
  defl_t_.reserve(std::max<long>(tsize, 1) * 8);
  double* T = defl_t_.as<double>();
  // T(q, s, q') = in[q] ket(q, s, q')
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  for (size_t p = 0; p < parts.size(); ++p) {
    const Part& pt = parts[p];
    const First& f = firsts[p];
    const int ib = (int)items.size();
    items.push_back({f.in, f.ket, f.ldi, f.ldk, f.ldi, 0, 1.0});
    tiles(units, T + pt.t_off, pt.cols, pt.rows, pt.cols, ib, ib + 1);
  }
  gemm_once(GEMM_NN, items, units);
  // out[q'] = sum bra(q, s, q')^T T(q, s, q')
  items.clear();
  units.clear();
  for (size_t r = 0; r < bb.sec.size(); ++r) {
    if (oout[r] < 0) continue;
    const int kr = kb.find(bb.sec[r].q);
    const int ib = (int)items.size();
    for (const Part& pt : parts)
      if (pt.out_sec == (int)r) items.push_back({pt.bra, T + pt.t_off, pt.lda, pt.cols, pt.rows, 0, 1.0});
    tiles(units, out + oout[r], kb.sec[kr].dim, bb.sec[r].dim, kb.sec[kr].dim, ib, (int)items.size());
  }
  gemm_once(GEMM_TN, items, units);
}

// in: overlap at cut site+1; out: cut site.
// out[q] = sum_{s, q'} bra(q, s, q') in[q'] ket(q, s, q')^T.
void Solver::ovl_update_right(const MPSView& bra, const MPSView& ket, int site, const double* in, double* out) {
  const Bond& ba = (*bra.bonds)[site];
  const Bond& bb = (*bra.bonds)[site + 1];
  const Bond& ka = (*ket.bonds)[site];
  const Bond& kb = (*ket.bonds)[site + 1];
  const SiteTensor& A = (*bra.sites)[site];
  const SiteTensor& K = (*ket.sites)[site];
  long s_in = 0, s_out = 0;
  const std::vector<long> oin = ovl_layout(bb, kb, s_in);
  const std::vector<long> oout = ovl_layout(ba, ka, s_out);
  struct Part {
    int out_sec;  // bra sector at cut site
    const double* bra;
    int lda;
    const double* in;
    int ldi;      // ket dim of the sector at cut site+1
    int rows;     // bra dim at cut site
    int kin;      // bra dim at cut site+1
    const double* ket;
    int ldk;
    long u_off;
  };
  std::vector<Part> parts;
  long usize = 0;
  for (size_t i = 0; i < ba.sec.size(); ++i) {
    if (oout[i] < 0) continue;
    const int j = ka.find(ba.sec[i].q);
    const int sa = A.lay.slab_of_left[i], sk = K.lay.slab_of_left[j];
    if (sa < 0 || sk < 0) continue;
    const Slab& SA = A.lay.slabs[sa];
    const Slab& SK = K.lay.slabs[sk];
    for (const auto& abk : SA.blocks) {
      if (oin[abk.ri] < 0) continue;
      const int rk = kb.find(bb.sec[abk.ri].q);
      const int kbk = SK.block_of(abk.phys, rk);
      if (kbk < 0) continue;
      parts.push_back({(int)i, A.buf.as<double>() + SA.off + abk.col0, SA.width, in + oin[abk.ri], kb.sec[rk].dim,
                       ba.sec[i].dim, abk.mr, K.buf.as<double>() + SK.off + SK.blocks[kbk].col0, SK.width, usize});
      usize += (long)ba.sec[i].dim * kb.sec[rk].dim;
    }
  }
  defl_t_.reserve(std::max<long>(usize, 1) * 8);
  double* U = defl_t_.as<double>();
  // U(q, s, q') = bra(q, s, q') in[q']
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  for (const Part& pt : parts) {
    const int ib = (int)items.size();
    items.push_back({pt.bra, pt.in, pt.lda, pt.ldi, pt.kin, 0, 1.0});
    tiles(units, U + pt.u_off, pt.ldi, pt.rows, pt.ldi, ib, ib + 1);
  }
  gemm_once(GEMM_NN, items, units);
  // out[q] = sum U(q, s, q') ket(q, s, q')^T
  items.clear();
  units.clear();
  for (size_t i = 0; i < ba.sec.size(); ++i) {
    if (oout[i] < 0) continue;
    const int j = ka.find(ba.sec[i].q);
    const int ib = (int)items.size();
    for (const Part& pt : parts)
      if (pt.out_sec == (int)i) items.push_back({U + pt.u_off, pt.ket, pt.ldi, pt.ldk, pt.ldi, 0, 1.0});
    tiles(units, out + oout[i], ka.sec[j].dim, ba.sec[i].dim, ka.sec[j].dim, ib, (int)items.size());
  }
  gemm_once(GEMM_NT, items, units);
}

// <bra|ket> over the whole chain (left to right from the vacuum).
double Solver::chain_overlap(const MPSView& bra, const MPSView& ket) {
  long sz = 0, mx = 1;
  for (int c = 0; c <= L_; ++c) {
    ovl_layout((*bra.bonds)[c], (*ket.bonds)[c], sz);
    mx = std::max(mx, sz);
  }
  defl_a_.reserve(mx * 8);
  defl_b_.reserve(mx * 8);
  double* cur = defl_a_.as<double>();
  double* nxt = defl_b_.as<double>();
  launch_fill(cur, 1, 1.0, st);  // cut 0: the vacuum on both sides
  for (int site = 0; site < L_; ++site) {
    ovl_update_left(bra, ket, site, cur, nxt);
    std::swap(cur, nxt);
  }
  ovl_layout((*bra.bonds)[L_], (*ket.bonds)[L_], sz);
  double v = 0.0;
  if (sz == 1) {
    hip_check(hipMemcpyAsync(&v, cur, 8, hipMemcpyDeviceToHost, st), "overlap");
    hip_check(hipStreamSynchronize(st), "overlap");
  }
  return v;
}

void Solver::deflate_add(const std::vector<Bond>& bonds, const std::vector<const double*>& sites, double w) {
  materialize();
  DMRG_REQUIRE(std::isfinite(w) && w > 0.0, ST_EINVAL, "deflation weight must be finite and positive");
  DMRG_REQUIRE((int)defl_.size() < 32, ST_EINVAL, "at most 32 deflated states");
  DMRG_REQUIRE((int)bonds.size() == L_ + 1 && (int)sites.size() == L_, ST_EINVAL, "MPS size mismatch");
  DMRG_REQUIRE((bonds[0].sec.size() == 1 && bonds[0].sec[0].q == QN{0, 0} && bonds[0].sec[0].dim == 1), ST_EINVAL,
               "left boundary bond must be the single vacuum state");
  DMRG_REQUIRE(bonds[L_].sec.size() == 1 && bonds[L_].sec[0].q == prob_->target() && bonds[L_].sec[0].dim == 1,
               ST_EINVAL, "right boundary bond must be the single target state");
  for (int c = 0; c <= L_; ++c)
    for (size_t i = 0; i < bonds[c].sec.size(); ++i) {
      DMRG_REQUIRE(bonds[c].sec[i].dim >= 1, ST_EINVAL, "sector dims must be positive");
      if (i) DMRG_REQUIRE(bonds[c].sec[i - 1].q < bonds[c].sec[i].q, ST_EINVAL, "sectors must be sorted");
    }
  Deflated d;
  d.w = w;
  d.bonds = bonds;
  d.sites.resize(L_);
  for (int k = 0; k < L_; ++k) {
    SiteTensor& t = d.sites[k];
    t.lay = make_tensor_layout(bonds[k], bonds[k + 1], site_phys_qn());
    t.buf.reserve(std::max<long>(t.lay.size, 1) * 8);
    if (t.lay.size > 0)
      hip_check(hipMemcpyAsync(t.buf.p, sites[k], t.lay.size * 8, hipMemcpyHostToDevice, st), "deflated upload");
  }
  hip_check(hipStreamSynchronize(st), "deflated upload");
  const MPSView v{&d.bonds, &d.sites};
  const double n2 = chain_overlap(v, v);
  DMRG_REQUIRE(std::isfinite(n2) && n2 > 0.0, ST_EINVAL, "deflated state has zero norm");
  d.norm = std::sqrt(n2);
  d.ol.resize(L_ + 1);
  d.orr.resize(L_ + 1);
  d.ol_ok.assign(L_ + 1, 0);
  d.orr_ok.assign(L_ + 1, 0);
  defl_.push_back(std::move(d));
}

void Solver::deflate_clear() { defl_.clear(); }

void Solver::ovl_invalidate(int first_left, int last_right) {
  for (Deflated& d : defl_) {
    for (int c = std::max(first_left, 0); c <= L_; ++c) d.ol_ok[c] = 0;
    for (int c = 0; c <= std::min(last_right, L_); ++c) d.orr_ok[c] = 0;
  }
}

void Solver::ensure_ovl_left(int j, int c) {
  Deflated& d = defl_[j];
  if (d.ol_ok[c]) return;
  long sz = 0;
  ovl_layout(bonds_[c], d.bonds[c], sz);
  if (c == 0) {
    d.ol[0].reserve(8);
    launch_fill(d.ol[0].as<double>(), 1, 1.0, st);
    d.ol_ok[0] = 1;
    return;
  }
  ensure_ovl_left(j, c - 1);
  d.ol[c].reserve(std::max<long>(sz, 1) * 8);
  ovl_update_left({&bonds_, &mps_}, {&d.bonds, &d.sites}, c - 1, d.ol[c - 1].as<double>(), d.ol[c].as<double>());
  d.ol_ok[c] = 1;
}

void Solver::ensure_ovl_right(int j, int c) {
  Deflated& d = defl_[j];
  if (d.orr_ok[c]) return;
  long sz = 0;
  ovl_layout(bonds_[c], d.bonds[c], sz);
  if (c == L_) {
    d.orr[L_].reserve(8);
    launch_fill(d.orr[L_].as<double>(), 1, 1.0, st);
    d.orr_ok[L_] = 1;
    return;
  }
  ensure_ovl_right(j, c + 1);
  d.orr[c].reserve(std::max<long>(sz, 1) * 8);
  ovl_update_right({&bonds_, &mps_}, {&d.bonds, &d.sites}, c, d.orr[c + 1].as<double>(), d.orr[c].as<double>());
  d.orr_ok[c] = 1;
}

void Solver::deflate_project(int k, int j, double scale, double* out) {
  DMRG_REQUIRE(j >= 0 && j < (int)defl_.size(), ST_EINVAL, "no such deflated state");
  DMRG_REQUIRE(k >= 0 && k + 1 < L_, ST_EINVAL, "two-site step out of range");
  materialize();
  ensure_ovl_left(j, k);
  ensure_ovl_right(j, k + 2);
  const Deflated& d = defl_[j];
  const Bond& pa = bonds_[k];
  const Bond& pb = bonds_[k + 2];
  const Bond& fa = d.bonds[k];
  const Bond& fm = d.bonds[k + 1];
  const Bond& fb = d.bonds[k + 2];
  const SiteTensor& F1 = d.sites[k];
  const SiteTensor& F2 = d.sites[k + 1];
  long s_l = 0, s_r = 0;
  const std::vector<long> ol = ovl_layout(pa, fa, s_l);
  const std::vector<long> orr = ovl_layout(pb, fb, s_r);
  const TensorLayout P = make_tensor_layout(pa, pb, twosite_phys_qn());
  // Z1(qa, s1) = OL[qa] Phi_k(qa, s1, qm): rows dim_Psi(qa), cols dim_Phi(qm)
  // Z2(qm, s2, qb) = Phi_{k+1}(qm, s2, qb) OR[qb]^T: rows dim_Phi(qm), cols dim_Psi(qb)
  std::vector<long> z1_off(pa.sec.size() * 4, -1);
  std::vector<int> z1_ld(pa.sec.size() * 4, 0);
  long zsize = 0;
  std::vector<GemmItem> it1, it2;
  std::vector<GemmUnit> un1, un2;
  struct Pend {
    long off;  // output block in Z
    int rows, cols;
    long env;  // block of OL (first products) or OR (second products)
  };
  std::vector<Pend> p1, p2;
  for (size_t ia = 0; ia < pa.sec.size(); ++ia) {
    if (ol[ia] < 0) continue;
    const int ja = fa.find(pa.sec[ia].q);
    const int sf = F1.lay.slab_of_left[ja];
    if (sf < 0) continue;
    const Slab& S = F1.lay.slabs[sf];
    for (const auto& b : S.blocks) {
      z1_off[ia * 4 + b.phys] = zsize;
      z1_ld[ia * 4 + b.phys] = b.mr;
      it1.push_back({nullptr, F1.buf.as<double>() + S.off + b.col0, fa.sec[ja].dim, S.width, fa.sec[ja].dim, 0, 1.0});
      p1.push_back({zsize, pa.sec[ia].dim, b.mr, ol[ia]});
      zsize += (long)pa.sec[ia].dim * b.mr;
    }
  }
  // per (Phi sector at k+1, s2, Psi sector at k+2)
  std::vector<long> z2_off(fm.sec.size() * 4 * pb.sec.size(), -1);
  for (size_t im = 0; im < fm.sec.size(); ++im) {
    const int sf = F2.lay.slab_of_left[im];
    if (sf < 0) continue;
    const Slab& S = F2.lay.slabs[sf];
    for (const auto& b : S.blocks) {
      const int ib = pb.find(fb.sec[b.ri].q);
      if (ib < 0 || orr[ib] < 0) continue;
      z2_off[(im * 4 + b.phys) * pb.sec.size() + ib] = zsize;
      it2.push_back({F2.buf.as<double>() + S.off + b.col0, nullptr, S.width, fb.sec[b.ri].dim, fb.sec[b.ri].dim, 0, 1.0});
      p2.push_back({zsize, fm.sec[im].dim, pb.sec[ib].dim, orr[ib]});
      zsize += (long)fm.sec[im].dim * pb.sec[ib].dim;
    }
  }
  defl_t_.reserve(std::max<long>(zsize, 1) * 8);
  double* Z = defl_t_.as<double>();
  const double* OL = d.ol[k].as<double>();
  const double* OR = d.orr[k + 2].as<double>();
  for (size_t i = 0; i < it1.size(); ++i) {
    it1[i].A = OL + p1[i].env;
    tiles(un1, Z + p1[i].off, p1[i].cols, p1[i].rows, p1[i].cols, (int)i, (int)i + 1);
  }
  for (size_t i = 0; i < it2.size(); ++i) {
    it2[i].B = OR + p2[i].env;
    tiles(un2, Z + p2[i].off, p2[i].cols, p2[i].rows, p2[i].cols, (int)i, (int)i + 1);
  }
  gemm_once(GEMM_NN, it1, un1);
  gemm_once(GEMM_NT, it2, un2);
  // phi block (qa, s1 s2, qb) = Z1(qa, s1) Z2(qm, s2, qb), qm = qa + q(s1): one product
  std::vector<GemmItem> it3;
  std::vector<GemmUnit> un3;
  for (const Slab& ps : P.slabs) {
    for (const auto& b : ps.blocks) {
      const int s1 = b.phys / 4, s2 = b.phys % 4;
      const int ib = (int)it3.size();
      const long o1 = z1_off[ps.li * 4 + s1];
      if (o1 >= 0) {
        const int im = fm.find(pa.sec[ps.li].q + site_qn(s1));
        const long o2 = im < 0 ? -1 : z2_off[((size_t)im * 4 + s2) * pb.sec.size() + b.ri];
        if (o2 >= 0) it3.push_back({Z + o1, Z + o2, z1_ld[ps.li * 4 + s1], b.mr, fm.sec[im].dim, 0, scale});
      }
      tiles(un3, out + ps.off + b.col0, ps.width, ps.ml, b.mr, ib, (int)it3.size());
    }
  }
  gemm_once(GEMM_NN, it3, un3);
}

double Solver::overlap(int j) {
  DMRG_REQUIRE(j >= 0 && j < (int)defl_.size(), ST_EINVAL, "no such deflated state");
  materialize();
  const MPSView me{&bonds_, &mps_};
  const double n2 = chain_overlap(me, me);
  DMRG_REQUIRE(n2 > 0.0, ST_ESTATE, "state has zero norm");
  const double o = chain_overlap(me, {&defl_[j].bonds, &defl_[j].sites});
  return o / (std::sqrt(n2) * defl_[j].norm);
}

void Solver::adopt_mps(const Solver& o) {
  DMRG_REQUIRE(o.L_ == L_ && o.prob_->target() == prob_->target(), ST_EINVAL, "MPS of another active space");
  DMRG_REQUIRE(o.pending_mps_.empty(), ST_ESTATE, "source MPS not on the device");
  std::vector<double>().swap(pending_mps_);
  bonds_ = o.bonds_;
  for (int k = 0; k < L_; ++k) {
    mps_[k].lay = o.mps_[k].lay;
    mps_[k].buf.reserve(std::max<long>(mps_[k].lay.size, 1) * 8);
    if (mps_[k].lay.size > 0)
      hip_check(hipMemcpyAsync(mps_[k].buf.p, o.mps_[k].buf.p, mps_[k].lay.size * 8, hipMemcpyDeviceToDevice, st),
                "mps copy");
  }
  centers_.clear();
  centers_.resize(o.centers_.size());
  center_lay_ = o.center_lay_;
  for (size_t r = 0; r < o.centers_.size(); ++r) {
    centers_[r].reserve(std::max<long>(center_lay_.size, 1) * 8);
    if (center_lay_.size > 0)
      hip_check(hipMemcpyAsync(centers_[r].p, o.centers_[r].p, center_lay_.size * 8, hipMemcpyDeviceToDevice, st),
                "centre copy");
  }
  center_site_ = o.center_site_;
  hip_check(hipStreamSynchronize(st), "mps copy");
  for (auto& e : left_) e.valid = false;
  for (auto& e : right_) e.valid = false;
  plan_k_ = -1;
  ovl_invalidate(0, L_);
}

// <S^2> = <S_- S_+> + S_z (S_z + 1) per root, through the solver's own
// environment and sigma kernels with the spin MPO in place of H (mps_energy of
// a solver of that operator holding a copy of this MPS).
std::vector<double> Solver::s_squared() {
  materialize();
  Problem p2;
  p2.n = L_;
  p2.n_alpha = prob_->n_alpha;
  p2.n_beta = prob_->n_beta;
  const double sz = 0.5 * (p2.n_alpha - p2.n_beta);
  p2.e_core = sz * (sz + 1.0);
  p2.mpo = build_spin_mpo(L_);
  Options o;
  o.M = 1;
  o.n_states = opt_.n_states;
  o.weights = opt_.weights;
  Solver s2(&p2, o, st);
  s2.adopt_mps(*this);
  return s2.mps_energy();
}

}  // namespace dmrg
