// Gradient of the MPS energy with respect to the active-space integrals: the
// Hellmann-Feynman contribution of the DMRG node's adjoint (Sec. II.C, the
// sweep as a differentiable node; Eq. (implicit) needs no response solve for
// the energy of a simple root of a stationary state).  The MPS is held fixed,
// so dE/dh and dE/dB^Q are contractions of the state's one- and two-body
// densities; those densities are never formed here.
//
// <Psi|H|Psi> is linear in the coefficients of the entries of any one MPO site.
// For an entry e = (alpha -> beta, c op) of W_k,
//   g_e = d<Psi|H|Psi>/dc_e = sum_{s s'} op[s][s'] < A_s R_{k+1}[beta] , L_k[alpha] A_s' >_F
// with the environments L_k (sites < k) and R_{k+1} (sites > k) of the stored
// MPS (any gauge).  The vectors P_{alpha,s'} = L_k[alpha] A_s' and
// Q_{beta,s} = A_s R_{k+1}[beta] live on blocks (i, j') of bond k x bond k+1
// with q(j') - q(i) fixed per (channel, state); grouped by that offset, every
// needed inner product is an entry of a dense G = P Q^T, a long-K GEMM on the
// fp64 matrix cores.  The MPO builder's provenance (d coefficient / d
// parameter) maps g to dE/dh_pq, dE/d(pq|rs) and dE/dB^Q_pq, and
// (pq|rs) = sum_Q B^Q_pq B^Q_rs carries the middle one back to B.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>

#include "solver.hpp"

namespace dmrg {

namespace {

struct PairBlock {
  int i, j;   // bond-k sector (bra), bond-(k+1) sector (ket)
  int mi, mj;
  long off;
};

struct PairClass {
  QN delta;  // q(j) - q(i)
  std::vector<PairBlock> blocks;
  long K = 0;
  std::vector<std::pair<int, int>> prow, qrow;  // (alpha, s'), (beta, s)
  std::map<std::pair<int, int>, int> prow_of, qrow_of;
};

int row_index(std::vector<std::pair<int, int>>& rows, std::map<std::pair<int, int>, int>& idx, int ch,
              int s) {
  auto key = std::make_pair(ch, s);
  auto it = idx.find(key);
  if (it != idx.end()) return it->second;
  int r = (int)rows.size();
  rows.push_back(key);
  idx.emplace(key, r);
  return r;
}

// Largest P or Q chunk, in doubles (two such buffers are live at once).
constexpr long kChunkElems = 1L << 29;
// K extent of one item of the G = P Q^T product (split-K granule).
constexpr int kGSplit = 4096;

}  // namespace

// g[e] = d<Psi|H|Psi>/dc_e for every entry of W_k (unnormalised state); with
// norm != nullptr also <Psi|Psi> = sum_s < A_s R_{k+1}[H], L_k[I] A_s >_F (the
// channels that are the identity on the left and on the right block).
void Solver::grad_site(int k, std::vector<double>& g, double* norm) {
  const MPO& mpo = prob_->mpo;
  ensure_left(k);
  ensure_right(k + 1);
  const Env& envl = left_[k];
  const Env& envr = right_[k + 1];
  const Bond& bl = bonds_[k];
  const Bond& br = bonds_[k + 1];
  const SiteTensor& A = mps_[k];
  const auto& W = mpo.W[k];
  g.assign(W.size(), 0.0);

  // classes of (i, j') blocks by quantum-number offset; rows each entry needs
  std::vector<PairClass> classes;
  std::map<std::pair<int, int>, int> class_of;
  auto get_class = [&](QN d) {
    auto it = class_of.find({d.n, d.sz});
    if (it != class_of.end()) return it->second;
    PairClass pc;
    pc.delta = d;
    for (int i = 0; i < (int)bl.sec.size(); ++i) {
      int j = br.find(bl.sec[i].q + d);
      if (j < 0) continue;
      pc.blocks.push_back({i, j, bl.sec[i].dim, br.sec[j].dim, pc.K});
      pc.K += (long)bl.sec[i].dim * br.sec[j].dim;
    }
    int c = (int)classes.size();
    classes.push_back(std::move(pc));
    class_of[{d.n, d.sz}] = c;
    return c;
  };
  struct Use { int cls, pr, qr; double w; };
  std::vector<std::vector<Use>> uses(W.size());
  const auto& chl = mpo.chans[k];
  const auto& chr = mpo.chans[k + 1];
  for (size_t e = 0; e < W.size(); ++e) {
    const Mat4& op = mpo.ops[W[e].op];
    for (int s = 0; s < 4; ++s)
      for (int sp = 0; sp < 4; ++sp) {
        double w = op[s * 4 + sp];
        if (w == 0.0) continue;
        QN d = site_qn(sp) - chl[W[e].a].dq;
        DMRG_REQUIRE(d == site_qn(s) - chr[W[e].b].dq, ST_EINVAL, "MPO entry breaks quantum-number conservation");
        int c = get_class(d);
        if (classes[c].K == 0) continue;
        int pr = row_index(classes[c].prow, classes[c].prow_of, W[e].a, sp);
        int qr = row_index(classes[c].qrow, classes[c].qrow_of, W[e].b, s);
        uses[e].push_back({c, pr, qr, w});
      }
  }
  std::vector<Use> norm_uses;
  if (norm) {
    const int I = mpo.chan_I[k], H = mpo.chan_H[k + 1];
    DMRG_REQUIRE(I >= 0 && H >= 0, ST_EINVAL, "no identity channels for the norm at this site");
    for (int s = 0; s < 4; ++s) {
      QN d = site_qn(s) - chl[I].dq;
      DMRG_REQUIRE(d == site_qn(s) - chr[H].dq, ST_EINVAL, "identity channels with a charge");
      int c = get_class(d);
      if (classes[c].K == 0) continue;
      int pr = row_index(classes[c].prow, classes[c].prow_of, I, s);
      int qr = row_index(classes[c].qrow, classes[c].qrow_of, H, s);
      norm_uses.push_back({c, pr, qr, 1.0});
    }
    *norm = 0.0;
  }

  std::vector<double> Ghost;
  for (size_t c = 0; c < classes.size(); ++c) {
    const PairClass& pc = classes[c];
    if (pc.prow.empty() || pc.K == 0) continue;
    const int nP = (int)pc.prow.size(), nQ = (int)pc.qrow.size();
    const int cP = (int)std::max<long>(1, std::min<long>(nP, kChunkElems / pc.K));
    const int cQ = (int)std::max<long>(1, std::min<long>(nQ, kChunkElems / pc.K));
    std::vector<double> Gc((size_t)nP * nQ, 0.0);
    for (int p0 = 0; p0 < nP; p0 += cP) {
      const int np = std::min(cP, nP - p0);
      // P rows: P_{alpha,s'}[i, j'] = L_k[alpha](i, i') A(i', s', j')
      Phase pp;
      pp.mode = GEMM_NN;
      for (int r = 0; r < np; ++r) {
        const int alpha = pc.prow[p0 + r].first, sp = pc.prow[p0 + r].second;
        const EnvClass& ec = envl.classes[envl.chan_class[alpha]];
        const long cbase = envl.chan_off(alpha);
        for (const PairBlock& pb : pc.blocks) {
          int ip = bl.find(bl.sec[pb.i].q - chl[alpha].dq);
          if (ip < 0) continue;
          int eb = ec.block_of_col[ip];
          if (eb < 0 || ec.blocks[eb].ri != pb.i) continue;
          int sl = A.lay.slab_of_left[ip];
          if (sl < 0) continue;
          const Slab& slab = A.lay.slabs[sl];
          int ab = slab.block_of(sp, pb.j);
          if (ab < 0) continue;
          int ib = (int)pp.items.size();
          pp.items.push_back({B_ENVL, cbase + ec.blocks[eb].off, B_PSI, slab.off + slab.blocks[ab].col0,
                              ec.blocks[eb].mc, slab.width, ec.blocks[eb].mc, 1.0});
          pp.units.push_back({B_T, (long)r * pc.K + pb.off, pb.mj, pb.mi, pb.mj, 0, 0, ib, ib + 1, 0});
          pp.flops += 2.0 * pb.mi * ec.blocks[eb].mc * pb.mj;
        }
      }
      grad_P_.reserve(std::max<long>((long)np * pc.K, 1) * 8);
      launch_fill(grad_P_.as<double>(), (long)np * pc.K, 0.0, st);
      for (int q0 = 0; q0 < nQ; q0 += cQ) {
        const int nq = std::min(cQ, nQ - q0);
        // Q rows: Q_{beta,s}[i, j'] = A(i, s, j) R_{k+1}[beta](j, j')
        Phase pq;
        pq.mode = GEMM_NN;
        for (int r = 0; r < nq; ++r) {
          const int beta = pc.qrow[q0 + r].first, s = pc.qrow[q0 + r].second;
          const EnvClass& ec = envr.classes[envr.chan_class[beta]];
          const long cbase = envr.chan_off(beta);
          for (const PairBlock& pb : pc.blocks) {
            int sl = A.lay.slab_of_left[pb.i];
            if (sl < 0) continue;
            int j = br.find(bl.sec[pb.i].q + site_qn(s));
            if (j < 0) continue;
            const Slab& slab = A.lay.slabs[sl];
            int ab = slab.block_of(s, j);
            if (ab < 0) continue;
            int eb = ec.block_of_col[pb.j];
            if (eb < 0 || ec.blocks[eb].ri != j) continue;
            int ib = (int)pq.items.size();
            pq.items.push_back({B_PSI, slab.off + slab.blocks[ab].col0, B_ENVR, cbase + ec.blocks[eb].off,
                                slab.width, ec.blocks[eb].mc, br.sec[j].dim, 1.0});
            pq.units.push_back({B_OUT, (long)r * pc.K + pb.off, pb.mj, pb.mi, pb.mj, 0, 0, ib, ib + 1, 0});
            pq.flops += 2.0 * pb.mi * br.sec[j].dim * pb.mj;
          }
        }
        // G chunk = P Q^T, K cut into split-K items
        Phase pg;
        pg.mode = GEMM_NT;
        for (long k0 = 0; k0 < pc.K; k0 += kGSplit) {
          int kk = (int)std::min<long>(kGSplit, pc.K - k0);
          pg.items.push_back({B_T, k0, B_OUT, k0, (int)pc.K, (int)pc.K, kk, 1.0});
        }
        pg.units.push_back({B_XMIX, 0, nq, np, nq, 0, 0, 0, (int)pg.items.size(), 0});
        pg.flops = 2.0 * np * nq * (double)pc.K;
        grad_Q_.reserve(std::max<long>((long)nq * pc.K, 1) * 8);
        grad_G_.reserve(std::max<long>((long)np * nq, 1) * 8);
        launch_fill(grad_Q_.as<double>(), (long)nq * pc.K, 0.0, st);
        void* bases[B_NBUF] = {};
        bases[B_PSI] = A.buf.p;
        bases[B_ENVL] = envl.buf.p;
        bases[B_ENVR] = envr.buf.p;
        bases[B_T] = grad_P_.p;
        bases[B_OUT] = grad_Q_.p;
        bases[B_XMIX] = grad_G_.p;
        size_t esz[B_NBUF] = {8, 8, 8, 8, 8, 8, 8, 8, 8};
        long sizes[B_NBUF] = {};
        sizes[B_PSI] = A.lay.size;
        sizes[B_ENVL] = envl.size;
        sizes[B_ENVR] = envr.size;
        sizes[B_T] = (long)np * pc.K;
        sizes[B_OUT] = (long)nq * pc.K;
        sizes[B_XMIX] = (long)np * nq;
        if (q0 == 0) run_phase(pp, PREC_F64, bases, esz, sizes);
        run_phase(pq, PREC_F64, bases, esz, sizes);
        run_phase(pg, PREC_F64, bases, esz, sizes);
        Ghost.resize((size_t)np * nq);
        hip_check(hipMemcpyAsync(Ghost.data(), grad_G_.p, Ghost.size() * 8, hipMemcpyDeviceToHost, st), "grad G");
        hip_check(hipStreamSynchronize(st), "grad site");  // local plans and staging die here
        for (int r = 0; r < np; ++r)
          for (int t = 0; t < nq; ++t) Gc[(size_t)(p0 + r) * nQ + q0 + t] = Ghost[(size_t)r * nq + t];
        st_.grad_flops += (q0 == 0 ? pp.flops : 0.0) + pq.flops + pg.flops;
      }
    }
    for (size_t e = 0; e < W.size(); ++e)
      for (const Use& u : uses[e])
        if (u.cls == (int)c) g[e] += u.w * Gc[(size_t)u.pr * nQ + u.qr];
    for (const Use& u : norm_uses)
      if (u.cls == (int)c) *norm += Gc[(size_t)u.pr * nQ + u.qr];
  }
}

// Per root r with weight w_r != 0: E_r = <Psi_r|H|Psi_r>/<Psi_r|Psi_r> + e_core and
// sum_r w_r dE_r/dh, dE_r/dB (entries of h and B treated as independent).
void Solver::grad(const std::vector<double>& w, std::vector<double>& dh, std::vector<double>& dB,
                  std::vector<double>& energies) {
  const MPO& mpo = prob_->mpo;
  const int n = prob_->n, nq = prob_->nq;
  const bool have_roots = center_site_ >= 0 && (int)centers_.size() == opt_.n_states;
  const int nr = have_roots ? opt_.n_states : 1;
  DMRG_REQUIRE(!w.empty() && (int)w.size() <= opt_.n_states, ST_EINVAL, "one weight per state");
  for (size_t r = (size_t)nr; r < w.size(); ++r)
    DMRG_REQUIRE(w[r] == 0.0, ST_ESTATE, "excited-state gradients need the centre tensors of a sweep");
  for (double x : w) DMRG_REQUIRE(std::isfinite(x), ST_EINVAL, "state weights must be finite");
  dh.assign((size_t)n * n, 0.0);
  dB.assign((size_t)nq * n * n, 0.0);
  energies.assign(w.size(), 0.0);
  std::vector<double> dg;  // d E / d(pq|rs), entries independent
  if (nq > 0) dg.assign((size_t)n * n * n * n, 0.0);
  auto t0 = std::chrono::steady_clock::now();

  const int c = center_site_;
  auto invalidate_around = [&](int site) {
    for (int cut = site + 1; cut <= L_; ++cut) left_[cut].valid = false;
    for (int cut = 0; cut <= site; ++cut) right_[cut].valid = false;
    plan_k_ = -1;
  };
  for (int r = 0; r < nr && r < (int)w.size(); ++r) {  // every root's energy is reported
    if (have_roots && r > 0) {
      launch_copy(mps_[c].buf.as<double>(), centers_[r].as<double>(), center_lay_.size, st);
      invalidate_around(c);
    }
    // g per site, normalised by <Psi|Psi> (the identity path through site 0)
    std::vector<std::vector<double>> gs(L_);
    double norm = 0.0;
    for (int k = 0; k < L_; ++k) grad_site(k, gs[k], k == 0 ? &norm : nullptr);
    DMRG_REQUIRE(norm > 0.0 && std::isfinite(norm), ST_ESTATE, "MPS has zero norm");
    double e0 = 0.0;
    for (size_t e = 0; e < mpo.W[0].size(); ++e) e0 += mpo.W[0][e].c * gs[0][e];
    energies[r] = e0 / norm + prob_->e_core;
    const double wr = w[r] / norm;
    if (wr != 0.0)
      for (int k = 0; k < L_; ++k)
        for (const Prov& p : mpo.prov[k]) {
          double v = wr * p.f * gs[k][p.entry];
          if (p.kind == PK_H) dh[(size_t)p.i[0] * n + p.i[1]] += v;
          else if (p.kind == PK_G) dg[(((size_t)p.i[0] * n + p.i[1]) * n + p.i[2]) * n + p.i[3]] += v;
          else dB[((size_t)p.i[0] * n + p.i[1]) * n + p.i[2]] += v;
        }
    if (have_roots && r > 0) {
      launch_copy(mps_[c].buf.as<double>(), centers_[0].as<double>(), center_lay_.size, st);
      invalidate_around(c);
    }
  }
  // (pq|rs) = sum_Q B^Q_pq B^Q_rs:  dE/dB^Q_ij += sum_rs (dg_ijrs + dg_rsij) B^Q_rs
  const size_t n2 = (size_t)n * n;
  for (int q = 0; q < nq; ++q) {
    const double* Bq = prob_->B.data() + (size_t)q * n2;
    double* out = dB.data() + (size_t)q * n2;
    for (size_t ij = 0; ij < n2; ++ij) {
      double acc = 0.0;
      for (size_t rs = 0; rs < n2; ++rs) acc += (dg[ij * n2 + rs] + dg[rs * n2 + ij]) * Bq[rs];
      out[ij] += acc;
    }
  }
  grad_P_.release();
  grad_Q_.release();
  grad_G_.release();
  st_.grad_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Two-orbital density matrices of the stored MPS (root 0), every pair i < j, in
// the determinant convention of the CI route (local creators moved to the front
// in the order i alpha, j alpha, i beta, j beta): each element is the
// derivative of <Psi|O|Psi> by one closing entry of the pair MPO (the same
// per-site contractions as the integral gradient), over <Psi|Psi>.  The MPO
// gives them with the site creators in chain order (i alpha, i beta, j alpha,
// j beta); reordering to the determinant convention flips the sign of a local
// state holding beta on i and alpha on j.
std::vector<double> Solver::pair_rdm_mps() {
  materialize();
  Problem p2;
  p2.n = L_;
  p2.n_alpha = prob_->n_alpha;
  p2.n_beta = prob_->n_beta;
  std::vector<PairClosing> closings;
  p2.mpo = build_pair_mpo(L_, closings);
  Options o;
  o.M = 1;
  Solver s2(&p2, o, st);
  s2.adopt_mps(*this);
  s2.centers_.clear();  // the MPS as stored
  std::vector<std::vector<double>> gs(L_);
  double norm = 0.0;
  for (int k = 0; k < L_; ++k) s2.grad_site(k, gs[k], k == 0 ? &norm : nullptr);
  DMRG_REQUIRE(norm > 0.0 && std::isfinite(norm), ST_ESTATE, "MPS has zero norm");
  const int np = L_ * (L_ - 1) / 2;
  std::vector<double> rho((size_t)np * 256, 0.0);
  auto pair_index = [&](int i, int j) { return i * L_ - i * (i + 1) / 2 + (j - i - 1); };
  auto tau = [](int ti, int tj) { return ((ti & 2) && (tj & 1)) ? -1.0 : 1.0; };
  for (const PairClosing& c : closings) {
    const int Lb = c.t + 4 * c.tj, Lk = c.s + 4 * c.sj;
    rho[(size_t)pair_index(c.i, c.j) * 256 + Lb * 16 + Lk] =
        tau(c.t, c.tj) * tau(c.s, c.sj) * gs[c.j][c.entry] / norm;
  }
  return rho;
}

}  // namespace dmrg
