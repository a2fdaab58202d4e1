// Environment layouts, factor premixing, and the grouped-GEMM plans of the
// environment updates and of sigma.
//
// The two-site effective Hamiltonian of sites (k, k+1) is written through the
// channels beta of the middle cut k+1:
//   H_eff = sum_beta  [sum_alpha L_k[alpha] (x) W_k[alpha,beta]]
//                  (x) [sum_gamma W_{k+1}[beta,gamma] (x) R_{k+2}[gamma]].
// Grouping W_k[., beta] by site operator gives left factors X_{beta,op} =
// sum_alpha c L_k[alpha] (a single channel when there is one source: no copy);
// likewise right factors Y_{beta,op}.  Sigma is then
//   T_X = X psi                       (phase A, one GEMM per factor and psi slab)
//   sigma = sum_terms c (op_l (x) op_r) T_X Y^T   (phase B, long-K GEMM per block)
// and the left (right) environment update reuses the same factors with the site
// tensor in place of psi.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstring>
#include <limits>
#include <thread>

#include "solver.hpp"

// smallest split-K chunk, in MFMA k-steps of one 32x32 tile
#ifndef DMRG_SPLIT_MIN
#define DMRG_SPLIT_MIN 256.0
#endif

namespace dmrg {

namespace {
// Host threads for plan building (the box's share of cores; at least 1).
int plan_threads() {
  static const int n = [] {
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, h ? h : 1u));
  }();
  return n;
}
// f(t, begin, end) on contiguous ranges of [0, n), one per thread, at least
// `grain` elements each (starting threads costs tens of microseconds, so light
// per-element work takes a large grain); the ranges follow thread order, so
// results gathered by thread index are in serial order.
template <class F>
void parallel_ranges(long n, F&& f, long grain = 4) {
  const int nt = (int)std::min<long>(plan_threads(), std::max<long>(n / grain, 1));
  if (nt <= 1) {
    f(0, 0L, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    const long b = n * t / nt, e = n * (t + 1) / nt;
    th.emplace_back([&f, t, b, e] { f(t, b, e); });
  }
  for (auto& x : th) x.join();
}
}  // namespace

// Grain of loops over a phase's units: about 4096 items per thread.
template <class PH>
long unit_grain(const PH& ph) {
  const long nu = (long)ph.units.size(), ni = (long)ph.items.size();
  return std::max<long>(4, ni > 0 ? nu * 4096 / ni : nu);
}

bool same_sectors(const std::vector<Sector>& a, const std::vector<Sector>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].q != b[i].q || a[i].dim != b[i].dim) return false;
  return true;
}

size_t Solver::workspace_estimate() const {
  // environment size of one cut from its bond and the MPO channels (as make_env_layout lays it out)
  auto env_size = [&](int cut) {
    const auto& ch = prob_->mpo.chans[cut];
    std::vector<QN> dqs;
    std::vector<long> count;
    for (const auto& c : ch) {
      int j = -1;
      for (size_t x = 0; x < dqs.size(); ++x)
        if (dqs[x] == c.dq) j = (int)x;
      if (j < 0) {
        dqs.push_back(c.dq);
        count.push_back(0);
        j = (int)dqs.size() - 1;
      }
      count[j]++;
    }
    std::vector<EnvClass> cls = make_env_classes(bonds_[cut], dqs);
    long n = 0;
    for (size_t j = 0; j < cls.size(); ++j) n += cls[j].nnz * count[j];
    return n;
  };
  long env_total = 0, env_max = 0, psi_max = 0, mps = 0;
  for (int c = 0; c <= L_; ++c) {
    const long e = env_size(c);
    env_total += 2 * e;  // left and right environments may both be kept at a cut
    env_max = std::max(env_max, e);
  }
  for (int k = 0; k + 1 < L_; ++k)
    psi_max = std::max(psi_max, make_tensor_layout(bonds_[k], bonds_[k + 2], twosite_phys_qn()).size);
  for (int k = 0; k < L_; ++k) mps += make_tensor_layout(bonds_[k], bonds_[k + 1], site_phys_qn()).size;
  const long kmax = std::min(opt_.max_subspace, 64);
  long dmax = 0;
  for (int c = 0; c <= L_; ++c) dmax = std::max<long>(dmax, prob_->mpo.dim(c));
  // sigma intermediates: T (one block row per left factor and psi slab) grows as
  // (MPO dimension) x |psi| (measured 2.2-2.4 times that product at CAS(12..20)
  // half sweeps) but is held one chunk at a time (with its low-precision copy);
  // the merged right blocks stay below (MPO dimension) x |psi|; premixed
  // factors and split-K partials as a few environments; Davidson: basis,
  // products and per-root work vectors
  long sig = 3 * dmax * psi_max;
  if (opt_.sigma_chunk_bytes > 0)
    sig = std::min<long>(sig, 2 * (opt_.sigma_chunk_bytes / (long)sizeof(double)) + dmax * psi_max);
  const long doubles = env_total + 12 * env_max + sig + (2 * kmax + 16 + 4 * opt_.n_states) * psi_max + 4 * mps;
  // half again as much for fragmentation: grow-only buffers are released and
  // re-carved as the bonds grow along a sweep
  return (size_t)doubles * 12 + (size_t(256) << 20);
}

void Solver::make_env_layout(Env& e, int cut, const Bond& b) {
  const auto& ch = prob_->mpo.chans[cut];
  std::vector<QN> dqs;
  e.chan_class.assign(ch.size(), -1);
  e.chan_slot.assign(ch.size(), -1);
  std::vector<int> count;
  for (size_t i = 0; i < ch.size(); ++i) {
    int c = -1;
    for (size_t j = 0; j < dqs.size(); ++j)
      if (dqs[j] == ch[i].dq) c = (int)j;
    if (c < 0) {
      c = (int)dqs.size();
      dqs.push_back(ch[i].dq);
      count.push_back(0);
    }
    e.chan_class[i] = c;
    e.chan_slot[i] = count[c]++;
  }
  e.classes = make_env_classes(b, dqs);
  e.class_base.assign(dqs.size(), 0);
  long off = 0;
  for (size_t c = 0; c < dqs.size(); ++c) {
    e.class_base[c] = off;
    off += e.classes[c].nnz * count[c];
  }
  e.size = off;
  e.buf.reserve(std::max<long>(off, 1) * sizeof(double));
}

void Solver::build_factor_side(FactorSide& fs, bool left, int site) {
  const MPO& mpo = prob_->mpo;
  const Env& env = left ? left_[site] : right_[site + 1];
  int mid_cut = left ? site + 1 : site;
  fs = FactorSide();
  fs.left = left;
  fs.mix = left ? &lmix_ : &rmix_;
  fs.cut = left ? site : site + 1;
  fs.by_mid.assign(mpo.chans[mid_cut].size(), {});
  // group W entries by (middle channel, op)
  std::map<std::pair<int, int>, std::vector<std::pair<int, double>>> groups;
  for (const auto& e : mpo.W[site]) {
    if (e.c == 0.0) continue;  // kept in the MPO only for its gradient
    int mid = left ? e.b : e.a;
    int src = left ? e.a : e.b;
    groups[{mid, e.op}].push_back({src, e.c});
  }
  std::map<int, int> alias_of;
  std::map<std::vector<std::pair<int, double>>, int> mixed_of;
  std::vector<std::vector<std::pair<int, double>>> mixed_src;
  for (auto& g : groups) {
    auto& src = g.second;
    std::sort(src.begin(), src.end());
    int f;
    double scale;
    if (src.size() == 1) {
      auto it = alias_of.find(src[0].first);
      if (it == alias_of.end()) {
        f = (int)fs.fac.size();
        int ch = src[0].first;
        fs.fac.push_back({env.chan_class[ch], true, env.chan_off(ch)});
        alias_of[ch] = f;
      } else {
        f = it->second;
      }
      scale = src[0].second;
    } else {
      scale = src[0].second;
      std::vector<std::pair<int, double>> norm;
      for (auto& s : src) norm.push_back({s.first, s.second / scale});
      auto it = mixed_of.find(norm);
      if (it == mixed_of.end()) {
        f = (int)fs.fac.size();
        fs.fac.push_back({env.chan_class[src[0].first], false, -1});
        mixed_of[norm] = f;
        mixed_src.push_back(norm);
      } else {
        f = it->second;
      }
    }
    fs.by_mid[g.first.first].push_back({g.first.second, f, scale});
  }
  // premix program, outputs grouped by class (one kernel launch per class)
  std::vector<int> mixed_ids;
  for (size_t f = 0; f < fs.fac.size(); ++f)
    if (!fs.fac[f].alias) mixed_ids.push_back((int)f);
  std::stable_sort(mixed_ids.begin(), mixed_ids.end(),
                   [&](int a, int b) { return fs.fac[a].cls < fs.fac[b].cls; });
  std::map<int, int> mix_index;  // factor -> index into mixed_src
  {
    int i = 0;
    for (size_t f = 0; f < fs.fac.size(); ++f)
      if (!fs.fac[f].alias) mix_index[(int)f] = i++;
  }
  long off = 0;
  fs.ptr.push_back(0);
  for (int f : mixed_ids) {
    const auto& src = mixed_src[mix_index[f]];
    long nnz = env.classes[fs.fac[f].cls].nnz;
    fs.fac[f].off = off;
    fs.out_off.push_back(off);
    fs.out_nnz.push_back(nnz);
    off += nnz;
    for (auto& s : src) {
      DMRG_REQUIRE(env.chan_class[s.first] == fs.fac[f].cls, ST_EINVAL, "premix sources of different classes");
      fs.src_off.push_back(env.chan_off(s.first));
      fs.coef.push_back(s.second);
    }
    fs.ptr.push_back((int)fs.coef.size());
  }
  fs.premix_size = off;
}

void Solver::run_premix(FactorSide& fs, const Env& env) {
  int n_out = (int)fs.out_off.size();
  if (n_out == 0) return;
  fs.mix->reserve(std::max<long>(fs.premix_size, 1) * sizeof(double));
  std::vector<const double*>& srcs = fs.h_srcs;
  srcs.resize(fs.src_off.size());
  for (size_t i = 0; i < srcs.size(); ++i) srcs[i] = env.buf.as<double>() + fs.src_off[i];
  fs.d_srcs.reserve(srcs.size() * sizeof(void*) + 8);
  fs.d_ptr.reserve(fs.ptr.size() * sizeof(int) + 8);
  fs.d_coef.reserve(fs.coef.size() * sizeof(double) + 8);
  hip_check(hipMemcpyAsync(fs.d_srcs.p, srcs.data(), srcs.size() * sizeof(void*), hipMemcpyHostToDevice, st), "premix srcs");
  hip_check(hipMemcpyAsync(fs.d_ptr.p, fs.ptr.data(), fs.ptr.size() * sizeof(int), hipMemcpyHostToDevice, st), "premix ptr");
  hip_check(hipMemcpyAsync(fs.d_coef.p, fs.coef.data(), fs.coef.size() * sizeof(double), hipMemcpyHostToDevice, st), "premix coef");
  // launch per run of equal nnz (outputs of one class are contiguous)
  int b = 0;
  while (b < n_out) {
    int e = b + 1;
    while (e < n_out && fs.out_nnz[e] == fs.out_nnz[b] && fs.out_off[e] == fs.out_off[e - 1] + fs.out_nnz[e - 1]) ++e;
    launch_premix(fs.mix->as<double>() + fs.out_off[b], fs.d_srcs.as<const double*>(), fs.d_ptr.as<int>() + b,
                  fs.d_coef.as<double>(), e - b, fs.out_nnz[b], st);
    b = e;
  }
}

void Solver::run_pairmix(int k) {
  const int ng = (int)pm_.out_off.size();
  if (ng == 0) return;
  pm_.mix = &pmix_;
  pm_.mix->reserve(std::max<long>(pm_.size, 1) * sizeof(double));
  std::vector<const double*>& srcs = pm_.h_srcs;
  srcs.resize(pm_.src_off.size());
  for (size_t i = 0; i < srcs.size(); ++i) {
    const double* base = pm_.src_buf[i] == B_YMIX ? rf_.mix->as<double>() : right_[k + 2].buf.as<double>();
    srcs[i] = base + pm_.src_off[i];
  }
  pm_.d_srcs.reserve(srcs.size() * sizeof(void*) + 8);
  pm_.d_ptr.reserve(pm_.ptr.size() * sizeof(int) + 8);
  pm_.d_coef.reserve(pm_.coef.size() * sizeof(double) + 8);
  pm_.d_out_off.reserve(pm_.out_off.size() * sizeof(long) + 8);
  pm_.d_nnz.reserve(pm_.nnz.size() * sizeof(int) + 8);
  hip_check(hipMemcpyAsync(pm_.d_srcs.p, srcs.data(), srcs.size() * sizeof(void*), hipMemcpyHostToDevice, st), "pairmix srcs");
  hip_check(hipMemcpyAsync(pm_.d_ptr.p, pm_.ptr.data(), pm_.ptr.size() * sizeof(int), hipMemcpyHostToDevice, st), "pairmix ptr");
  hip_check(hipMemcpyAsync(pm_.d_coef.p, pm_.coef.data(), pm_.coef.size() * sizeof(double), hipMemcpyHostToDevice, st),
            "pairmix coef");
  hip_check(hipMemcpyAsync(pm_.d_out_off.p, pm_.out_off.data(), pm_.out_off.size() * sizeof(long), hipMemcpyHostToDevice, st),
            "pairmix out");
  hip_check(hipMemcpyAsync(pm_.d_nnz.p, pm_.nnz.data(), pm_.nnz.size() * sizeof(int), hipMemcpyHostToDevice, st), "pairmix nnz");
  launch_pairmix(pm_.mix->as<double>(), pm_.d_srcs.as<const double*>(), pm_.d_ptr.as<int>(), pm_.d_coef.as<double>(),
                 pm_.d_out_off.as<long>(), pm_.d_nnz.as<int>(), ng, st);
}

// One logical unit per output block; tiles are cut when the plan is resolved
// (the tile shape depends on the kernel chosen for the precision).
static void add_units(std::vector<PUnit>& units, int cbuf, long coff, int ldc, int M, int N, int ib,
                      int ie, int acc) {
  units.push_back({cbuf, coff, ldc, M, N, 0, 0, ib, ie, acc});
}

// Host check that every tile of every item stays inside its buffer (in
// elements); a plan bug becomes an error instead of a device fault.
// Also returns whether every item fits the buffer-load kernels (buffer_reach_ok).
static bool validate_phase(const Phase& ph, const long* sizes, const size_t* esz) {
  std::vector<char> bad(plan_threads(), 0), reach(plan_threads(), 1);
  parallel_ranges((long)ph.units.size(), [&](int t, long u0, long u1) {
    for (long ui = u0; ui < u1 && !bad[t]; ++ui) {
      const PUnit& u = ph.units[ui];
      long cmax = u.coff + (long)(u.M - 1) * u.ldc + (u.N - 1);
      if (u.coff < 0 || cmax >= sizes[u.cbuf]) bad[t] = 1;
      for (int i = u.ib; i < u.ie && !bad[t]; ++i) {
        const PItem& it = ph.items[i];
        long amax, bmax;
        if (ph.mode == GEMM_TN) amax = it.aoff + (long)(it.K - 1) * it.lda + (u.M - 1);
        else amax = it.aoff + (long)(u.M - 1) * it.lda + (it.K - 1);
        if (ph.mode == GEMM_NT) bmax = it.boff + (long)(u.N - 1) * it.ldb + (it.K - 1);
        else bmax = it.boff + (long)(it.K - 1) * it.ldb + (u.N - 1);
        if (it.K <= 0 || it.aoff < 0 || it.boff < 0 || amax >= sizes[it.abuf] || bmax >= sizes[it.bbuf]) bad[t] = 2;
        if (reach[t] && !buffer_reach_ok(ph.mode, u.M, u.N, it.K, it.lda, it.ldb, esz[it.abuf], esz[it.bbuf]))
          reach[t] = 0;
      }
    }
  }, unit_grain(ph));
  for (char b : bad) {
    if (b == 1) throw Error(ST_EINVAL, "plan: output block out of bounds");
    if (b == 2) throw Error(ST_EINVAL, "plan: operand block out of bounds");
  }
  bool ok = true;
  for (char r : reach) ok = ok && r;
  return ok;
}

void Solver::run_phase(Phase& ph, int prec, void* const* bases, size_t const* esz, const long* sizes) {
  if (ph.units.empty()) return;
  int slot = prec == PREC_F64 ? 0 : (prec == PREC_F32 ? 1 : 2);
  bool same = ph.uploaded[slot] && (ph.n_tiles[slot] == 0 || ph.slot_base[slot] == splitk_.p);
  for (int b = 0; b < B_NBUF && same; ++b) same = ph.last_bases[slot][b] == bases[b];
  if (same) {  // plan already resolved against these buffers
    launch_resolved(ph, prec, slot);
    return;
  }
  const auto tr0 = std::chrono::steady_clock::now();
  if (opt_.verbose > 2) {
    std::string moved;
    for (int b = 0; b < B_NBUF; ++b)
      if (ph.uploaded[slot] && ph.last_bases[slot][b] != bases[b]) moved += " " + std::to_string(b);
    fprintf(stderr, "resolve: mode %d, %zu items, %s%s\n", ph.mode, ph.items.size(),
            ph.uploaded[slot] ? "moved buffers" : "first use", moved.c_str());
  }
  const bool buf_ok = validate_phase(ph, sizes, esz);
  for (int b = 0; b < B_NBUF; ++b) ph.last_bases[slot][b] = bases[b];
  ph.uploaded[slot] = true;
  // the tables are written into pinned staging buffers that every resolve of
  // the solver reuses (no page faults, DMA uploads); the last upload from them
  // must have finished (it precedes, in stream order, the kernels launched since)
  if (stage_pending_) hip_check(hipEventSynchronize(stage_ev_), "staging");
  const long n_items = (long)ph.items.size();
  GemmItem* items = stage_items_.get<GemmItem>(n_items);
  parallel_ranges(n_items, [&](int, long i0, long i1) {
    for (long i = i0; i < i1; ++i) {
      const PItem& p = ph.items[i];
      items[i].A = (const char*)bases[p.abuf] + p.aoff * esz[p.abuf];
      items[i].B = (const char*)bases[p.bbuf] + p.boff * esz[p.bbuf];
      items[i].lda = p.lda;
      items[i].ldb = p.ldb;
      items[i].K = p.K;
      items[i].pad = 0;
      items[i].coef = p.coef;
    }
  }, 4096);
  ph.buf_ok[slot] = buf_ok;
  // fp64 / fp32 NT phases with long item lists (sigma phase B) take the
  // workgroup block kernel: whole-block tiles up to 96 x 64, operands read once
  // per block
  const bool use_wg = ph.wg && (prec == PREC_F64 || prec == PREC_F32) && ph.mode == GEMM_NT && buf_ok;
  ph.wg_used[slot] = use_wg;
  GemmUnit* units = nullptr;
  SplitTile* tiles = nullptr;
  long nun = 0, ntl = 0;
  long n_slot_elems = 0;
  if (prec == PREC_F64 || prec == PREC_F32 || prec == PREC_BF16 || prec == 3) {
    // One-wave tiles of (16 RB) x (16 CB), RB <= 4, CB <= 2: block rows are cut
    // into strips of 64 while more than 64 remain, columns into strips of 32, and
    // the last strip is rounded up to a multiple of 16 (MFMA blocks are 16 x 16).
    // Long item lists are cut into chunks of about `chunk` MFMA k-steps, each
    // writing a partial tile that splitk_reduce sums in order.
    auto strips = [](int n, int wmax, std::vector<std::pair<int, int>>& v) {
      v.clear();
      int x = 0;
      while (n - x > wmax) {
        v.push_back({x, wmax});
        x += wmax;
      }
      if (x < n) v.push_back({x, (n - x + 15) / 16 * 16});
    };
    struct TileShape { int m0, n0, tm, tn, shape; };
    // one-wave tiles: up to 64 x 32; workgroup block tiles: up to 96 x 64
    const int wm = use_wg ? 96 : 64, wn = use_wg ? 64 : 32;
    auto tiles_of = [&](const PUnit& u, std::vector<TileShape>& ts) {
      std::vector<std::pair<int, int>> rs, cs;
      strips(u.M, wm, rs);
      strips(u.N, wn, cs);
      ts.clear();
      for (auto& r : rs)
        for (auto& c : cs) ts.push_back({r.first, c.first, r.second, c.second, 8 * (r.second / 16) + c.second / 16});
    };
    // work in MFMA k-steps of 32 x 32 tiles (integers: the same sum in any order)
    const long nu = (long)ph.units.size();
    std::vector<long> wunit(nu, 0);
    parallel_ranges(nu, [&](int, long u0, long u1) {
      for (long x = u0; x < u1; ++x) {
        const PUnit& u = ph.units[x];
        long w = 0;
        for (int i = u.ib; i < u.ie; ++i) w += (long)((u.M + 31) / 32) * ((u.N + 31) / 32) * ((ph.items[i].K + 3) / 4);
        wunit[x] = w;
      }
    }, unit_grain(ph));
    double work = 0;
    {
      long wsum = 0;
      for (long w : wunit) wsum += w;
      work = (double)wsum;
    }
    if (ph.split_work > 0) work = ph.split_work;
    // about 16384 one-wave units; workgroup units are cut finer (65536, measured
    // best for sigma phase B at CAS(20,20), M = 1024: smaller pieces of the
    // largest blocks spread over more CUs, against more split-K partial tiles)
    const double chunk = std::max(DMRG_SPLIT_MIN, work / (use_wg ? 65536.0 : 16384.0));
    // pass 1 (parallel over blocks): tiles and item chunks of each block, counts
    struct UnitPlan {
      std::vector<TileShape> ts;
      std::vector<std::pair<int, int>> cuts;  // empty: no split
      long n_units = 0, n_tiles = 0, n_slot = 0;
    };
    std::vector<UnitPlan> up(nu);
    std::vector<char> too_big(plan_threads(), 0);
    parallel_ranges(nu, [&](int t, long u0, long u1) {
      for (long x = u0; x < u1; ++x) {
        const PUnit& u = ph.units[x];
        UnitPlan& q = up[x];
        tiles_of(u, q.ts);
        long w = 0;
        for (int i = u.ib; i < u.ie; ++i) w += (ph.items[i].K + 3) / 4;
        if ((double)w <= chunk || u.ie - u.ib <= 1) {
          q.n_units = (long)q.ts.size();
          continue;
        }
        // the same item chunks for every tile of the block; units chunk-major, so the
        // waves of one workgroup run one chunk on neighbouring tiles (shared rows of A
        // or columns of B)
        for (int b = u.ib; b < u.ie;) {
          int e = b;
          double cw = 0;
          while (e < u.ie && (cw < chunk || e == b)) cw += (ph.items[e++].K + 3) / 4;
          q.cuts.push_back({b, e});
          b = e;
        }
        const long nc = (long)q.cuts.size();
        q.n_units = nc * (long)q.ts.size();
        q.n_tiles = (long)q.ts.size();
        for (const TileShape& ts : q.ts) {
          // the reduction covers tiles of up to 96 x 64 elements
          if (ts.tm * ts.tn > 96 * 64) too_big[t] = 1;
          q.n_slot += nc * ts.tm * ts.tn;
        }
      }
    }, unit_grain(ph));
    for (char b : too_big) DMRG_REQUIRE(!b, ST_EINVAL, "split-K tile larger than the reduction covers");
    // offsets, then pass 2 (parallel): units, tiles and slot offsets in place
    std::vector<long> uat(nu), tat(nu), sat(nu);
    for (long x = 0; x < nu; ++x) {
      uat[x] = nun;
      tat[x] = ntl;
      sat[x] = n_slot_elems;
      nun += up[x].n_units;
      ntl += up[x].n_tiles;
      n_slot_elems += up[x].n_slot;
    }
    units = stage_units_.get<GemmUnit>(nun);
    tiles = stage_tiles_.get<SplitTile>(ntl);
    // grow-only: a move invalidates other resolved plans, which re-resolve (slot_base)
    const size_t slot_esz = prec == PREC_F64 ? sizeof(double) : sizeof(float);
    if (n_slot_elems > 0) splitk_.reserve(n_slot_elems * slot_esz);
    char* const slot0 = (char*)splitk_.p;
    parallel_ranges(nu, [&](int, long u0, long u1) {
      for (long x = u0; x < u1; ++x) {
        const PUnit& u = ph.units[x];
        const UnitPlan& q = up[x];
        char* C = (char*)bases[u.cbuf] + u.coff * esz[u.cbuf];
        GemmUnit* uo = units + uat[x];
        if (q.cuts.empty()) {
          for (const TileShape& t : q.ts) *uo++ = {C, u.ldc, u.M, u.N, t.m0, t.n0, u.ib, u.ie, u.acc, t.shape};
          continue;
        }
        const int nc = (int)q.cuts.size();
        long so = sat[x];
        SplitTile* to = tiles + tat[x];
        for (size_t t = 0; t < q.ts.size(); ++t) {
          const TileShape& ts = q.ts[t];
          to[t] = {C, so, u.ldc, u.M, u.N, ts.m0, ts.n0, nc, ts.tm, ts.tn, u.acc, 0};
          so += (long)nc * ts.tm * ts.tn;
        }
        for (int c = 0; c < nc; ++c)
          for (size_t t = 0; t < q.ts.size(); ++t) {
            const SplitTile& st_ = to[t];
            *uo++ = {slot0 + (st_.s0 + (long)c * st_.tm * st_.tn) * (long)slot_esz, st_.tn, u.M, u.N, st_.m0, st_.n0,
                     q.cuts[c].first, q.cuts[c].second, 2, q.ts[t].shape};
          }
      }
    }, unit_grain(ph));
    ph.slot_base[slot] = splitk_.p;
  } else {
    std::vector<GemmUnit> v;
    for (const PUnit& u : ph.units) {
      char* C = (char*)bases[u.cbuf] + u.coff * esz[u.cbuf];
      for (int m0 = 0; m0 < u.M; m0 += 64)
        for (int n0 = 0; n0 < u.N; n0 += 64) v.push_back({C, u.ldc, u.M, u.N, m0, n0, u.ib, u.ie, u.acc});
    }
    nun = (long)v.size();
    units = stage_units_.get<GemmUnit>(nun);
    std::copy(v.begin(), v.end(), units);
  }
  ph.n_units[slot] = (int)nun;
  ph.n_tiles[slot] = (int)ntl;
  const auto tr1 = std::chrono::steady_clock::now();
  ph.d_items[slot].reserve(n_items * sizeof(GemmItem) + 64);
  ph.d_units[slot].reserve(nun * sizeof(GemmUnit) + 64);
  ph.d_tiles[slot].reserve(ntl * sizeof(SplitTile) + 64);
  hip_check(hipMemcpyAsync(ph.d_items[slot].p, items, n_items * sizeof(GemmItem), hipMemcpyHostToDevice, st), "items");
  hip_check(hipMemcpyAsync(ph.d_units[slot].p, units, nun * sizeof(GemmUnit), hipMemcpyHostToDevice, st), "units");
  if (ntl > 0)
    hip_check(hipMemcpyAsync(ph.d_tiles[slot].p, tiles, ntl * sizeof(SplitTile), hipMemcpyHostToDevice, st), "tiles");
  if (!stage_ev_) hip_check(hipEventCreateWithFlags(&stage_ev_, hipEventDisableTiming), "staging event");
  hip_check(hipEventRecord(stage_ev_, st), "staging event");
  stage_pending_ = true;
  const auto tr2 = std::chrono::steady_clock::now();
  st_.resolve_ms += std::chrono::duration<double, std::milli>(tr2 - tr0).count();
  if (opt_.verbose > 1)
    fprintf(stderr, "resolve: %ld items, %ld units: host %.2f ms, upload %.2f ms\n", n_items, nun,
            std::chrono::duration<double, std::milli>(tr1 - tr0).count(),
            std::chrono::duration<double, std::milli>(tr2 - tr1).count());
  launch_resolved(ph, prec, slot);
}

void Solver::launch_resolved(Phase& ph, int prec, int slot) {
  if (prec == PREC_F64) {
    if (ph.wg_used[slot])
      launch_gemm_wg(PREC_F64, ph.tag, ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot], ph.d_items[slot].as<GemmItem>(), st);
    else
      launch_gemm_w32(ph.mode, ph.tag, ph.buf_ok[slot], ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot],
                      ph.d_items[slot].as<GemmItem>(), st);
    if (ph.gemm_done) (void)hipEventRecord(ph.gemm_done, st);  // GEMM-only timing
    launch_splitk_reduce(ph.d_tiles[slot].as<SplitTile>(), ph.n_tiles[slot], splitk_.as<double>(), st);
  } else if (prec == PREC_F32 && ph.wg_used[slot]) {
    launch_gemm_wg(PREC_F32, 0, ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot], ph.d_items[slot].as<GemmItem>(), st);
    launch_splitk_reduce_f32(ph.d_tiles[slot].as<SplitTile>(), ph.n_tiles[slot], splitk_.as<float>(), st);
  } else if (prec == PREC_F32) {
    launch_gemm_w32_f32(ph.mode, ph.buf_ok[slot], ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot], ph.d_items[slot].as<GemmItem>(), st);
    launch_splitk_reduce_f32(ph.d_tiles[slot].as<SplitTile>(), ph.n_tiles[slot], splitk_.as<float>(), st);
  } else if (prec == PREC_BF16 || prec == 3) {
    launch_gemm_w32_bf16(ph.mode, prec == 3, ph.buf_ok[slot], ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot],
                         ph.d_items[slot].as<GemmItem>(), st);
    launch_splitk_reduce_f32(ph.d_tiles[slot].as<SplitTile>(), ph.n_tiles[slot], splitk_.as<float>(), st);
  } else {
    launch_gemm(prec, ph.mode, ph.d_units[slot].as<GemmUnit>(), ph.n_units[slot], ph.d_items[slot].as<GemmItem>(), st);
  }
}

// L_{k+1}[beta] = sum_{(op,X)} s sum_{ss'} op[s][s'] A_s^T X A_{s'}
void Solver::env_update_left(int k, const FactorSide& fs) {
  const MPO& mpo = prob_->mpo;
  const Bond& bk = bonds_[k];
  const Env& envk = left_[k];
  const SiteTensor& A = mps_[k];
  Env& out = left_[k + 1];
  const auto te0 = std::chrono::steady_clock::now();
  make_env_layout(out, k + 1, bonds_[k + 1]);
  const auto te1 = std::chrono::steady_clock::now();
  // the plan depends on bonds k, k+1 and the MPO only: reuse it while they hold
  EnvPlan& ep = env_plans_[{k, 0}];
  const bool hit = same_sectors(ep.key_a, bonds_[k].sec) && same_sectors(ep.key_b, bonds_[k + 1].sec);
  if (!hit) {
  ep.pa = Phase();
  ep.pb = Phase();
  Phase& pa = ep.pa;
  Phase& pb = ep.pb;
  // phase A: Z_X = X A for every factor used
  std::vector<char> used(fs.fac.size(), 0);
  for (auto& v : fs.by_mid)
    for (auto& u : v) used[u.f] = 1;
  pa.mode = GEMM_NN;
  std::vector<std::vector<long>> zoff(fs.fac.size());  // per factor, per A slab: offset or -1
  long zsize = 0;
  for (size_t f = 0; f < fs.fac.size(); ++f) {
    if (!used[f]) continue;
    const EnvClass& cls = envk.classes[fs.fac[f].cls];
    zoff[f].assign(A.lay.slabs.size(), -1);
    for (size_t si = 0; si < A.lay.slabs.size(); ++si) {
      const Slab& sl = A.lay.slabs[si];
      int bi = cls.block_of_col[sl.li];
      if (bi < 0) continue;
      const EnvBlock& eb = cls.blocks[bi];
      zoff[f][si] = zsize;
      int ib = (int)pa.items.size();
      pa.items.push_back({fs.fac[f].alias ? B_ENVL : B_XMIX, fs.fac[f].off + eb.off, B_PSI, sl.off,
                          eb.mc, sl.width, eb.mc, 1.0});
      add_units(pa.units, B_T, zsize, sl.width, eb.mr, sl.width, ib, ib + 1, 0);
      pa.flops += 2.0 * eb.mr * eb.mc * sl.width;
      zsize += (long)eb.mr * sl.width;
    }
  }
  // phase B
  pb.mode = GEMM_TN;
  const auto& mids = mpo.chans[k + 1];
  for (size_t beta = 0; beta < mids.size(); ++beta) {
    const EnvClass& ocls = out.classes[out.chan_class[beta]];
    long cbase = out.chan_off((int)beta);
    std::vector<std::vector<PItem>> per_block(ocls.blocks.size());
    for (const auto& u : fs.by_mid[beta]) {
      const Mat4& op = mpo.ops[u.op];
      const EnvClass& icls = envk.classes[fs.fac[u.f].cls];
      for (int s = 0; s < 4; ++s)
        for (int sp = 0; sp < 4; ++sp) {
          double w = op[s * 4 + sp];
          if (w == 0.0) continue;
          for (size_t si = 0; si < A.lay.slabs.size(); ++si) {
            if (zoff[u.f][si] < 0) continue;
            const Slab& sl = A.lay.slabs[si];
            int bi = icls.block_of_col[sl.li];
            int lo = icls.blocks[bi].ri;  // row sector of X A
            int slo = A.lay.slab_of_left[lo];
            if (slo < 0) continue;
            const Slab& slab_lo = A.lay.slabs[slo];
            // block (s', ri) of the source slab gives Z columns
            for (const auto& blk : sl.blocks) {
              if (blk.phys != sp) continue;
              int ri = blk.ri;
              int ob = ocls.block_of_col[ri];
              if (ob < 0) continue;
              int ro = ocls.blocks[ob].ri;
              int ab = slab_lo.block_of(s, ro);
              if (ab < 0) continue;
              const SlabBlock& ablk = slab_lo.blocks[ab];
              per_block[ob].push_back({B_PSI, slab_lo.off + ablk.col0, B_T, zoff[u.f][si] + blk.col0,
                                       slab_lo.width, sl.width, slab_lo.ml, u.scale * w});
              pb.flops += 2.0 * ablk.mr * blk.mr * slab_lo.ml;
            }
          }
        }
    }
    for (size_t ob = 0; ob < per_block.size(); ++ob) {
      if (per_block[ob].empty()) continue;
      int ib = (int)pb.items.size();
      pb.items.insert(pb.items.end(), per_block[ob].begin(), per_block[ob].end());
      const EnvBlock& eb = ocls.blocks[ob];
      add_units(pb.units, B_OUT, cbase + eb.off, eb.mc, eb.mr, eb.mc, ib, (int)pb.items.size(), 0);
    }
  }
  ep.zsize = zsize;
  ep.key_a = bonds_[k].sec;
  ep.key_b = bonds_[k + 1].sec;
  }
  Phase& pa = ep.pa;
  Phase& pb = ep.pb;
  const long zsize = ep.zsize;
  env_t_buf_.reserve(std::max<long>(zsize, 1) * sizeof(double));
  launch_fill(out.buf.as<double>(), out.size, 0.0, st);
  void* bases[B_NBUF] = {};
  bases[B_PSI] = A.buf.p;
  bases[B_OUT] = out.buf.p;
  bases[B_T] = env_t_buf_.p;
  bases[B_XMIX] = fs.mix->p;
  bases[B_ENVL] = envk.buf.p;
  size_t esz[B_NBUF] = {8, 8, 8, 8, 8, 8, 8, 8, 8};
  long sizes[B_NBUF] = {};
  sizes[B_PSI] = A.lay.size;
  sizes[B_OUT] = out.size;
  sizes[B_T] = zsize;
  sizes[B_XMIX] = fs.premix_size;
  sizes[B_ENVL] = envk.size;
  const auto te2 = std::chrono::steady_clock::now();
  st_.env_plan_ms += std::chrono::duration<double, std::milli>(te2 - te1).count();
  run_phase(pa, PREC_F64, bases, esz, sizes);
  run_phase(pb, PREC_F64, bases, esz, sizes);
  const auto te3 = std::chrono::steady_clock::now();
  st_.env_flops += pa.flops + pb.flops;
  hip_check(hipStreamSynchronize(st), "env update");
  out.valid = true;
  if (opt_.verbose > 2) {
    auto ms = [](std::chrono::steady_clock::time_point x, std::chrono::steady_clock::time_point y) {
      return std::chrono::duration<double, std::milli>(y - x).count();
    };
    fprintf(stderr, "env left k=%d: layout %.2f ms, plan %.2f ms (%s), launch %.2f ms, GPU wait %.2f ms\n", k,
            ms(te0, te1), ms(te1, te2), hit ? "cached" : "built", ms(te2, te3),
            ms(te3, std::chrono::steady_clock::now()));
  }
}

// R_j[beta] = sum_{(op,Y)} s sum_{ss'} op[s][s'] B_s Y B_{s'}^T
void Solver::env_update_right(int j, const FactorSide& fs) {
  const MPO& mpo = prob_->mpo;
  const Bond& bj1 = bonds_[j + 1];
  const Env& envr = right_[j + 1];
  const SiteTensor& Bt = mps_[j];
  Env& out = right_[j];
  const auto te0 = std::chrono::steady_clock::now();
  make_env_layout(out, j, bonds_[j]);
  const auto te1 = std::chrono::steady_clock::now();
  EnvPlan& ep = env_plans_[{j, 1}];
  const bool hit = same_sectors(ep.key_a, bonds_[j].sec) && same_sectors(ep.key_b, bonds_[j + 1].sec);
  if (!hit) {
  ep.pa = Phase();
  ep.pb = Phase();
  Phase& pa = ep.pa;
  Phase& pb = ep.pb;
  std::vector<char> used(fs.fac.size(), 0);
  for (auto& v : fs.by_mid)
    for (auto& u : v) used[u.f] = 1;
  // phase A: U_Y = B Y, stored per (factor, slab) as a slab of blocks (s, c)
  struct USlab {
    long off = -1;
    int width = 0;
    std::vector<std::array<int, 3>> blocks;  // s, c (bond j+1 sector), col0
  };
  std::vector<std::vector<USlab>> U(fs.fac.size());
  pa.mode = GEMM_NN;
  long usize = 0;
  for (size_t f = 0; f < fs.fac.size(); ++f) {
    if (!used[f]) continue;
    const EnvClass& cls = envr.classes[fs.fac[f].cls];
    U[f].resize(Bt.lay.slabs.size());
    for (size_t si = 0; si < Bt.lay.slabs.size(); ++si) {
      const Slab& sl = Bt.lay.slabs[si];
      USlab& us = U[f][si];
      for (const auto& blk : sl.blocks) {
        int c = bj1.find(bj1.sec[blk.ri].q - cls.dq);
        if (c < 0) continue;
        int ybi = cls.block_of_col[c];
        if (ybi < 0 || cls.blocks[ybi].ri != blk.ri) continue;
        us.blocks.push_back({blk.phys, c, us.width});
        us.width += bj1.sec[c].dim;
      }
      if (us.width == 0) continue;
      us.off = usize;
      for (const auto& ub : us.blocks) {
        const SlabBlock* blk = nullptr;
        for (const auto& b2 : sl.blocks)
          if (b2.phys == ub[0]) blk = &b2;  // one block per physical state in a slab
        const EnvBlock& yb = cls.blocks[cls.block_of_col[ub[1]]];
        int ib = (int)pa.items.size();
        pa.items.push_back({B_SITE2, sl.off + blk->col0, fs.fac[f].alias ? B_ENVR : B_YMIX,
                            fs.fac[f].off + yb.off, sl.width, yb.mc, blk->mr, 1.0});
        add_units(pa.units, B_T, usize + ub[2], us.width, sl.ml, yb.mc, ib, ib + 1, 0);
        pa.flops += 2.0 * sl.ml * blk->mr * yb.mc;
      }
      usize += (long)sl.ml * us.width;
    }
  }
  pb.mode = GEMM_NT;
  const Bond& bj = bonds_[j];
  const auto& mids = mpo.chans[j];
  for (size_t beta = 0; beta < mids.size(); ++beta) {
    const EnvClass& ocls = out.classes[out.chan_class[beta]];
    long cbase = out.chan_off((int)beta);
    std::vector<std::vector<PItem>> per_block(ocls.blocks.size());
    for (const auto& u : fs.by_mid[beta]) {
      const Mat4& op = mpo.ops[u.op];
      for (int s = 0; s < 4; ++s)
        for (int sp = 0; sp < 4; ++sp) {
          double w = op[s * 4 + sp];
          if (w == 0.0) continue;
          for (size_t si = 0; si < Bt.lay.slabs.size(); ++si) {
            const USlab& us = U[u.f][si];
            if (us.off < 0) continue;
            const Slab& sa = Bt.lay.slabs[si];
            for (const auto& ub : us.blocks) {
              if (ub[0] != s) continue;
              int c = ub[1];
              int lap = bj.find(bj1.sec[c].q - site_qn(sp));
              if (lap < 0) continue;
              int slp = Bt.lay.slab_of_left[lap];
              if (slp < 0) continue;
              const Slab& sb = Bt.lay.slabs[slp];
              int bb = sb.block_of(sp, c);
              if (bb < 0) continue;
              int ob = ocls.block_of_col[lap];
              if (ob < 0 || ocls.blocks[ob].ri != sa.li) continue;
              per_block[ob].push_back({B_T, us.off + ub[2], B_SITE2, sb.off + sb.blocks[bb].col0, us.width,
                                       sb.width, bj1.sec[c].dim, u.scale * w});
              pb.flops += 2.0 * sa.ml * sb.ml * bj1.sec[c].dim;
            }
          }
        }
    }
    for (size_t ob = 0; ob < per_block.size(); ++ob) {
      if (per_block[ob].empty()) continue;
      int ib = (int)pb.items.size();
      pb.items.insert(pb.items.end(), per_block[ob].begin(), per_block[ob].end());
      const EnvBlock& eb = ocls.blocks[ob];
      add_units(pb.units, B_OUT, cbase + eb.off, eb.mc, eb.mr, eb.mc, ib, (int)pb.items.size(), 0);
    }
  }
  ep.zsize = usize;
  ep.key_a = bonds_[j].sec;
  ep.key_b = bonds_[j + 1].sec;
  }
  Phase& pa = ep.pa;
  Phase& pb = ep.pb;
  const long usize = ep.zsize;
  env_t_buf_.reserve(std::max<long>(usize, 1) * sizeof(double));
  launch_fill(out.buf.as<double>(), out.size, 0.0, st);
  void* bases[B_NBUF] = {};
  bases[B_OUT] = out.buf.p;
  bases[B_T] = env_t_buf_.p;
  bases[B_YMIX] = fs.mix->p;
  bases[B_ENVR] = envr.buf.p;
  bases[B_SITE2] = Bt.buf.p;
  size_t esz[B_NBUF] = {8, 8, 8, 8, 8, 8, 8, 8, 8};
  long sizes[B_NBUF] = {};
  sizes[B_OUT] = out.size;
  sizes[B_T] = usize;
  sizes[B_YMIX] = fs.premix_size;
  sizes[B_ENVR] = envr.size;
  sizes[B_SITE2] = Bt.lay.size;
  const auto te2 = std::chrono::steady_clock::now();
  st_.env_plan_ms += std::chrono::duration<double, std::milli>(te2 - te1).count();
  run_phase(pa, PREC_F64, bases, esz, sizes);
  run_phase(pb, PREC_F64, bases, esz, sizes);
  const auto te3 = std::chrono::steady_clock::now();
  st_.env_flops += pa.flops + pb.flops;
  hip_check(hipStreamSynchronize(st), "env update");
  out.valid = true;
  if (opt_.verbose > 2) {
    auto ms = [](std::chrono::steady_clock::time_point x, std::chrono::steady_clock::time_point y) {
      return std::chrono::duration<double, std::milli>(y - x).count();
    };
    fprintf(stderr, "env right j=%d: layout %.2f ms, plan %.2f ms (%s), launch %.2f ms, GPU wait %.2f ms\n", j,
            ms(te0, te1), ms(te1, te2), hit ? "cached" : "built", ms(te2, te3),
            ms(te3, std::chrono::steady_clock::now()));
  }
}

void Solver::build_sigma_plan(int k) {
  using clk = std::chrono::steady_clock;
  const auto tp0 = clk::now();
  const MPO& mpo = prob_->mpo;
  const Env& envl = left_[k];
  const Env& envr = right_[k + 2];
  psi_lay_ = make_tensor_layout(bonds_[k], bonds_[k + 2], twosite_phys_qn());
  const TensorLayout& P = psi_lay_;
  const Bond& bk2 = bonds_[k + 2];
  int nmid = (int)mpo.chans[k + 1].size();
  // which left factors are used by terms
  std::vector<char> used(lf_.fac.size(), 0);
  for (int b = 0; b < nmid; ++b)
    if (!rf_.by_mid[b].empty())
      for (auto& u : lf_.by_mid[b]) used[u.f] = 1;
  // Left factors in chunks of at most sigma_chunk_bytes of T_X (0: one chunk; a
  // factor larger than the bound is a chunk of its own).  Phase A of a chunk
  // writes its T_X into one chunk-sized buffer and phase B of the chunk consumes
  // them at once, adding into sigma: the intermediates take one chunk of memory.
  // (Measured at CAS(20,20), M = 1024: 8.5 ms per sigma unchunked, 9.5 ms with
  // 1 GiB chunks, 13.8 ms with 128 MiB: the shorter launches cost more than the
  // memory-side cache saves.)
  const long chunk_cap = opt_.sigma_chunk_bytes > 0
                             ? std::max<long>(1, opt_.sigma_chunk_bytes / (long)sizeof(double))
                             : std::numeric_limits<long>::max();
  std::vector<int> chunk_of(lf_.fac.size(), -1);
  std::vector<std::vector<long>> toff(lf_.fac.size());
  std::vector<std::vector<int>> trow(lf_.fac.size());
  std::vector<long> chunk_t;  // T_X doubles per chunk
  for (size_t f = 0; f < lf_.fac.size(); ++f) {
    if (!used[f]) continue;
    const EnvClass& cls = envl.classes[lf_.fac[f].cls];
    long fs = 0;
    for (size_t si = 0; si < P.slabs.size(); ++si) {
      const Slab& sl = P.slabs[si];
      int bi = cls.block_of_col[sl.li];
      if (bi < 0) continue;
      const EnvBlock& eb = cls.blocks[bi];
      if (P.slab_of_left[eb.ri] < 0) continue;  // output rows would fall outside sigma
      fs += (long)eb.mr * sl.width;
    }
    if (chunk_t.empty() || (chunk_t.back() > 0 && chunk_t.back() + fs > chunk_cap)) chunk_t.push_back(0);
    const int c = (int)chunk_t.size() - 1;
    chunk_of[f] = c;
    toff[f].assign(P.slabs.size(), -1);
    trow[f].assign(P.slabs.size(), -1);
    for (size_t si = 0; si < P.slabs.size(); ++si) {
      const Slab& sl = P.slabs[si];
      int bi = cls.block_of_col[sl.li];
      if (bi < 0) continue;
      const EnvBlock& eb = cls.blocks[bi];
      if (P.slab_of_left[eb.ri] < 0) continue;
      toff[f][si] = chunk_t[c];
      trow[f][si] = eb.ri;
      chunk_t[c] += (long)eb.mr * sl.width;
    }
  }
  if (chunk_t.empty()) chunk_t.push_back(0);  // sigma = 0 still needs its zero-writing tiles
  const int nch = (int)chunk_t.size();
  t_size_ = *std::max_element(chunk_t.begin(), chunk_t.end());
  phA_.clear();
  phB_.clear();
  phA_.resize(nch);
  phB_.resize(nch);
  for (int c = 0; c < nch; ++c) {
    phA_[c].mode = GEMM_NN;
    phA_[c].flops_exec = 0;
    phB_[c].mode = GEMM_NT;
    phB_[c].flops_exec = 0;
    phB_[c].wg = true;
  }
  for (size_t f = 0; f < lf_.fac.size(); ++f) {
    if (chunk_of[f] < 0) continue;
    const EnvClass& cls = envl.classes[lf_.fac[f].cls];
    for (size_t si = 0; si < P.slabs.size(); ++si)
      if (toff[f][si] >= 0) {
        const EnvBlock& eb = cls.blocks[cls.block_of_col[P.slabs[si].li]];
        phA_[chunk_of[f]].flops += 2.0 * eb.mr * eb.mc * P.slabs[si].width;  // algorithmic: every T_X block
      }
  }
  // column blocks of each T_X slab that phase B reads; phase A computes only those
  std::vector<std::vector<std::vector<char>>> tused(lf_.fac.size());
  for (size_t f = 0; f < lf_.fac.size(); ++f)
    if (!toff[f].empty()) {
      tused[f].resize(P.slabs.size());
      for (size_t si = 0; si < P.slabs.size(); ++si)
        if (toff[f][si] >= 0) tused[f][si].assign(P.slabs[si].blocks.size(), 0);
    }
  // phase B: gather items per chunk and output block of sigma
  pm_ = PairMix();
  pm_.ptr.push_back(0);
  std::vector<std::vector<std::vector<std::vector<PItem>>>> per(nch);
  for (int c = 0; c < nch; ++c) {
    per[c].resize(P.slabs.size());
    for (size_t si = 0; si < P.slabs.size(); ++si) per[c][si].resize(P.slabs[si].blocks.size());
  }
  // lookups: the block of each physical state in a slab (a slab has at most one
  // per state: the right sector follows from the left one), each factor's slabs,
  // and per right-factor class the output right sector of an input one
  std::vector<std::array<int, 16>> blk_of(P.slabs.size());
  for (size_t si = 0; si < P.slabs.size(); ++si) {
    blk_of[si].fill(-1);
    for (size_t sb = 0; sb < P.slabs[si].blocks.size(); ++sb) blk_of[si][P.slabs[si].blocks[sb].phys] = (int)sb;
  }
  std::vector<std::vector<int>> fslabs(lf_.fac.size());
  for (size_t f = 0; f < lf_.fac.size(); ++f)
    for (size_t si = 0; si < toff[f].size(); ++si)
      if (toff[f][si] >= 0) fslabs[f].push_back((int)si);
  std::vector<std::vector<int>> ro_of(envr.classes.size());  // right class -> (input sector -> output sector)
  for (size_t c = 0; c < envr.classes.size(); ++c) {
    const EnvClass& ycls = envr.classes[c];
    ro_of[c].assign(bk2.sec.size(), -1);
    for (size_t ri = 0; ri < bk2.sec.size(); ++ri) {
      const int ro = bk2.find(bk2.sec[ri].q + ycls.dq);
      const int yb = ycls.block_of_col[ri];
      if (ro >= 0 && yb >= 0 && ycls.blocks[yb].ri == ro) ro_of[c][ri] = ro;
    }
  }
  // items by middle-cut channel, in parallel over contiguous channel ranges;
  // each range fills its own lists, appended in range order afterwards (the
  // serial order, whatever the thread count); the T_X column blocks read are
  // recorded alongside and marked after
  struct Used {
    int f, si, sb;
  };
  const int nthr = plan_threads();
  std::vector<std::vector<std::vector<std::vector<std::vector<PItem>>>>> part(nthr);
  std::vector<std::vector<Used>> uses(nthr);
  parallel_ranges(nmid, [&](int t, long b0, long b1) {
    auto& pt = part[t];
    pt.resize(nch);
    for (int c = 0; c < nch; ++c) {
      pt[c].resize(P.slabs.size());
      for (size_t si = 0; si < P.slabs.size(); ++si) pt[c][si].resize(P.slabs[si].blocks.size());
    }
    std::vector<Used>& ut = uses[t];
    for (long b = b0; b < b1; ++b) {
      if (lf_.by_mid[b].empty() || rf_.by_mid[b].empty()) continue;
      for (const auto& ul : lf_.by_mid[b]) {
        const Mat4& opl = mpo.ops[ul.op];
        const int ch = chunk_of[ul.f];
        const std::vector<int>& sls = fslabs[ul.f];
        for (const auto& ur : rf_.by_mid[b]) {
          const Mat4& opr = mpo.ops[ur.op];
          const int ycl = rf_.fac[ur.f].cls;
          const EnvClass& ycls = envr.classes[ycl];
          const std::vector<int>& rmap = ro_of[ycl];
          const int ybuf = rf_.fac[ur.f].alias ? B_ENVR : B_YMIX;
          const long ybase = rf_.fac[ur.f].off;
          double sc = ul.scale * ur.scale;
          for (int s1 = 0; s1 < 4; ++s1)
            for (int t1 = 0; t1 < 4; ++t1) {
              double wl = opl[s1 * 4 + t1];
              if (wl == 0.0) continue;
              for (int s2 = 0; s2 < 4; ++s2)
                for (int t2 = 0; t2 < 4; ++t2) {
                  double wr = opr[s2 * 4 + t2];
                  if (wr == 0.0) continue;
                  int sout = 4 * s1 + s2, sin = 4 * t1 + t2;
                  for (int si : sls) {
                    const int sb = blk_of[si][sin];
                    if (sb < 0) continue;
                    const Slab& src = P.slabs[si];
                    const SlabBlock& blk = src.blocks[sb];
                    const int ro = rmap[blk.ri];
                    if (ro < 0) continue;
                    const int so = P.slab_of_left[trow[ul.f][si]];
                    const int ob = blk_of[so][sout];
                    if (ob < 0 || P.slabs[so].blocks[ob].ri != ro) continue;
                    ut.push_back({ul.f, si, sb});
                    pt[ch][so][ob].push_back({B_T, toff[ul.f][si] + blk.col0, ybuf,
                                              ybase + ycls.blocks[ycls.block_of_col[blk.ri]].off, src.width,
                                              blk.mr, blk.mr, sc * wl * wr});
                  }
                }
            }
        }
      }
    }
  });
  const auto tp05 = clk::now();
  for (int t = 0; t < nthr; ++t) {
    for (const Used& u : uses[t]) tused[u.f][u.si][u.sb] = 1;
    std::vector<Used>().swap(uses[t]);
  }
  // every output block's list: the ranges' lists in range order, then sorted by
  // operand (consecutive items read neighbouring stretches of T rows)
  struct BlockRef {
    int c, so, ob;
  };
  std::vector<BlockRef> blocks;
  for (int c = 0; c < nch; ++c)
    for (size_t so = 0; so < P.slabs.size(); ++so)
      for (size_t ob = 0; ob < per[c][so].size(); ++ob) blocks.push_back({c, (int)so, (int)ob});
  parallel_ranges((long)blocks.size(), [&](int, long i0, long i1) {
    for (long i = i0; i < i1; ++i) {
      const BlockRef& br = blocks[i];
      auto& dst = per[br.c][br.so][br.ob];
      size_t tot = 0;
      for (int t = 0; t < nthr; ++t)
        if (!part[t].empty()) tot += part[t][br.c][br.so][br.ob].size();
      dst.reserve(tot);
      for (int t = 0; t < nthr; ++t)
        if (!part[t].empty()) {
          auto& src = part[t][br.c][br.so][br.ob];
          dst.insert(dst.end(), src.begin(), src.end());
          std::vector<PItem>().swap(src);
        }
      std::stable_sort(dst.begin(), dst.end(), [](const PItem& x, const PItem& y) {
        if (x.aoff != y.aoff) return x.aoff < y.aoff;
        return x.boff < y.boff;
      });
    }
  });
  part.clear();
  const auto tp1 = clk::now();
  // phase A: T_X = X psi over each run of consecutive column blocks that phase B reads
  for (size_t f = 0; f < lf_.fac.size(); ++f) {
    if (toff[f].empty()) continue;
    Phase& pa = phA_[chunk_of[f]];
    const EnvClass& cls = envl.classes[lf_.fac[f].cls];
    for (size_t si = 0; si < P.slabs.size(); ++si) {
      if (toff[f][si] < 0) continue;
      const Slab& sl = P.slabs[si];
      const EnvBlock& eb = cls.blocks[cls.block_of_col[sl.li]];
      const std::vector<char>& ub = tused[f][si];
      for (size_t b0 = 0; b0 < ub.size();) {
        if (!ub[b0]) {
          ++b0;
          continue;
        }
        size_t b1 = b0 + 1;
        while (b1 < ub.size() && ub[b1] && sl.blocks[b1].col0 == sl.blocks[b1 - 1].col0 + sl.blocks[b1 - 1].mr) ++b1;
        const int c0 = sl.blocks[b0].col0, w = sl.blocks[b1 - 1].col0 + sl.blocks[b1 - 1].mr - c0;
        int ib = (int)pa.items.size();
        pa.items.push_back({lf_.fac[f].alias ? B_ENVL : B_XMIX, lf_.fac[f].off + eb.off, B_PSI, sl.off + c0,
                            eb.mc, sl.width, eb.mc, 1.0});
        add_units(pa.units, B_T, toff[f][si] + c0, sl.width, eb.mr, w, ib, ib + 1, 0);
        pa.flops_exec += 2.0 * eb.mr * eb.mc * w;
        b0 = b1;
      }
    }
  }
  const auto tp2 = clk::now();
  // phase B of chunk c adds into sigma; chunk 0 writes every output block (zero
  // where no item reaches it), later chunks only the blocks they have items for.
  // Items with one A slice (adjacent after the sort) become one product with the
  // weighted sum of their right blocks (N x K, row stride K): merged per block in
  // parallel with block-local offsets into the merged-block buffer, then
  // concatenated in block order.
  struct Merged {
    std::vector<PItem> items;  // B_YPAIR items carry block-local offsets
    std::vector<int> src_buf, ptr_len, nnz;
    std::vector<long> src_off;
    std::vector<double> coef;
    long pm_size = 0;
    double flops = 0, flops_exec = 0;
  };
  std::vector<Merged> merged(blocks.size());
  parallel_ranges((long)blocks.size(), [&](int, long i0, long i1) {
    for (long i = i0; i < i1; ++i) {
      const BlockRef& br = blocks[i];
      auto& v = per[br.c][br.so][br.ob];
      if (br.c > 0 && v.empty()) continue;
      Merged& m = merged[i];
      const Slab& dst = P.slabs[br.so];
      const int nb = dst.blocks[br.ob].mr;
      for (size_t a = 0; a < v.size();) {
        size_t b = a + 1;
        while (b < v.size() && v[b].abuf == v[a].abuf && v[b].aoff == v[a].aoff && v[b].K == v[a].K &&
               v[b].ldb == v[b].K && v[a].ldb == v[a].K)
          ++b;
        if (b - a == 1) {
          m.items.push_back(v[a]);
        } else {
          for (size_t j = a; j < b; ++j) {
            m.src_buf.push_back(v[j].bbuf);
            m.src_off.push_back(v[j].boff);
            m.coef.push_back(v[j].coef);
          }
          m.ptr_len.push_back((int)(b - a));
          m.nnz.push_back(nb * v[a].K);
          m.items.push_back({v[a].abuf, v[a].aoff, B_YPAIR, m.pm_size, v[a].lda, v[a].K, v[a].K, 1.0});
          m.pm_size += (long)nb * v[a].K;
        }
        for (size_t j = a; j < b; ++j) m.flops += 2.0 * dst.ml * nb * v[j].K;  // algorithmic: unmerged
        m.flops_exec += 2.0 * dst.ml * nb * v[a].K;
        a = b;
      }
      std::vector<PItem>().swap(v);
    }
  });
  // offsets of every block's items (per chunk) and merged groups, then a parallel
  // copy into place
  std::vector<long> item_at(blocks.size(), -1), grp_at(blocks.size(), 0), src_at(blocks.size(), 0),
      pm_at(blocks.size(), 0);
  {
    std::vector<long> n_items(nch, 0);
    long ng = 0, nsrc = 0, npm = pm_.size;
    for (size_t i = 0; i < blocks.size(); ++i) {
      const BlockRef& br = blocks[i];
      if (br.c > 0 && merged[i].items.empty()) continue;
      item_at[i] = n_items[br.c];
      n_items[br.c] += (long)merged[i].items.size();
      grp_at[i] = ng;
      ng += (long)merged[i].ptr_len.size();
      src_at[i] = nsrc;
      nsrc += (long)merged[i].src_buf.size();
      pm_at[i] = npm;
      npm += merged[i].pm_size;
    }
    for (int c = 0; c < nch; ++c) phB_[c].items.resize(n_items[c]);
    const size_t g0 = pm_.out_off.size(), s0 = pm_.src_buf.size();
    pm_.ptr.resize(g0 + 1 + ng);
    pm_.out_off.resize(g0 + ng);
    pm_.nnz.resize(g0 + ng);
    pm_.src_buf.resize(s0 + nsrc);
    pm_.src_off.resize(s0 + nsrc);
    pm_.coef.resize(s0 + nsrc);
    parallel_ranges((long)blocks.size(), [&](int, long i0, long i1) {
      for (long i = i0; i < i1; ++i) {
        if (item_at[i] < 0) continue;
        const Merged& m = merged[i];
        PItem* out = phB_[blocks[i].c].items.data() + item_at[i];
        for (size_t j = 0; j < m.items.size(); ++j) {
          out[j] = m.items[j];
          if (out[j].bbuf == B_YPAIR) out[j].boff += pm_at[i];
        }
        long o = pm_at[i], sp = (long)s0 + src_at[i];
        for (size_t g = 0; g < m.ptr_len.size(); ++g) {
          const size_t gi = g0 + grp_at[i] + g;
          pm_.out_off[gi] = o;
          pm_.nnz[gi] = m.nnz[g];
          o += m.nnz[g];
          sp += m.ptr_len[g];
          pm_.ptr[gi + 1] = (int)sp;
        }
        std::copy(m.src_buf.begin(), m.src_buf.end(), pm_.src_buf.begin() + s0 + src_at[i]);
        std::copy(m.src_off.begin(), m.src_off.end(), pm_.src_off.begin() + s0 + src_at[i]);
        std::copy(m.coef.begin(), m.coef.end(), pm_.coef.begin() + s0 + src_at[i]);
      }
    });
    pm_.size = npm;
  }
  for (size_t i = 0; i < blocks.size(); ++i) {
    if (item_at[i] < 0) continue;
    const BlockRef& br = blocks[i];
    Phase& pb = phB_[br.c];
    const Slab& dst = P.slabs[br.so];
    pb.flops += merged[i].flops;
    pb.flops_exec += merged[i].flops_exec;
    add_units(pb.units, B_OUT, dst.off + dst.blocks[br.ob].col0, dst.width, dst.ml, dst.blocks[br.ob].mr,
              (int)item_at[i], (int)(item_at[i] + merged[i].items.size()), br.c == 0 ? 0 : 1);
  }
  merged.clear();
  // split-K granularity of every chunk from the work of all chunks of the phase
  // (pieces of the same size whatever the chunking)
  for (std::vector<Phase>* v : {&phA_, &phB_}) {
    double w = 0;
    for (const Phase& ph : *v)
      for (const PUnit& u : ph.units)
        for (int i = u.ib; i < u.ie; ++i) w += ((u.M + 31) / 32) * ((u.N + 31) / 32) * ((ph.items[i].K + 3) / 4);
    if (v->size() > 1)
      for (Phase& ph : *v) ph.split_work = w;
  }
  if (opt_.verbose > 1) {
    auto ms = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    fprintf(stderr, "sigma plan k=%d (%d threads): items %.2f ms (generation %.2f), phase A %.2f ms, phase B %.2f ms\n",
            k, plan_threads(), ms(tp0, tp1), ms(tp0, tp05), ms(tp1, tp2), ms(tp2, clk::now()));
    // shape statistics: executed (tile-padded) vs useful flops per phase
    for (const Phase* ph : {&phA_[0], &phB_[0]}) {
      double padded = 0, kpad = 0, ksum = 0;
      long nit = 0;
      for (const PUnit& u : ph->units)
        for (int i = u.ib; i < u.ie; ++i) {
          int K = ph->items[i].K;
          padded += 2.0 * 32 * 32 * ((u.M + 31) / 32) * ((u.N + 31) / 32) * ((K + 3) / 4 * 4);
          kpad += (K + 3) / 4 * 4;
          ksum += K;
          ++nit;
        }
      fprintf(stderr, "plan k=%d phase %s: units %zu items %zu (unit-items %ld) useful %.3e padded %.3e (x%.1f) "
              "mean K %.1f (padded %.1f)\n", k, ph == &phA_[0] ? "A" : "B", ph->units.size(), ph->items.size(), nit,
              ph->flops, padded, padded / std::max(ph->flops, 1.0), ksum / std::max(nit, 1L), kpad / std::max(nit, 1L));
    }
    {
      // operand sharing inside phase-B output blocks: items with one A slice
      // (or one B block) in common, and the operand bytes items read
      long ga = 0, gb = 0;
      double abytes = 0, bbytes = 0;
      for (const PUnit& u : phB_[0].units) {
        std::vector<long> ka, kb;
        for (int i = u.ib; i < u.ie; ++i) {
          const PItem& p = phB_[0].items[i];
          ka.push_back(p.aoff * 16 + p.abuf);
          kb.push_back(p.boff * 16 + p.bbuf);
          abytes += 8.0 * u.M * p.K;
          bbytes += 8.0 * u.N * p.K;
        }
        std::sort(ka.begin(), ka.end());
        std::sort(kb.begin(), kb.end());
        ga += std::unique(ka.begin(), ka.end()) - ka.begin();
        gb += std::unique(kb.begin(), kb.end()) - kb.begin();
      }
      fprintf(stderr, "phase B sharing: items %zu, distinct (block, A slice) %ld, distinct (block, B block) %ld, "
              "item A bytes %.3e, item B bytes %.3e\n", phB_[0].items.size(), ga, gb, abytes, bbytes);
      // how much of T phase B reads: distinct (offset, K) column slices of T over all items
      std::vector<std::pair<long, long>> sl;  // (offset, rows x K)
      for (const PUnit& u : phB_[0].units)
        for (int i = u.ib; i < u.ie; ++i)
          if (phB_[0].items[i].abuf == B_T) sl.push_back({phB_[0].items[i].aoff, (long)u.M * phB_[0].items[i].K});
      std::sort(sl.begin(), sl.end());
      sl.erase(std::unique(sl.begin(), sl.end()), sl.end());
      double tread = 0;
      for (auto& x : sl) tread += x.second;
      fprintf(stderr, "phase B reads %zu distinct T slices, %.3e of the %.3e doubles of T\n", sl.size(), tread,
              (double)t_size_);
    }
    std::string dims;
    for (auto& s : bonds_[k].sec) dims += std::to_string(s.dim) + " ";
    fprintf(stderr, "bond %d sectors %zu dims: %s\n", k, bonds_[k].sec.size(), dims.c_str());
    fprintf(stderr, "factors: left %zu (premixed %zu) right %zu (premixed %zu), T chunks %d (largest %ld doubles), psi %ld\n",
            lf_.fac.size(), lf_.out_off.size(), rf_.fac.size(), rf_.out_off.size(), nch, t_size_, P.size);
  }
}

void Solver::build_diag_plan(int k) {
  const MPO& mpo = prob_->mpo;
  const Env& envl = left_[k];
  const Env& envr = right_[k + 2];
  const TensorLayout& P = psi_lay_;
  const Bond& bk = bonds_[k];
  const Bond& bk2 = bonds_[k + 2];
  dblocks_.clear();
  dterms_host_.clear();
  diag_desc_.clear();
  // diagonals of shift-0 factors, per sector
  long dsize = 0;
  std::vector<std::vector<long>> xd(lf_.fac.size()), yd(rf_.fac.size());
  auto extract = [&](const Factor& fac, const Env& env, const Bond& b, std::vector<long>& dst, long base_ofs) {
    const EnvClass& cls = env.classes[fac.cls];
    dst.assign(b.sec.size(), -1);
    if (cls.dq != QN{0, 0}) return;
    for (size_t ci = 0; ci < b.sec.size(); ++ci) {
      int bi = cls.block_of_col[ci];
      if (bi < 0) continue;
      const EnvBlock& eb = cls.blocks[bi];
      dst[ci] = dsize;
      diag_desc_.insert(diag_desc_.end(), {base_ofs + fac.off + eb.off, (int64_t)eb.mc, (int64_t)eb.mc, dsize});
      dsize += eb.mc;
    }
  };
  // the descriptor's source offset is resolved against one buffer per pass; record which
  std::vector<int> desc_buf;
  for (size_t f = 0; f < lf_.fac.size(); ++f) {
    size_t before = diag_desc_.size();
    extract(lf_.fac[f], envl, bk, xd[f], 0);
    for (size_t i = before; i < diag_desc_.size(); i += 4) desc_buf.push_back(lf_.fac[f].alias ? B_ENVL : B_XMIX);
  }
  for (size_t f = 0; f < rf_.fac.size(); ++f) {
    size_t before = diag_desc_.size();
    extract(rf_.fac[f], envr, bk2, yd[f], 0);
    for (size_t i = before; i < diag_desc_.size(); i += 4) desc_buf.push_back(rf_.fac[f].alias ? B_ENVR : B_YMIX);
  }
  diagvec_.reserve(std::max<long>(dsize, 1) * sizeof(double));
  // run the extraction now, one launch per source buffer
  for (int bufid : {B_ENVL, B_XMIX, B_ENVR, B_YMIX}) {
    std::vector<int64_t> d;
    for (size_t i = 0; i < desc_buf.size(); ++i)
      if (desc_buf[i] == bufid) d.insert(d.end(), diag_desc_.begin() + 4 * i, diag_desc_.begin() + 4 * i + 4);
    if (d.empty()) continue;
    const double* src = bufid == B_ENVL ? left_[k].buf.as<double>()
                        : bufid == B_XMIX ? lf_.mix->as<double>()
                        : bufid == B_ENVR ? right_[k + 2].buf.as<double>()
                                          : rf_.mix->as<double>();
    DevMem dd;
    dd.reserve(d.size() * sizeof(int64_t));
    hip_check(hipMemcpyAsync(dd.p, d.data(), d.size() * sizeof(int64_t), hipMemcpyHostToDevice, st), "diag desc");
    launch_extract_diag(dd.as<int64_t>(), (int)(d.size() / 4), src, diagvec_.as<double>(), st);
    hip_check(hipStreamSynchronize(st), "diag extract");
  }
  // terms per output block
  std::vector<std::vector<std::vector<DiagTerm>>> per(P.slabs.size());
  for (size_t si = 0; si < P.slabs.size(); ++si) per[si].resize(P.slabs[si].blocks.size());
  int nmid = (int)mpo.chans[k + 1].size();
  const double* dv = diagvec_.as<double>();
  for (int b = 0; b < nmid; ++b)
    for (const auto& ul : lf_.by_mid[b]) {
      if (envl.classes[lf_.fac[ul.f].cls].dq != QN{0, 0}) continue;
      const Mat4& opl = mpo.ops[ul.op];
      for (const auto& ur : rf_.by_mid[b]) {
        if (envr.classes[rf_.fac[ur.f].cls].dq != QN{0, 0}) continue;
        const Mat4& opr = mpo.ops[ur.op];
        for (int s1 = 0; s1 < 4; ++s1) {
          double wl = opl[s1 * 5];
          if (wl == 0.0) continue;
          for (int s2 = 0; s2 < 4; ++s2) {
            double wr = opr[s2 * 5];
            if (wr == 0.0) continue;
            for (size_t si = 0; si < P.slabs.size(); ++si) {
              const Slab& sl = P.slabs[si];
              long xo = xd[ul.f][sl.li];
              if (xo < 0) continue;
              for (size_t bi = 0; bi < sl.blocks.size(); ++bi) {
                if (sl.blocks[bi].phys != 4 * s1 + s2) continue;
                long yo = yd[ur.f][sl.blocks[bi].ri];
                if (yo < 0) continue;
                per[si][bi].push_back({dv + xo, dv + yo, ul.scale * ur.scale * wl * wr});
              }
            }
          }
        }
      }
    }
  for (size_t si = 0; si < P.slabs.size(); ++si)
    for (size_t bi = 0; bi < per[si].size(); ++bi) {
      const Slab& sl = P.slabs[si];
      int t0 = (int)dterms_host_.size();
      dterms_host_.insert(dterms_host_.end(), per[si][bi].begin(), per[si][bi].end());
      dblocks_.push_back({sl.off + sl.blocks[bi].col0, sl.width, sl.ml, sl.blocks[bi].mr, t0,
                          (int)dterms_host_.size()});
    }
  d_dblocks_.reserve(dblocks_.size() * sizeof(DiagBlock) + 64);
  d_dterms_.reserve(dterms_host_.size() * sizeof(DiagTerm) + 64);
  hip_check(hipMemcpyAsync(d_dblocks_.p, dblocks_.data(), dblocks_.size() * sizeof(DiagBlock), hipMemcpyHostToDevice, st), "dblocks");
  hip_check(hipMemcpyAsync(d_dterms_.p, dterms_host_.data(), dterms_host_.size() * sizeof(DiagTerm), hipMemcpyHostToDevice, st), "dterms");
  diag_ready_ = true;
}

}  // namespace dmrg
