// Two-site sweep driver: MPS setup, environments, sigma, Davidson, SVD truncation.
#include "solver.hpp"

#include "mlp.hpp"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

namespace dmrg {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error(ST_EHIP, std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
}

namespace {
std::atomic<long> g_hip_allocs{0};
constexpr size_t kGranule = 256;
}  // namespace

Arena*& current_arena() {
  thread_local Arena* a = nullptr;
  return a;
}

long library_device_allocations() { return g_hip_allocs.load(); }

Arena::Arena(void* base, size_t bytes) : base_((char*)base), size_(bytes) {
  const size_t skip = (kGranule - (uintptr_t)base_ % kGranule) % kGranule;
  DMRG_REQUIRE(bytes > skip + kGranule, ST_EINVAL, "workspace too small");
  free_[skip] = (bytes - skip) / kGranule * kGranule;
}

void* Arena::alloc(size_t bytes) {
  const size_t need = (std::max<size_t>(bytes, 1) + kGranule - 1) / kGranule * kGranule;
  // best fit; large buffers (environments, sigma intermediates, Davidson basis)
  // are cut from the top of their range and small ones (plan tables) from the
  // bottom, so the small ones do not split the space the large ones need
  auto best = free_.end();
  for (auto it = free_.begin(); it != free_.end(); ++it)
    if (it->second >= need && (best == free_.end() || it->second < best->second)) best = it;
  if (best != free_.end()) {
    const size_t off = best->first, len = best->second;
    free_.erase(best);
    size_t at = off;
    if (need >= (size_t(64) << 20)) {
      at = off + len - need;
      if (len > need) free_[off] = len - need;
    } else if (len > need) {
      free_[off + need] = len - need;
    }
    used_[at] = need;
    in_use_ += need;
    peak_ = std::max(peak_, in_use_);
    return base_ + at;
  }
  failed_ = need;
  throw Error(ST_ENOMEM, "workspace exhausted: " + std::to_string(need) + " bytes requested with " +
                             std::to_string(in_use_) + " of " + std::to_string(size_) +
                             " in use; dmrg_workspace_query gives the size to attach");
}

void Arena::free(void* p) {
  const size_t off = (size_t)((char*)p - base_);
  auto it = used_.find(off);
  if (it == used_.end()) return;
  size_t start = off, len = it->second;
  in_use_ -= len;
  used_.erase(it);
  auto nx = free_.lower_bound(start);
  if (nx != free_.end() && nx->first == start + len) {  // merge with the next free range
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = len;
}

PinnedStage::~PinnedStage() {
  if (p) (void)hipHostFree(p);
}
void* PinnedStage::reserve(size_t b) {
  if (b <= bytes && p) return p;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  const size_t want = std::max(b, bytes + bytes / 2);
  hip_check(hipHostMalloc(&p, want, hipHostMallocDefault), "pinned staging");
  bytes = want;
  return p;
}

DevMem::~DevMem() { release(); }
void DevMem::release() {
  if (p) {
    if (arena) arena->free(p);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
  arena = nullptr;
}
void DevMem::reserve(size_t b) {
  if (b <= bytes && p) return;
  const size_t grown = p ? bytes : 0;
  release();
  if (b == 0) b = 8;
  if (Arena* a = current_arena()) {
    // a grown buffer keeps a quarter of headroom: fewer reallocations, less fragmentation
    const size_t want = grown ? std::max(b, grown + grown / 4) : b;
    try {
      p = a->alloc(want);
      bytes = want;
    } catch (const Error&) {
      if (want == b) throw;
      p = a->alloc(b);
      bytes = b;
    }
    arena = a;
    return;
  }
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    throw Error(ST_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
  }
  ++g_hip_allocs;
  bytes = b;
}

namespace {

struct Rng {  // splitmix64 + Box-Muller: a seeded, platform-independent normal stream
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Host check of block-copy descriptors against source / destination sizes.
void check_desc(const std::vector<int64_t>& d, size_t begin, size_t end, long src_n, long dst_n) {
  for (size_t i = begin; i < end; i += 9) {
    long rows = d[i + 6], cols = d[i + 7];
    if (rows <= 0 || cols <= 0) continue;
    for (int side = 0; side < 2; ++side) {  // all four corners (strides may be negative)
      long base = d[i + 3 * side], rs = d[i + 1 + 3 * side], cs = d[i + 2 + 3 * side];
      long lim = side ? dst_n : src_n;
      long lo = base + std::min(0L, (rows - 1) * rs) + std::min(0L, (cols - 1) * cs);
      long hi = base + std::max(0L, (rows - 1) * rs) + std::max(0L, (cols - 1) * cs);
      if (lo < 0 || hi >= lim) throw Error(ST_EINVAL, "block copy out of bounds");
    }
  }
}

int64_t dbits(double x) {
  int64_t b;
  std::memcpy(&b, &x, 8);
  return b;
}

}  // namespace

Solver::Solver(const Problem* p, const Options& o, hipStream_t s) : prob_(p), opt_(o), st(s) {
  L_ = p->n;
  bonds_.resize(L_ + 1);
  mps_.resize(L_);
  left_.resize(L_ + 1);
  right_.resize(L_ + 1);
  DMRG_REQUIRE(opt_.n_states >= 1 && opt_.n_states <= 8, ST_EINVAL, "n_states must be in [1, 8]");
  DMRG_REQUIRE(opt_.M >= 1, ST_EINVAL, "M must be positive");
  if (opt_.weights.empty()) opt_.weights.assign(opt_.n_states, 1.0 / opt_.n_states);
  DMRG_REQUIRE((int)opt_.weights.size() == opt_.n_states, ST_EINVAL, "weights size mismatch");
  {
    double wsum = 0.0;
    for (double w : opt_.weights) {
      DMRG_REQUIRE(std::isfinite(w) && w >= 0.0, ST_EINVAL, "state weights must be finite and >= 0");
      wsum += w;
    }
    DMRG_REQUIRE(wsum > 0.0, ST_EINVAL, "state weights must not all be zero");
    for (double& w : opt_.weights) w /= wsum;
  }
  opt_.max_subspace = std::max(std::min(opt_.max_subspace, 64), 2 * opt_.n_states + 2);
  DMRG_REQUIRE(opt_.precond >= 0 && opt_.precond <= 3, ST_EINVAL, "unknown preconditioner");
  precond_ = opt_.precond;
  init_random_mps();
}

Solver::~Solver() {
  for (hipEvent_t e : sig_ev_) (void)hipEventDestroy(e);
  if (stage_ev_) {
    (void)hipEventSynchronize(stage_ev_);  // the pinned staging is freed after this
    (void)hipEventDestroy(stage_ev_);
  }
  for (int i = 0; i < kAuxStreams; ++i) {
    if (aux_rb_[i]) rocblas_destroy_handle(aux_rb_[i]);
    if (aux_st_[i]) (void)hipStreamDestroy(aux_st_[i]);
  }
  for (hipEvent_t& e : aux_ev_)
    if (e) (void)hipEventDestroy(e);
}

// Right-canonical random MPS in the target sector: every slab (rows of one
// left sector) has orthonormal rows.  Bond sectors are the full sector
// dimensions scaled to fit M, clipped so each slab has at least as many
// columns as rows.
void Solver::init_random_mps() {
  const int L = L_, na = prob_->n_alpha, nb = prob_->n_beta;
  for (int c = 0; c <= L; ++c) {
    Bond b;
    long tot = 0;
    for (int a = 0; a <= std::min(c, na); ++a)
      for (int bb = 0; bb <= std::min(c, nb); ++bb) {
        if (na - a > L - c || nb - bb > L - c) continue;
        long d = std::min(binom(c, a) * binom(c, bb), binom(L - c, na - a) * binom(L - c, nb - bb));
        if (d <= 0) continue;
        b.sec.push_back({{a + bb, a - bb}, (int)std::min<long>(d, 1 << 30)});
        tot += d;
      }
    std::sort(b.sec.begin(), b.sec.end(), [](const Sector& x, const Sector& y) { return x.q < y.q; });
    if (tot > opt_.M)
      for (auto& s : b.sec) s.dim = (int)std::max<long>(1, (long)s.dim * opt_.M / tot);
    bonds_[c] = b;
  }
  DMRG_REQUIRE(!bonds_[L].sec.empty() && !bonds_[0].sec.empty(), ST_ESECTOR, "empty target sector");
  for (int c = L - 1; c >= 0; --c) {
    Bond& b = bonds_[c];
    for (auto& s : b.sec) {
      int cap = 0;
      for (int p = 0; p < 4; ++p) {
        int ri = bonds_[c + 1].find(s.q + site_qn(p));
        if (ri >= 0) cap += bonds_[c + 1].sec[ri].dim;
      }
      s.dim = std::min(s.dim, cap);
    }
    b.sec.erase(std::remove_if(b.sec.begin(), b.sec.end(), [](const Sector& x) { return x.dim <= 0; }),
                b.sec.end());
  }
  DMRG_REQUIRE(!bonds_[0].sec.empty(), ST_ESECTOR, "empty target sector");
  Rng rng(opt_.seed);
  for (int k = 0; k < L; ++k) {
    SiteTensor& t = mps_[k];
    t.lay = make_tensor_layout(bonds_[k], bonds_[k + 1], site_phys_qn());
    std::vector<double> h(t.lay.size);
    for (const Slab& sl : t.lay.slabs) {
      double* S = h.data() + sl.off;
      for (long i = 0; i < (long)sl.ml * sl.width; ++i) S[i] = rng.normal();
      for (int pass = 0; pass < 2; ++pass)
        for (int r = 0; r < sl.ml; ++r) {
          double* row = S + (long)r * sl.width;
          for (int q = 0; q < r; ++q) {
            const double* prev = S + (long)q * sl.width;
            double d = 0;
            for (int c = 0; c < sl.width; ++c) d += prev[c] * row[c];
            for (int c = 0; c < sl.width; ++c) row[c] -= d * prev[c];
          }
          double nrm = 0;
          for (int c = 0; c < sl.width; ++c) nrm += row[c] * row[c];
          nrm = std::sqrt(nrm);
          for (int c = 0; c < sl.width; ++c) row[c] /= nrm;
        }
    }
    pending_mps_.insert(pending_mps_.end(), h.begin(), h.end());
  }
  for (auto& e : left_) e.valid = false;
  for (auto& e : right_) e.valid = false;
  ovl_invalidate(0, L_);
  plan_k_ = -1;
  centers_.clear();
  center_site_ = 0;  // every site right-canonical: the orthogonality centre is site 0
}

void Solver::materialize() {
  if (pending_mps_.empty()) return;
  long off = 0;
  for (int k = 0; k < L_; ++k) {
    SiteTensor& t = mps_[k];
    t.buf.reserve(std::max<long>(t.lay.size, 1) * sizeof(double));
    hip_check(hipMemcpy(t.buf.p, pending_mps_.data() + off, t.lay.size * sizeof(double), hipMemcpyHostToDevice),
              "mps upload");
    off += t.lay.size;
  }
  std::vector<double>().swap(pending_mps_);
}

SolverState Solver::save_state() {
  SolverState s;
  s.bonds = bonds_;
  s.mps = pending_mps_.empty() ? export_mps() : pending_mps_;
  s.center_site = center_site_;
  for (const DevMem& c : centers_) {
    std::vector<double> h(center_lay_.size);
    if (center_lay_.size > 0)
      hip_check(hipMemcpy(h.data(), c.p, center_lay_.size * sizeof(double), hipMemcpyDeviceToHost), "centre save");
    s.centers.push_back(std::move(h));
  }
  if (!centers_.empty()) {
    const int cs = center_site_;
    s.center_bond_l = bonds_[cs].sec;
    s.center_bond_r = bonds_[cs + 1].sec;
  }
  s.opt = opt_;
  s.precond = precond_;
  s.net = net_;
  s.rec_cap = rec_cap_;
  s.rec_sample = rec_sample_;
  s.kernel_tag = kernel_tag_;
  s.stats = st_;
  for (const Deflated& d : defl_) {
    SolverState::Lower lo;
    lo.bonds = d.bonds;
    lo.w = d.w;
    for (const SiteTensor& t : d.sites) {
      const size_t at = lo.mps.size();
      lo.mps.resize(at + t.lay.size);
      if (t.lay.size > 0)
        hip_check(hipMemcpy(lo.mps.data() + at, t.buf.p, t.lay.size * 8, hipMemcpyDeviceToHost), "deflated save");
    }
    s.lower.push_back(std::move(lo));
  }
  return s;
}

void Solver::restore_state(const SolverState& s) {
  std::vector<const double*> sites(L_);
  long off = 0;
  for (int k = 0; k < L_; ++k) {
    sites[k] = s.mps.data() + off;
    off += make_tensor_layout(s.bonds[k], s.bonds[k + 1], site_phys_qn()).size;
  }
  std::vector<double>().swap(pending_mps_);
  set_mps(s.bonds, sites);
  center_site_ = s.center_site;
  if (!s.centers.empty() && s.center_site >= 0) {
    Bond bl, br;
    bl.sec = s.center_bond_l;
    br.sec = s.center_bond_r;
    center_lay_ = make_tensor_layout(bl, br, site_phys_qn());
    centers_.resize(s.centers.size());
    for (size_t r = 0; r < s.centers.size(); ++r) {
      centers_[r].reserve(std::max<long>(center_lay_.size, 1) * 8);
      if (center_lay_.size > 0)
        hip_check(hipMemcpy(centers_[r].p, s.centers[r].data(), center_lay_.size * 8, hipMemcpyHostToDevice),
                  "centre restore");
    }
  }
  opt_ = s.opt;
  precond_ = s.precond;
  net_ = (MLP*)s.net;
  rec_cap_ = s.rec_cap;
  rec_sample_ = s.rec_sample;
  kernel_tag_ = s.kernel_tag;
  st_ = s.stats;
  defl_.clear();
  for (const SolverState::Lower& lo : s.lower) {
    std::vector<const double*> ptr(L_);
    long o = 0;
    for (int k = 0; k < L_; ++k) {
      ptr[k] = lo.mps.data() + o;
      o += make_tensor_layout(lo.bonds[k], lo.bonds[k + 1], site_phys_qn()).size;
    }
    deflate_add(lo.bonds, ptr, lo.w);
  }
}

void Solver::set_mps(const std::vector<Bond>& bonds, const std::vector<const double*>& sites) {
  DMRG_REQUIRE((int)bonds.size() == L_ + 1 && (int)sites.size() == L_, ST_EINVAL, "MPS size mismatch");
  DMRG_REQUIRE((bonds[0].sec.size() == 1 && bonds[0].sec[0].q == QN{0, 0} && bonds[0].sec[0].dim == 1),
               ST_EINVAL, "left boundary bond must be the single vacuum state");
  DMRG_REQUIRE(bonds[L_].sec.size() == 1 && bonds[L_].sec[0].q == prob_->target() && bonds[L_].sec[0].dim == 1,
               ST_EINVAL, "right boundary bond must be the single target state");
  for (int c = 0; c <= L_; ++c)
    for (size_t i = 0; i < bonds[c].sec.size(); ++i) {
      DMRG_REQUIRE(bonds[c].sec[i].dim >= 1, ST_EINVAL, "sector dims must be positive");
      if (i) DMRG_REQUIRE(bonds[c].sec[i - 1].q < bonds[c].sec[i].q, ST_EINVAL, "sectors must be sorted");
    }
  bonds_ = bonds;
  std::vector<double>().swap(pending_mps_);
  for (int k = 0; k < L_; ++k) {
    SiteTensor& t = mps_[k];
    t.lay = make_tensor_layout(bonds_[k], bonds_[k + 1], site_phys_qn());
    t.buf.reserve(std::max<long>(t.lay.size, 1) * sizeof(double));
    hip_check(hipMemcpy(t.buf.p, sites[k], t.lay.size * sizeof(double), hipMemcpyHostToDevice), "mps upload");
  }
  for (auto& e : left_) e.valid = false;
  for (auto& e : right_) e.valid = false;
  ovl_invalidate(0, L_);
  plan_k_ = -1;
  centers_.clear();
  center_site_ = -1;  // gauge unknown
}

void Solver::ensure_left(int c) {
  if (left_[c].valid) return;
  if (c == 0) {
    Env& e = left_[0];
    make_env_layout(e, 0, bonds_[0]);
    launch_fill(e.buf.as<double>(), e.size, 0.0, st);
    int I = prob_->mpo.chan_I[0];
    DMRG_REQUIRE(I >= 0, ST_EINVAL, "no identity channel at the left end");
    double one = 1.0;
    hip_check(hipMemcpyAsync(e.buf.as<double>() + e.chan_off(I), &one, 8, hipMemcpyHostToDevice, st), "env0");
    hip_check(hipStreamSynchronize(st), "env0");
    e.valid = true;
    return;
  }
  ensure_left(c - 1);
  plan_k_ = -1;  // the update reuses the left premix buffer of the prepared step
  FactorSide fs;
  build_factor_side(fs, true, c - 1);
  run_premix(fs, left_[c - 1]);
  env_update_left(c - 1, fs);
  hip_check(hipStreamSynchronize(st), "env left");
}

void Solver::ensure_right(int c) {
  if (right_[c].valid) return;
  if (c == L_) {
    Env& e = right_[L_];
    make_env_layout(e, L_, bonds_[L_]);
    launch_fill(e.buf.as<double>(), e.size, 0.0, st);
    int H = prob_->mpo.chan_H[L_];
    DMRG_REQUIRE(H >= 0, ST_EINVAL, "no closing channel at the right end");
    double one = 1.0;
    hip_check(hipMemcpyAsync(e.buf.as<double>() + e.chan_off(H), &one, 8, hipMemcpyHostToDevice, st), "envL");
    hip_check(hipStreamSynchronize(st), "envL");
    e.valid = true;
    return;
  }
  ensure_right(c + 1);
  plan_k_ = -1;  // the update reuses the right premix buffer of the prepared step
  FactorSide fs;
  build_factor_side(fs, false, c);
  run_premix(fs, right_[c + 1]);
  env_update_right(c, fs);
  hip_check(hipStreamSynchronize(st), "env right");
}

void Solver::prepare(int k) {
  DMRG_REQUIRE(k >= 0 && k + 1 < L_, ST_EINVAL, "two-site step out of range");
  const auto tp0 = std::chrono::steady_clock::now();
  ensure_left(k);
  ensure_right(k + 2);
  // park the current plan, then reuse the cached one of step k if its outer bonds match
  hip_check(hipStreamSynchronize(st), "prepare");  // host staging of the parked plan is no longer read
  if (plan_built_k_ >= 0) {
    StepPlan& c = plan_cache_[plan_built_k_];
    c.key_l = bonds_at_build_l_;
    c.key_r = bonds_at_build_r_;
    c.lf = std::move(lf_);
    c.rf = std::move(rf_);
    c.pm = std::move(pm_);
    c.psi_lay = std::move(psi_lay_);
    c.phA = std::move(phA_);
    c.phB = std::move(phB_);
    c.t_size = t_size_;
    plan_built_k_ = -1;
  }
  auto same_bond = [](const std::vector<Sector>& a, const std::vector<Sector>& b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
      if (a[i].q != b[i].q || a[i].dim != b[i].dim) return false;
    return true;
  };
  auto hit = plan_cache_.find(k);
  if (hit != plan_cache_.end() && same_bond(hit->second.key_l, bonds_[k].sec) &&
      same_bond(hit->second.key_r, bonds_[k + 2].sec)) {
    StepPlan& c = hit->second;
    lf_ = std::move(c.lf);
    rf_ = std::move(c.rf);
    pm_ = std::move(c.pm);
    psi_lay_ = std::move(c.psi_lay);
    phA_ = std::move(c.phA);
    phB_ = std::move(c.phB);
    t_size_ = c.t_size;
    plan_cache_.erase(hit);
    run_premix(lf_, left_[k]);
    run_premix(rf_, right_[k + 2]);
    run_pairmix(k);
    st_.plan_hits++;
  } else {
    if (hit != plan_cache_.end()) plan_cache_.erase(hit);
    const auto tb0 = std::chrono::steady_clock::now();
    build_factor_side(lf_, true, k);
    run_premix(lf_, left_[k]);
    build_factor_side(rf_, false, k + 1);
    run_premix(rf_, right_[k + 2]);
    const auto tb1 = std::chrono::steady_clock::now();
    build_sigma_plan(k);
    const auto tb2 = std::chrono::steady_clock::now();
    st_.plan_build_ms += std::chrono::duration<double, std::milli>(tb2 - tb0).count();
    if (opt_.verbose > 1)
      fprintf(stderr, "plan k=%d: factor sides and premix %.2f ms, sigma plan %.2f ms\n", k,
              std::chrono::duration<double, std::milli>(tb1 - tb0).count(),
              std::chrono::duration<double, std::milli>(tb2 - tb1).count());
    run_pairmix(k);
    for (std::vector<Phase>* v : {&phA_, &phB_})
      for (Phase& ph : *v)
        for (int i = 0; i < 3; ++i) ph.uploaded[i] = false;
  }
  plan_built_k_ = k;
  bonds_at_build_l_ = bonds_[k].sec;
  bonds_at_build_r_ = bonds_[k + 2].sec;
  t_buf_.reserve(std::max<long>(t_size_, 1) * sizeof(double));
  psi_in_.reserve(std::max<long>(psi_lay_.size, 1) * sizeof(double));
  out_buf_.reserve(std::max<long>(psi_lay_.size, 1) * sizeof(double));
  lowp_prec_ = -1;
  diag_ready_ = false;
  // dense blocks of the two-site vector, for the preconditioner features
  fblocks_host_.clear();
  for (const Slab& sl : psi_lay_.slabs)
    for (const auto& b : sl.blocks)
      fblocks_host_.insert(fblocks_host_.end(), {(int64_t)(sl.off + b.col0), (int64_t)sl.width, (int64_t)sl.ml,
                                                 (int64_t)b.mr});
  nfb_ = (int)(fblocks_host_.size() / 4);
  d_fblocks_.reserve(fblocks_host_.size() * 8 + 8);
  if (nfb_ > 0)
    hip_check(hipMemcpyAsync(d_fblocks_.p, fblocks_host_.data(), fblocks_host_.size() * 8, hipMemcpyHostToDevice, st),
              "feature blocks");
  plan_k_ = k;
  hip_check(hipStreamSynchronize(st), "prepare");
  st_.prepare_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count();
}

std::vector<double> Solver::env_host(int cut, int side) {
  Env& e = side == 0 ? left_[cut] : right_[cut];
  if (side == 0) ensure_left(cut);
  else ensure_right(cut);
  std::vector<double> v(e.size);
  hip_check(hipMemcpy(v.data(), e.buf.p, e.size * sizeof(double), hipMemcpyDeviceToHost), "env copy");
  return v;
}

long Solver::twosite_size(int k) const {
  DMRG_REQUIRE(k >= 0 && k + 1 < L_, ST_EINVAL, "two-site step out of range");
  return make_tensor_layout(bonds_[k], bonds_[k + 2], twosite_phys_qn()).size;
}

double Solver::last_sigma_flops() const {
  double f = 0;
  for (const std::vector<Phase>* v : {&phA_, &phB_})
    for (const Phase& ph : *v) f += ph.flops;
  return f;
}
double Solver::last_sigma_flops_exec() const {
  double f = 0;
  for (const std::vector<Phase>* v : {&phA_, &phB_})
    for (const Phase& ph : *v) f += ph.flops_exec < 0 ? ph.flops : ph.flops_exec;
  return f;
}

void Solver::ensure_lowp(int prec) {
  if (lowp_prec_ == prec) return;
  const int k = plan_k_;
  struct Src { int id; const double* p; long n; };
  Src src[] = {{B_ENVL, left_[k].buf.as<double>(), left_[k].size},
               {B_ENVR, right_[k + 2].buf.as<double>(), right_[k + 2].size},
               {B_XMIX, lmix_.as<double>(), lf_.premix_size},
               {B_YMIX, rmix_.as<double>(), rf_.premix_size},
               {B_YPAIR, pmix_.as<double>(), pm_.size}};
  size_t esz = prec == PREC_F32 ? 4 : 2;
  for (auto& s : src) {
    lowp_[s.id].reserve(std::max<long>(s.n, 1) * esz);
    if (s.n <= 0 || !s.p) continue;
    if (prec == PREC_F32) launch_f64_to_f32(s.p, lowp_[s.id].as<float>(), s.n, st);
    else launch_f64_to_bf16(s.p, lowp_[s.id].as<uint16_t>(), s.n, st);
  }
  lowp_[B_PSI].reserve(std::max<long>(psi_lay_.size, 1) * esz);
  lowp_[B_T].reserve(std::max<long>(t_size_, 1) * 4);
  lowp_[B_OUT].reserve(std::max<long>(psi_lay_.size, 1) * 4);
  setup_lowp_shift(k);
  if (shift_on_) {
    const double shift[3] = {shift_a_, shift_b_, shift_b_};
    const int ids[3] = {B_ENVL, B_ENVR, B_YPAIR};
    const double* srcs[3] = {left_[k].buf.as<double>(), right_[k + 2].buf.as<double>(), pmix_.as<double>()};
    for (int i = 0; i < 3; ++i)
      launch_shift_entries(srcs[i], lowp_[ids[i]].p, prec != PREC_F32, shift_idx_[i].as<long>(),
                           shift_w_[i].as<double>(), shift_n_[i], shift[i], st);
  }
  lowp_prec_ = prec;  // resolved low-precision plans stay valid while their buffers do (bases are compared)
}

void Solver::setup_lowp_shift(int k) {
  shift_on_ = false;
  shift_a_ = shift_b_ = 0.0;
  for (long& n : shift_n_) n = 0;
  if (center_site_ != k && center_site_ != k + 1) return;
  const MPO& mpo = prob_->mpo;
  const int chH = mpo.chan_H[k], chI = mpo.chan_I[k + 2];
  std::vector<long> idx[3];
  std::vector<double> w[3];
  // a channel's square diagonal blocks: element offsets of their diagonals
  auto diag_of = [](const Env& e, int ch, std::vector<long>& out, std::map<long, int>* blocks) {
    const EnvClass& c = e.classes[e.chan_class[ch]];
    const long base = e.chan_off(ch);
    for (const EnvBlock& b : c.blocks) {
      if (b.ri != b.ci || b.mr != b.mc) continue;
      if (blocks) (*blocks)[base + b.off] = b.mr;
      for (int i = 0; i < b.mr; ++i) out.push_back(base + b.off + (long)i * (b.mc + 1));
    }
  };
  // the mean of those diagonal entries (host copy of the channel)
  auto diag_mean = [&](const Env& e, int ch, const std::vector<long>& d) {
    const long base = e.chan_off(ch), nnz = e.classes[e.chan_class[ch]].nnz;
    std::vector<double> h(nnz);
    hip_check(hipMemcpy(h.data(), e.buf.as<double>() + base, nnz * 8, hipMemcpyDeviceToHost), "shift");
    double acc = 0;
    for (long x : d) acc += h[x - base];
    return d.empty() ? 0.0 : acc / (double)d.size();
  };
  // a channel read through a premixed factor would carry the shift into other terms
  auto premixed = [](const FactorSide& fs, long off) {
    return std::find(fs.src_off.begin(), fs.src_off.end(), off) != fs.src_off.end();
  };
  if (chH >= 0 && !premixed(lf_, left_[k].chan_off(chH))) {
    diag_of(left_[k], chH, idx[0], nullptr);
    shift_a_ = diag_mean(left_[k], chH, idx[0]);
    w[0].assign(idx[0].size(), 1.0);
  }
  if (chI >= 0 && !premixed(rf_, right_[k + 2].chan_off(chI))) {
    std::map<long, int> rblocks;
    diag_of(right_[k + 2], chI, idx[1], &rblocks);
    shift_b_ = diag_mean(right_[k + 2], chI, idx[1]);
    w[1].assign(idx[1].size(), 1.0);
    // merged right blocks that include a block of R_I: shift c b on their diagonals
    for (size_t g = 0; g + 1 < pm_.ptr.size(); ++g)
      for (int j = pm_.ptr[g]; j < pm_.ptr[g + 1]; ++j) {
        if (pm_.src_buf[j] != B_ENVR) continue;
        auto it = rblocks.find(pm_.src_off[j]);
        if (it == rblocks.end()) continue;
        const int d = it->second;
        if ((long)d * d != pm_.nnz[g]) continue;
        for (int i = 0; i < d; ++i) {
          idx[2].push_back(pm_.out_off[g] + (long)i * (d + 1));
          w[2].push_back(pm_.coef[j]);
        }
      }
  }
  if (idx[0].empty() && idx[1].empty()) return;
  for (int i = 0; i < 3; ++i) {
    shift_n_[i] = (long)idx[i].size();
    shift_idx_[i].reserve(std::max<size_t>(idx[i].size(), 1) * 8);
    shift_w_[i].reserve(std::max<size_t>(w[i].size(), 1) * 8);
    if (!idx[i].empty()) {
      hip_check(hipMemcpy(shift_idx_[i].p, idx[i].data(), idx[i].size() * 8, hipMemcpyHostToDevice), "shift");
      hip_check(hipMemcpy(shift_w_[i].p, w[i].data(), w[i].size() * 8, hipMemcpyHostToDevice), "shift");
    }
  }
  shift_on_ = true;
}

void Solver::sigma(int k, int prec, const double* psi, double* out) {
  if (plan_k_ != k) prepare(k);
  const long n = psi_lay_.size;
  long sizes[B_NBUF] = {};
  sizes[B_PSI] = n;
  sizes[B_OUT] = n;
  sizes[B_T] = t_size_;
  sizes[B_XMIX] = lf_.premix_size;
  sizes[B_YMIX] = rf_.premix_size;
  sizes[B_YPAIR] = pm_.size;
  sizes[B_ENVL] = left_[k].size;
  sizes[B_ENVR] = right_[k + 2].size;
  // events per chunk c: [3c] before phase A, [3c+1] before phase B, [3c+2] after
  // phase B's GEMM (before its split-K reduction); [3 nch] after the last chunk
  const int nch = (int)phA_.size();
  const size_t nev = 3 * (size_t)nch + 1;
  while (sig_ev_.size() < nev) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "event");
    sig_ev_.push_back(e);
  }
  const bool f64 = prec == PREC_F64;
  void* bases[B_NBUF] = {};
  size_t esz[B_NBUF] = {8, 8, 8, 8, 8, 8, 8, 8, 8};
  int pa_prec = PREC_F64, pb_prec = PREC_F64;
  if (f64) {
    // fixed input/output buffers keep the resolved plan valid for every call
    bases[B_PSI] = psi_in_.p;
    bases[B_OUT] = out_buf_.p;
    bases[B_T] = t_buf_.p;
    bases[B_XMIX] = lmix_.p;
    bases[B_YMIX] = rmix_.p;
    bases[B_ENVL] = left_[k].buf.p;
    bases[B_ENVR] = right_[k + 2].buf.p;
    bases[B_YPAIR] = pmix_.p;
    launch_copy(psi_in_.as<double>(), psi, n, st);
  } else {
    ensure_lowp(prec);
    for (int i = 0; i < B_NBUF; ++i) bases[i] = lowp_[i].p;
    const size_t le = prec == PREC_F32 ? 4 : 2;
    for (int i = 0; i < B_NBUF; ++i) esz[i] = le;
    esz[B_OUT] = esz[B_T] = 4;
    if (prec == PREC_F32) launch_f64_to_f32(psi, lowp_[B_PSI].as<float>(), n, st);
    else launch_f64_to_bf16(psi, lowp_[B_PSI].as<uint16_t>(), n, st);
    pa_prec = prec == PREC_F32 ? PREC_F32 : PREC_BF16;
    pb_prec = prec == PREC_F32 ? PREC_F32 : 3;
  }
  for (int c = 0; c < nch; ++c) {
    phA_[c].tag = 1 + 2 * kernel_tag_;
    phB_[c].tag = 2 + 2 * kernel_tag_;
    (void)hipEventRecord(sig_ev_[3 * c], st);
    run_phase(phA_[c], pa_prec, bases, esz, sizes);
    (void)hipEventRecord(sig_ev_[3 * c + 1], st);
    phB_[c].gemm_done = f64 ? sig_ev_[3 * c + 2] : nullptr;
    run_phase(phB_[c], pb_prec, bases, esz, sizes);
    phB_[c].gemm_done = nullptr;
    if (!f64 || phB_[c].units.empty()) (void)hipEventRecord(sig_ev_[3 * c + 2], st);
  }
  (void)hipEventRecord(sig_ev_[3 * nch], st);
  if (f64) {
    launch_copy(out, out_buf_.as<double>(), n, st);
  } else {
    launch_f32_to_f64(lowp_[B_OUT].as<float>(), out, n, st);
    if (shift_on_) launch_axpy(out, psi, shift_a_ + shift_b_, n, st);  // the shift back, in fp64
  }
  hip_check(hipEventSynchronize(sig_ev_[3 * nch]), "sigma");
  float a = 0, b = 0, g = 0;
  for (int c = 0; c < nch; ++c) {
    float x = 0, y = 0, z = 0;
    (void)hipEventElapsedTime(&x, sig_ev_[3 * c], sig_ev_[3 * c + 1]);
    (void)hipEventElapsedTime(&y, sig_ev_[3 * c + 1], sig_ev_[3 * c + 3]);
    (void)hipEventElapsedTime(&z, sig_ev_[3 * c + 1], sig_ev_[3 * c + 2]);
    a += x;
    b += y;
    g += f64 ? z : y;
  }
  sigma_phase_ms_[0] = a;
  sigma_phase_ms_[1] = b;
  st_.sigma_a_ms += a;
  st_.sigma_b_ms += b;
  st_.sigma_b_gemm_ms += g;
  for (int c = 0; c < nch; ++c) {
    st_.sigma_a_flops += phA_[c].flops;
    st_.sigma_b_flops += phB_[c].flops;
    st_.sigma_a_flops_exec += phA_[c].flops_exec < 0 ? phA_[c].flops : phA_[c].flops_exec;
    st_.sigma_b_flops_exec += phB_[c].flops_exec < 0 ? phB_[c].flops : phB_[c].flops_exec;
    st_.sigma_flops += phA_[c].flops + phB_[c].flops;
  }
  st_.sigma_ms += a + b;
  st_.matvecs++;
  if (prec != PREC_F64) st_.lowp_matvecs++;
}

void Solver::diag(int k, double* out) {
  if (plan_k_ != k) prepare(k);
  if (!diag_ready_) build_diag_plan(k);
  launch_diag(out, d_dblocks_.as<DiagBlock>(), (int)dblocks_.size(), d_dterms_.as<DiagTerm>(), st);
}

void Solver::gemm_once(int mode, std::vector<GemmItem>& items, std::vector<GemmUnit>& units) {
  if (units.empty()) return;
  scratch_h_items_ = items;
  scratch_h_units_ = units;
  scratch_items_.reserve(items.size() * sizeof(GemmItem) + 64);
  scratch_units_.reserve(units.size() * sizeof(GemmUnit) + 64);
  hip_check(hipMemcpyAsync(scratch_items_.p, scratch_h_items_.data(), items.size() * sizeof(GemmItem),
                           hipMemcpyHostToDevice, st), "items");
  hip_check(hipMemcpyAsync(scratch_units_.p, scratch_h_units_.data(), units.size() * sizeof(GemmUnit),
                           hipMemcpyHostToDevice, st), "units");
  launch_gemm(PREC_F64, mode, scratch_units_.as<GemmUnit>(), (int)units.size(), scratch_items_.as<GemmItem>(), st);
  hip_check(hipStreamSynchronize(st), "gemm_once");
}

static void tile_units(std::vector<GemmUnit>& units, double* C, int ldc, int M, int N, int ib, int ie) {
  for (int m0 = 0; m0 < M; m0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) units.push_back({C, ldc, M, N, m0, n0, ib, ie, 0});
}

// out (two-site, sites k,k+1) = a (site k) * b (site k+1), contracted over bond k+1.
void Solver::form_twosite(int k, const SiteTensor& a, const SiteTensor& b, double* out) {
  TensorLayout P = make_tensor_layout(bonds_[k], bonds_[k + 2], twosite_phys_qn());
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  for (const Slab& ps : P.slabs) {
    int sa = a.lay.slab_of_left[ps.li];
    for (const auto& pb : ps.blocks) {
      int s1 = pb.phys / 4, s2 = pb.phys % 4;
      int ib = (int)items.size();
      if (sa >= 0) {
        const Slab& as = a.lay.slabs[sa];
        for (const auto& ab : as.blocks) {
          if (ab.phys != s1) continue;
          int sbi = b.lay.slab_of_left[ab.ri];
          if (sbi < 0) continue;
          const Slab& bs = b.lay.slabs[sbi];
          int bb = bs.block_of(s2, pb.ri);
          if (bb < 0) continue;
          items.push_back({a.buf.as<double>() + as.off + ab.col0, b.buf.as<double>() + bs.off + bs.blocks[bb].col0,
                           as.width, bs.width, ab.mr, 0, 1.0});
        }
      }
      tile_units(units, out + ps.off + pb.col0, ps.width, ps.ml, pb.mr, ib, (int)items.size());
    }
  }
  gemm_once(GEMM_NN, items, units);
}

// ---------------------------------------------------------------- Davidson --
// Block Davidson for the n_states lowest roots of H_eff (fp64 basis, subspace
// matrix, Rayleigh-Ritz and residuals).  With a low-precision sigma the basis
// is expanded with low-precision products; convergence is only declared on the
// fp64 residual of the Ritz vectors (defect correction: on a stall or on low-
// precision convergence the Ritz vectors' fp64 sigma replaces the subspace).
// Olsen's correction (the preconditioner family of the two-site Davidson, Sec.
// III): with q_r = -(D - theta)^-1 r (in t on entry) and q_x = -(D - theta)^-1 x,
// t = q_r - (x.q_r / x.q_x) q_x: the diagonal correction less its part along
// (D - theta)^-1 x, which for a nearly converged root only re-adds x.
void Solver::olsen(const double* x, const double* D, const double* theta, double* t) {
  const long n = psi_lay_.size;
  double* qx = dv_pcg_.as<double>();
  double* sc = dv_sc_.as<double>();
  double* part = dv_part_.as<double>();
  launch_precond_diag(x, D, theta, qx, n, st);
  launch_dots(x, n, 1, t, n, part, sc + 192, st);
  launch_dots(x, n, 1, qx, n, part, sc + 193, st);
  launch_axpy_ratio(t, qx, sc + 192, sc + 193, -1.0, n, st);
}

// Shift-and-invert correction (the inner-PCG member of that family, Sec. III): a
// few preconditioned conjugate-gradient steps on the projected correction
// equation (1 - x x^T)(theta - H)(1 - x x^T) t = r, t orthogonal to x, with the
// projected diagonal (theta - D)^-1 as preconditioner.  Both are negative
// definite near the lowest root, where CG runs as on the positive pair; H - theta
// is indefinite away from it, so a direction of non-negative curvature p.(theta -
// H)p (or a non-negative rho) ends the iteration (the guard), and if that happens
// on the first step the projected diagonal correction is taken.  Stops at
// pcg_rtol |r| or after pcg_steps steps.  Returns the products made.
template <class Apply>
int Solver::shift_invert(const double* x, const double* r, const double* D, const double* theta, double rnorm,
                         double* t, int prec, Apply& apply) {
  const int kInner = opt_.pcg_steps;
  const long n = psi_lay_.size;
  double* res = dv_pcg_.as<double>();
  double* z = res + n;
  double* p = res + 2 * n;
  double* w = res + 3 * n;
  double* sc = dv_sc_.as<double>();
  double* part = dv_part_.as<double>();
  auto project = [&](double* v) {  // v -= (x.v) x
    launch_dots(x, n, 1, v, n, part, sc + 195, st);
    launch_axpy_dev(v, x, sc + 195, -1.0, n, st);
  };
  launch_fill(t, n, 0.0, st);
  launch_copy(res, r, n, st);
  project(res);
  launch_precond_diag(res, D, theta, z, n, st);  // (theta - D)^-1 res
  project(z);
  launch_dots(res, n, 1, z, n, part, sc + 192, st);  // rho = res.z
  launch_copy(p, z, n, st);
  int mv = 0;
  double h[2];
  for (int j = 0; j < kInner; ++j) {
    apply(prec, p, w);
    ++mv;
    launch_axpy_dev(w, p, theta, -1.0, n, st);  // w = (H - theta) p
    project(w);
    launch_dots(p, n, 1, w, n, part, sc + 193, st);  // p.(H - theta)p
    hip_check(hipMemcpyAsync(h, sc + 192, 16, hipMemcpyDeviceToHost, st), "pcg");
    hip_check(hipStreamSynchronize(st), "pcg");
    if (!(h[1] > 0.0) || !(h[0] < 0.0)) {  // the guard: not a descent pair
      if (j == 0) launch_copy(t, z, n, st);
      break;
    }
    // alpha = rho / p.(theta - H)p = -rho / p.w; t += alpha p; res -= alpha (theta - H)p = res + alpha w
    launch_axpy_ratio(t, p, sc + 192, sc + 193, -1.0, n, st);
    launch_axpy_ratio(res, w, sc + 192, sc + 193, -1.0, n, st);
    if (j + 1 == kInner) break;
    launch_dots(res, n, 1, res, n, part, sc + 196, st);
    double rr;
    hip_check(hipMemcpyAsync(&rr, sc + 196, 8, hipMemcpyDeviceToHost, st), "pcg");
    hip_check(hipStreamSynchronize(st), "pcg");
    if (std::sqrt(std::max(rr, 0.0)) <= opt_.pcg_rtol * rnorm) break;
    launch_precond_diag(res, D, theta, z, n, st);
    project(z);
    launch_dots(res, n, 1, z, n, part, sc + 194, st);  // rho'
    launch_xpby_ratio(p, z, sc + 194, sc + 192, n, st);  // p = z + (rho'/rho) p
    launch_copy(sc + 192, sc + 194, 1, st);
  }
  return mv;
}

// One correction of the preconditioner family outside a solve: x the Ritz
// vector (unit norm), r its residual, d the diagonal of H_eff, theta the Ritz
// value; the shift-and-invert products are the fp64 sigma of step k.
int Solver::correction_host_theta(int k, int mode, const double* x, const double* r, const double* d,
                                  double theta, double* t) {
  if (plan_k_ != k) prepare(k);
  const long n = psi_lay_.size;
  dv_sc_.reserve(256 * 8);
  dv_part_.reserve((size_t)512 * 64 * 8);
  dv_pcg_.reserve((size_t)4 * n * 8);
  double* sc = dv_sc_.as<double>();
  hip_check(hipMemcpyAsync(sc + 203, &theta, 8, hipMemcpyHostToDevice, st), "theta");
  launch_precond_diag(r, d, sc + 203, t, n, st);
  int mv = 0;
  if (mode == 2) olsen(x, d, sc + 203, t);
  if (mode == 3) {
    launch_dots(r, n, 1, r, n, dv_part_.as<double>(), sc + 204, st);
    double rr;
    hip_check(hipMemcpyAsync(&rr, sc + 204, 8, hipMemcpyDeviceToHost, st), "rnorm");
    hip_check(hipStreamSynchronize(st), "rnorm");
    auto apply = [&](int p, const double* a, double* b) { sigma(k, p, a, b); };
    mv = shift_invert(x, r, d, sc + 203, std::sqrt(std::max(rr, 0.0)), t, PREC_F64, apply);
  }
  hip_check(hipStreamSynchronize(st), "correction");
  return mv;
}

int Solver::davidson(int k, std::vector<DevMem>& guess, std::vector<double>& evals) {
  if (plan_k_ != k) prepare(k);
  const auto td0 = std::chrono::steady_clock::now();
  struct WallTimer {
    std::chrono::steady_clock::time_point t0;
    double* acc;
    ~WallTimer() { *acc += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); }
  } wall_timer{td0, &st_.davidson_ms};
  const long n = psi_lay_.size;
  const int nr = opt_.n_states;
  const int kmax = std::min<long>(opt_.max_subspace, std::max<long>(n, 1));
  DMRG_REQUIRE(n >= nr, ST_ESECTOR, "two-site space smaller than the number of states");
  dv_V_.reserve((size_t)kmax * n * 8);
  dv_AV_.reserve((size_t)kmax * n * 8);
  dv_G_.reserve((size_t)64 * 64 * 8);
  dv_evals_.reserve(64 * 8);
  dv_evecs_.reserve(64 * 64 * 8);
  dv_X_.reserve((size_t)nr * n * 8);
  dv_R_.reserve((size_t)nr * n * 8);
  dv_C_.reserve((size_t)nr * n * 8);
  dv_t_.reserve((size_t)n * 8);
  dv_diag_.reserve((size_t)n * 8);
  dv_part_.reserve((size_t)512 * 64 * 8);
  dv_sc_.reserve(256 * 8);
  if (precond_ == 2 || precond_ == 3) dv_pcg_.reserve((size_t)4 * n * 8);
  double* V = dv_V_.as<double>();
  double* AV = dv_AV_.as<double>();
  double* G = dv_G_.as<double>();
  double* ev = dv_evals_.as<double>();
  double* evec = dv_evecs_.as<double>();
  double* X = dv_X_.as<double>();
  double* R = dv_R_.as<double>();
  double* Cc = dv_C_.as<double>();
  double* t = dv_t_.as<double>();
  double* D = dv_diag_.as<double>();
  double* part = dv_part_.as<double>();
  double* sc = dv_sc_.as<double>();
  const int ldg = 64;
  diag(k, D);
  const int prec = opt_.precision;
  int kcur = 0, matvecs = 0;
  // penalty deflation (Sec. II.F): the operator is H_eff + Phi Phi^T with the
  // projected lower states as the columns of Phi (scaled by sqrt(w_j) / ||Phi_j||),
  // added in fp64 to every product; the preconditioner's diagonal includes it
  const int nd = (int)defl_.size();
  double* Phi = nullptr;
  if (nd > 0) {
    defl_phi_.reserve((size_t)nd * n * 8);
    Phi = defl_phi_.as<double>();
    for (int j = 0; j < nd; ++j) deflate_project(k, j, std::sqrt(defl_[j].w) / defl_[j].norm, Phi + (long)j * n);
    launch_add_squares(D, Phi, n, nd, n, st);
  }
  auto apply = [&](int p, const double* x, double* y) {
    sigma(k, p, x, y);
    if (nd > 0) {
      launch_dots(Phi, n, nd, x, n, part, sc + 128, st);
      launch_gemv(Phi, n, nd, sc + 128, 1.0, y, 1.0, n, st);
    }
    if (onesite_) onesite_project(k, y);
  };

  auto host_scalar = [&](const double* dptr) {
    double v;
    hip_check(hipMemcpyAsync(&v, dptr, 8, hipMemcpyDeviceToHost, st), "scalar");
    hip_check(hipStreamSynchronize(st), "scalar");
    return v;
  };
  // orthonormalise t against V[0..kcur) (two passes of classical Gram-Schmidt), append
  // min_ratio: smallest accepted |t after projection|^2 / |t|^2
  // error of each subspace column's product, in units of the low-precision
  // sigma error per unit vector (0: fp64 product); rotations propagate it as
  // independent errors (square root of the sum of squares)
  std::vector<double> colerr(64, 0.0);
  // Row i of the subspace matrix, G_ji = v_j . A v_i for j <= i.  H is
  // symmetric, so the entry can also be formed as (A v_j) . v_i; with
  // low-precision products the more accurate of the two columns' products is
  // used, so couplings to fp64 columns (the roots after a refinement) are exact.
  std::vector<double> gtmp(128);
  auto gcol = [&](int i) {
    launch_dots(V, n, i + 1, AV + (long)i * n, n, part, G + (long)i * ldg, st);
    bool mixed = false;
    for (int j = 0; j <= i; ++j) mixed = mixed || colerr[j] < colerr[i];
    if (!mixed) return;
    launch_dots(AV, n, i + 1, V + (long)i * n, n, part, sc + 64, st);
    hip_check(hipMemcpyAsync(gtmp.data(), G + (long)i * ldg, (i + 1) * 8, hipMemcpyDeviceToHost, st), "g row");
    hip_check(hipMemcpyAsync(gtmp.data() + 64, sc + 64, (i + 1) * 8, hipMemcpyDeviceToHost, st), "g row");
    hip_check(hipStreamSynchronize(st), "g row");
    for (int j = 0; j <= i; ++j)
      if (colerr[j] < colerr[i]) gtmp[j] = gtmp[64 + j];
    hip_check(hipMemcpyAsync(G + (long)i * ldg, gtmp.data(), (i + 1) * 8, hipMemcpyHostToDevice, st), "g row");
    hip_check(hipStreamSynchronize(st), "g row");
  };
  auto append = [&](const double* src, int sprec, double min_ratio = 1e-20) -> bool {
    if (src != t) launch_copy(t, src, n, st);
    launch_dots(t, n, 1, t, n, part, sc + 1, st);
    for (int pass = 0; pass < 2 && kcur > 0; ++pass) {
      launch_dots(V, n, kcur, t, n, part, sc + 8, st);
      launch_gemv(V, n, kcur, sc + 8, -1.0, t, 1.0, n, st);
    }
    launch_dots(t, n, 1, t, n, part, sc, st);
    // both squared norms in one read (t is scratch: a rejected candidate leaves
    // V and AV untouched)
    double nq[2];
    hip_check(hipMemcpyAsync(nq, sc, 16, hipMemcpyDeviceToHost, st), "norms");
    hip_check(hipStreamSynchronize(st), "norms");
    const double nn = nq[0], n0 = nq[1];
    if (!(n0 > 0) || !std::isfinite(n0)) return false;
    if (!(nn > min_ratio * n0) || !std::isfinite(nn)) return false;
    launch_scale_by_norm(t, n, sc, st);
    launch_copy(V + (long)kcur * n, t, n, st);
    apply(sprec, V + (long)kcur * n, AV + (long)kcur * n);
    ++matvecs;
    colerr[kcur] = sprec == PREC_F64 ? 0.0 : 1.0;
    gcol(kcur);
    ++kcur;
    return true;
  };

  for (int r = 0; r < nr && r < (int)guess.size(); ++r) append(guess[r].as<double>(), PREC_F64);
  if (kcur < nr) {  // fill with unit vectors at the lowest diagonal entries
    std::vector<double> hd(n);
    hip_check(hipMemcpy(hd.data(), D, n * 8, hipMemcpyDeviceToHost), "diag");
    std::vector<long> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](long a, long b) { return hd[a] < hd[b]; });
    for (long j = 0; j < n && kcur < nr; ++j) {
      std::vector<double> e(n, 0.0);
      e[idx[j]] = 1.0;
      hip_check(hipMemcpy(t, e.data(), n * 8, hipMemcpyHostToDevice), "unit");
      append(t, PREC_F64);
    }
  }
  DMRG_REQUIRE(kcur >= nr, ST_ESECTOR, "could not build an initial Davidson basis");
  // learned preconditioner: judged by the exact residual, the diagonal one is the fallback
  bool lrn_on = precond_ == 1;
  DMRG_REQUIRE(!lrn_on || net_, ST_ESTATE, "learned preconditioner selected without a network");
  int lw_count = 0;
  double lw_r0 = 0.0;
  float* F = nullptr;
  float* Y = nullptr;
  double* Lc = nullptr;
  double* Tmp = nullptr;
  const bool rec = rec_cap_ > 0 && n >= rec_sample_ && rec_sample_ > 0;
  const int kRecHist = 64;
  std::vector<int> rec_slots;
  if (lrn_on || rec) {
    feat_.reserve((size_t)n * 8 * 4);
    nety_.reserve((size_t)n * 4);
    dv_L_.reserve((size_t)nr * n * 8);
    feat_t_.reserve((size_t)n * 8);
    fstats_.reserve((size_t)std::max(nfb_, 1) * 4 * 8);
    F = feat_.as<float>();
    Y = nety_.as<float>();
    Lc = dv_L_.as<double>();
    Tmp = feat_t_.as<double>();
  }
  if (rec) {  // this step's amplitude sample: a seeded draw without replacement
    rec_hist_.reserve((size_t)kRecHist * n * 8);
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    uint64_t z = 0x9E3779B97F4A7C15ull * (++rec_seed_ + 1);
    for (int j = 0; j < rec_sample_; ++j) {
      z ^= z >> 33;
      z *= 0xff51afd7ed558ccdull;
      z ^= z >> 33;
      z = z * 0xc4ceb9fe1a85ec53ull + (uint64_t)j;
      long pick = j + (long)(z % (uint64_t)(n - j));
      std::swap(idx[j], idx[pick]);
    }
    rec_idx_.reserve((size_t)rec_sample_ * 8);
    hip_check(hipMemcpyAsync(rec_idx_.p, idx.data(), (size_t)rec_sample_ * 8, hipMemcpyHostToDevice, st), "sample");
    hip_check(hipStreamSynchronize(st), "sample");
  }
  evals.assign(nr, 0.0);
  std::vector<double> rn(nr, 0.0), hv(2 * nr);
  int iter = 0;
  // Precision form (defect correction).  The start vectors get fp64 products
  // and one low-precision product of the first of them measures delta, the
  // low-precision sigma error per unit vector at this step.  New directions get
  // low-precision products; the error of a Ritz vector's product is then
  // delta * sqrt(sum_j y_j^2 colerr_j^2) over its coefficients y.  While the
  // residual estimate is far above that error the iteration is plain Davidson.
  // When it comes within kNear of it (or below tol), the subspace is rotated
  // to its lowest Ritz vectors and the roots' vectors get fp64 products
  // (refinement): their residuals are exact again, and the other kept vectors'
  // errors enter later Ritz vectors only through small coefficients.
  // Convergence is declared only on a residual whose error bound is below
  // tol / 10.  Two refinements that do not halve the exact residual end the low
  // precision for this step (the rest is fp64).
  const double kNear = 10.0;
  int sprec = prec;  // precision of new sigma products
  double delta = 0.0;
  if (sprec != PREC_F64) {
    const double one = 1.0;
    hip_check(hipMemcpyAsync(sc + 40, &one, 8, hipMemcpyHostToDevice, st), "one");
    apply(sprec, V, t);
    ++matvecs;
    launch_axpy_dev(t, AV, sc + 40, -1.0, n, st);  // t - 1 * AV[0] (sc[40] = 1)
    launch_dots(t, n, 1, t, n, part, sc + 41, st);
    delta = std::sqrt(std::max(0.0, host_scalar(sc + 41)));
  }
  double r_last_ref = -1.0;  // exact residual after the last refinement
  int bad_refs = 0;
  bool after_ref = false;
  std::vector<double> hy((size_t)64 * 64);
  auto rotate_keep = [&](int keep) {
    // V, AV <- the lowest `keep` Ritz vectors (in place); errors propagate
    hip_check(hipMemcpyAsync(hy.data(), evec, (size_t)kcur * keep * 8, hipMemcpyDeviceToHost, st), "evecs");
    launch_subspace_rotate(V, n, kcur, evec, keep, n, st);
    launch_subspace_rotate(AV, n, kcur, evec, keep, n, st);
    hip_check(hipStreamSynchronize(st), "rotate");
    std::vector<double> ne(keep, 0.0);
    for (int i = 0; i < keep; ++i) {
      double acc = 0;
      for (int j = 0; j < kcur; ++j) acc += hy[(size_t)i * kcur + j] * hy[(size_t)i * kcur + j] * colerr[j] * colerr[j];
      ne[i] = std::sqrt(acc);
    }
    for (int i = 0; i < keep; ++i) colerr[i] = ne[i];
    for (int i = 0; i < keep; ++i) gcol(i);
    kcur = keep;
  };
  // refinement: rotate to the lowest Ritz vectors, fp64 products for the roots'
  auto refine = [&]() {
    const int keep = std::min(kcur, std::min(16, std::max(nr + 2, kmax / 3)));
    rotate_keep(keep);
    for (int i = 0; i < nr; ++i) {
      apply(PREC_F64, V + (long)i * n, AV + (long)i * n);
      ++matvecs;
      colerr[i] = 0.0;
    }
    for (int i = 0; i < keep; ++i) gcol(i);
    st_.refinements++;
    after_ref = true;
  };
  int conv = 0;
  for (; iter < opt_.max_iter; ++iter) {
    launch_jacobi_eig(G, ldg, kcur, ev, evec, st);
    for (int i = 0; i < nr; ++i) {
      launch_gemv(V, n, kcur, evec + (long)i * kcur, 1.0, X + (long)i * n, 0.0, n, st);
      launch_gemv(AV, n, kcur, evec + (long)i * kcur, 1.0, R + (long)i * n, 0.0, n, st);
      launch_axpy_dev(R + (long)i * n, X + (long)i * n, ev + i, -1.0, n, st);
      launch_dots(R + (long)i * n, n, 1, R + (long)i * n, n, part, sc + 16 + i, st);
    }
    hip_check(hipMemcpyAsync(hv.data(), ev, nr * 8, hipMemcpyDeviceToHost, st), "evals");
    hip_check(hipMemcpyAsync(hv.data() + nr, sc + 16, nr * 8, hipMemcpyDeviceToHost, st), "rnorm");
    if (delta > 0) hip_check(hipMemcpyAsync(hy.data(), evec, (size_t)kcur * nr * 8, hipMemcpyDeviceToHost, st), "evecs");
    hip_check(hipStreamSynchronize(st), "davidson");
    double rmax = 0, errmax = 0;
    for (int i = 0; i < nr; ++i) {
      evals[i] = hv[i];
      rn[i] = std::sqrt(std::max(0.0, hv[nr + i]));
      rmax = std::max(rmax, rn[i]);
      if (delta > 0) {
        double acc = 0;
        for (int j = 0; j < kcur; ++j) acc += hy[(size_t)i * kcur + j] * hy[(size_t)i * kcur + j] * colerr[j] * colerr[j];
        errmax = std::max(errmax, delta * std::sqrt(acc));
      }
    }
    if (opt_.verbose > 1)
      fprintf(stderr, "  dav k=%d it=%d sub=%d E=%.12f r=%.3e err=%.1e prec=%d\n", k, iter, kcur, evals[0], rmax,
              errmax, sprec);
    if (onesite_ && iter == 0) first_res_ = std::max(first_res_, rmax);  // the local tangent gradient
    if (!std::isfinite(rmax)) throw Error(ST_ENOCONV, "non-finite Davidson residual");
    if (after_ref) {  // the roots' residuals are exact: judge the refinement
      after_ref = false;
      if (r_last_ref > 0 && rmax > 0.5 * r_last_ref && ++bad_refs >= 2) sprec = PREC_F64;
      r_last_ref = rmax;
    }
    if (errmax <= 0.1 * opt_.davidson_tol) {
      if (rmax <= opt_.davidson_tol) {
        conv = 1;
        break;
      }
    } else if (rmax <= opt_.davidson_tol || rmax <= kNear * errmax) {
      refine();
      continue;
    }
    // training triple of root 0: features now, target once the step has converged
    if (rec && rn[0] > opt_.davidson_tol && (int)rec_slots.size() < kRecHist &&
        rec_count_ + (int)rec_slots.size() < rec_cap_) {
      const int slot = rec_count_ + (int)rec_slots.size();
      launch_precond_diag(R, D, ev, Tmp, n, st);
      features(R, D, ev, Tmp, F);
      launch_gather_rows(F, 8, rec_idx_.as<int64_t>(), rec_sample_, rec_X_.as<float>() + (size_t)slot * rec_sample_ * 8, st);
      launch_copy(rec_hist_.as<double>() + (size_t)rec_slots.size() * n, X, n, st);
      rec_slots.push_back(slot);
    }
    // learned candidates: stop using them when 3 iterations cut |r| by less than 10%
    if (lrn_on) {
      if (lw_count == 0) {
        lw_r0 = rmax;
      } else if (lw_count >= 3) {
        if (rmax > 0.9 * lw_r0) {
          lrn_on = false;
          st_.fallbacks++;
        } else {
          lw_count = 0;
          lw_r0 = rmax;
        }
      }
      if (lrn_on) ++lw_count;
    }
    // corrections from the residuals of unconverged roots
    int nnew = 0;
    for (int i = 0; i < nr; ++i) {
      if (rn[i] <= opt_.davidson_tol) continue;
      launch_precond_diag(R + (long)i * n, D, ev + i, Cc + (long)nnew * n, n, st);
      if (precond_ == 2) olsen(X + (long)i * n, D, ev + i, Cc + (long)nnew * n);
      else if (precond_ == 3) matvecs += shift_invert(X + (long)i * n, R + (long)i * n, D, ev + i, rn[i],
                                                      Cc + (long)nnew * n, sprec, apply);
      if (lrn_on) {
        features(R + (long)i * n, D, ev + i, Cc + (long)nnew * n, F);
        net_->forward(PREC_BF16, F, n, Y, st);
        launch_f32_to_f64(Y, Lc + (long)nnew * n, n, st);
        if (onesite_) onesite_project(k, Lc + (long)nnew * n);
      }
      if (onesite_) onesite_project(k, Cc + (long)nnew * n);
      ++nnew;
    }
    if (kcur + nnew > kmax) {
      // thick restart: keep the lowest Ritz vectors, more than the roots, so a
      // near-degenerate neighbour of the last root is not lost at every restart
      rotate_keep(std::min(kcur, std::min(16, std::max(nr + 2, kmax / 3))));
    }
    int added = 0;
    for (int j = 0; j < nnew; ++j) {
      if (lrn_on) {  // rejected: non-finite, or (almost) inside the current subspace
        if (append(Lc + (long)j * n, sprec, 1e-6)) {
          ++added;
          continue;
        }
        st_.fallbacks++;
      }
      if (append(Cc + (long)j * n, sprec)) ++added;
    }

    if (added == 0) {
      if (errmax > 0.1 * opt_.davidson_tol) {  // nothing new to add on inexact products
        sprec = PREC_F64;
        refine();
        continue;
      }
      conv = rmax <= 1e3 * opt_.davidson_tol;
      break;
    }
  }
  st_.davidson_iters += iter;
  if (!conv) {
    st_.converged = 0;
    if (opt_.verbose)
      fprintf(stderr, "  davidson k=%d not converged: %d iterations, subspace %d, residuals", k, iter, kcur);
    if (opt_.verbose) {
      for (int i = 0; i < nr; ++i) fprintf(stderr, " %.3e", rn[i]);
      fprintf(stderr, " (tol %.1e, n %ld)\n", opt_.davidson_tol, n);
    }
  }
  last_converged_ = conv != 0;
  if (rec && conv && !rec_slots.empty()) {  // Delta = P_perp psi*, psi* oriented along psi_i
    for (size_t j = 0; j < rec_slots.size(); ++j) {
      const double* hj = rec_hist_.as<double>() + j * n;
      launch_dots(hj, n, 1, X, n, part, sc + 210, st);
      launch_triple_target(hj, X, sc + 210, rec_idx_.as<int64_t>(), rec_sample_,
                           rec_T_.as<float>() + (size_t)rec_slots[j] * rec_sample_, st);
    }
    hip_check(hipStreamSynchronize(st), "triples");
    rec_count_ += (int)rec_slots.size();
  }
  if (nd > 0) {  // energies of H: theta_r - sum_j (Phi_j . x_r)^2
    std::vector<double> c((size_t)nd);
    for (int i = 0; i < nr; ++i) {
      launch_dots(Phi, n, nd, X + (long)i * n, n, part, sc + 160, st);
      hip_check(hipMemcpyAsync(c.data(), sc + 160, (size_t)nd * 8, hipMemcpyDeviceToHost, st), "deflation");
      hip_check(hipStreamSynchronize(st), "deflation");
      for (int j = 0; j < nd; ++j) evals[i] -= c[j] * c[j];
    }
  }
  // converged Ritz vectors are in X
  return matvecs;
}

// ----------------------------------------------------------------- SVD step --
// Reshape psi to (a s1) x (s2 b); it is block diagonal in the middle-bond
// sector q_m = q_a + q_s1.  One fp64 SVD per sector (state-averaged: of the
// weighted concatenation of the roots), global truncation with the cluster rule,
// new site tensors and next-step guesses.
void Solver::svd_step(int k, bool l2r, int nr, std::vector<DevMem>& next_guess, double& tau) {
  const TensorLayout& P = psi_lay_;
  const Bond& bk = bonds_[k];
  const Bond& bk2 = bonds_[k + 2];
  const long n = P.size;
  struct Part { int idx, dim; long off; };
  struct Mid { QN q; std::vector<Part> rows, cols; int R = 0, C = 0; };
  std::vector<Mid> mids;
  auto mid_of = [&](QN q) {
    for (size_t i = 0; i < mids.size(); ++i)
      if (mids[i].q == q) return (int)i;
    mids.push_back({q, {}, {}, 0, 0});
    return (int)mids.size() - 1;
  };
  for (const Slab& sl : P.slabs)
    for (const auto& b : sl.blocks) mid_of(bk.sec[sl.li].q + site_qn(b.phys / 4));
  std::sort(mids.begin(), mids.end(), [](const Mid& a, const Mid& b) { return a.q < b.q; });
  for (Mid& m : mids) {
    for (int s1 = 0; s1 < 4; ++s1) {
      int li = bk.find(m.q - site_qn(s1));
      if (li < 0 || P.slab_of_left[li] < 0) { m.rows.push_back({li, 0, m.R}); continue; }
      m.rows.push_back({li, bk.sec[li].dim, m.R});
      m.R += bk.sec[li].dim;
    }
    for (int s2 = 0; s2 < 4; ++s2) {
      int ri = bk2.find(m.q + site_qn(s2));
      if (ri < 0) { m.cols.push_back({ri, 0, m.C}); continue; }
      m.cols.push_back({ri, bk2.sec[ri].dim, m.C});
      m.C += bk2.sec[ri].dim;
    }
  }
  // gather: per-root sector matrices Psi_r (column-major, R x C)
  long tot_plain = 0;
  std::vector<long> off_plain(mids.size());
  for (size_t i = 0; i < mids.size(); ++i) {
    off_plain[i] = tot_plain;
    tot_plain += (long)mids[i].R * mids[i].C * nr;
  }
  DevMem plain, gram, evals, info, Uv, Vv;
  plain.reserve(std::max<long>(tot_plain, 1) * 8);
  std::vector<int64_t> desc_plain;
  for (size_t mi = 0; mi < mids.size(); ++mi) {
    const Mid& m = mids[mi];
    for (int s1 = 0; s1 < 4; ++s1) {
      const Part& rp = m.rows[s1];
      if (rp.dim == 0) continue;
      const Slab& sl = P.slabs[P.slab_of_left[rp.idx]];
      for (int s2 = 0; s2 < 4; ++s2) {
        const Part& cp = m.cols[s2];
        if (cp.dim == 0) continue;
        int b = sl.block_of(4 * s1 + s2, cp.idx);
        if (b < 0) continue;
        for (int r = 0; r < nr; ++r) {
          long src = (long)r * n + sl.off + sl.blocks[b].col0;
          long dst = off_plain[mi] + (long)r * m.R * m.C + rp.off + (long)cp.off * m.R;
          desc_plain.insert(desc_plain.end(), {src, sl.width, 1, dst, 1, m.R, rp.dim, cp.dim, dbits(1.0)});
        }
      }
    }
  }
  check_desc(desc_plain, 0, desc_plain.size(), (long)nr * n, tot_plain);
  launch_fill(plain.as<double>(), tot_plain, 0.0, st);
  DevMem dd;
  dd.reserve(desc_plain.size() * 8 + 8);
  hip_check(hipMemcpyAsync(dd.p, desc_plain.data(), desc_plain.size() * 8, hipMemcpyHostToDevice, st), "svd desc");
  launch_copy_blocks(dd.as<int64_t>(), (int)(desc_plain.size() / 9), dv_X_.as<double>(), plain.as<double>(), st);
  // Density matrix of the sector (the reduced density matrix of the kept side):
  // moving right G = sum_r w_r Psi_r Psi_r^T (R x R), moving left sum_r w_r Psi_r^T Psi_r
  // (C x C).  Its eigenvalues are the squared singular values of the weighted
  // concatenation and its eigenvectors the kept singular vectors.  Sectors are
  // padded with zeros into size buckets, one batched eigensolve per bucket.
  auto bucket_of = [](int d) { return d <= 64 ? std::max(8, (d + 7) / 8 * 8) : (d + 63) / 64 * 64; };
  std::vector<int> gd(mids.size()), gb(mids.size());
  std::map<int, std::vector<int>> buckets;
  for (size_t i = 0; i < mids.size(); ++i) {
    gd[i] = l2r ? mids[i].R : mids[i].C;
    gb[i] = bucket_of(std::max(gd[i], 1));
    buckets[gb[i]].push_back((int)i);
  }
  std::vector<long> goff(mids.size()), eoff(mids.size());
  long gtot = 0, etot = 0;
  for (auto& bk_ : buckets)
    for (int i : bk_.second) {
      goff[i] = gtot;
      gtot += (long)gb[i] * gb[i];
      eoff[i] = etot;
      etot += gb[i];
    }
  gram.reserve(std::max<long>(gtot, 1) * 8);
  evals.reserve(std::max<long>(etot, 1) * 8 * 2);
  info.reserve((mids.size() + 1) * sizeof(rocblas_int));
  launch_fill(gram.as<double>(), gtot, 0.0, st);
  // Padding rows/columns of a bucket get -4 on the diagonal: with normalised roots
  // and weights summing to one every true eigenvalue lies in [0, 1], so padding
  // eigenpairs sort below all of them and are never taken as kept vectors.
  static const double kPad = -4.0;
  DevMem pad_src, pad_desc;
  std::vector<int64_t> pdesc;
  for (size_t i = 0; i < mids.size(); ++i)
    if (gb[i] > gd[i]) {
      long d0 = goff[i] + (long)gd[i] * gb[i] + gd[i];
      pdesc.insert(pdesc.end(), {0, 0, 0, d0, gb[i] + 1, 0, gb[i] - gd[i], 1, dbits(1.0)});
    }
  if (!pdesc.empty()) {
    check_desc(pdesc, 0, pdesc.size(), 1, gtot);
    pad_src.reserve(8);
    pad_desc.reserve(pdesc.size() * 8);
    hip_check(hipMemcpyAsync(pad_src.p, &kPad, 8, hipMemcpyHostToDevice, st), "pad value");
    hip_check(hipMemcpyAsync(pad_desc.p, pdesc.data(), pdesc.size() * 8, hipMemcpyHostToDevice, st), "pad desc");
    launch_copy_blocks(pad_desc.as<int64_t>(), (int)(pdesc.size() / 9), pad_src.as<double>(), gram.as<double>(), st);
  }
  {
    std::vector<GemmItem> items;
    std::vector<GemmUnit> units;
    for (size_t i = 0; i < mids.size(); ++i) {
      const Mid& m = mids[i];
      if (m.R == 0 || m.C == 0) continue;
      int ib = (int)items.size();
      for (int r = 0; r < nr; ++r) {
        const double* Pr = plain.as<double>() + off_plain[i] + (long)r * m.R * m.C;
        // moving right: TN with K = C (A = B = Psi_r read as C x R row-major);
        // moving left: NT with K = R (A = B = Psi_r read as C x R row-major)
        items.push_back({Pr, Pr, m.R, m.R, l2r ? m.C : m.R, 0, opt_.weights[r]});
      }
      tile_units(units, gram.as<double>() + goff[i], gb[i], gd[i], gd[i], ib, (int)items.size());
    }
    gemm_once(l2r ? GEMM_TN : GEMM_NT, items, units);
  }
  // one bucket per auxiliary stream, joined back into the solver stream
  if (!aux_st_[0]) {
    for (int i = 0; i < kAuxStreams; ++i) {
      hip_check(hipStreamCreateWithFlags(&aux_st_[i], hipStreamNonBlocking), "aux stream");
      if (rocblas_create_handle(&aux_rb_[i]) != rocblas_status_success) throw Error(ST_EHIP, "rocblas handle");
      rocblas_set_stream(aux_rb_[i], aux_st_[i]);
    }
    for (hipEvent_t& e : aux_ev_) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "aux event");
  }
  hip_check(hipEventRecord(aux_ev_[kAuxStreams], st), "eigensolve fork");
  for (int i = 0; i < kAuxStreams; ++i) hip_check(hipStreamWaitEvent(aux_st_[i], aux_ev_[kAuxStreams], 0), "fork");
  {
    int bi = 0;
    long info_off = 0;
    for (auto& bk_ : buckets) {
      int nbk = bk_.first;
      int first = bk_.second[0];
      rocblas_handle hb = aux_rb_[bi % kAuxStreams];
      auto call = [&]() {
        return rocsolver_dsyevd_strided_batched(
            hb, rocblas_evect_original, rocblas_fill_upper, nbk, gram.as<double>() + goff[first], nbk,
            (rocblas_stride)nbk * nbk, evals.as<double>() + eoff[first], nbk, evals.as<double>() + etot + eoff[first],
            nbk, info.as<rocblas_int>() + info_off, (rocblas_int)bk_.second.size());
      };
      if (current_arena()) {
        // in an arena the handle's device workspace comes from it too: size query, then attach
        size_t need = 0;
        if (rocblas_start_device_memory_size_query(hb) != rocblas_status_success)
          throw Error(ST_EHIP, "rocBLAS workspace size query");
        (void)call();
        if (rocblas_stop_device_memory_size_query(hb, &need) != rocblas_status_success)
          throw Error(ST_EHIP, "rocBLAS workspace size query");
        DevMem& w = rb_work_[bi % kAuxStreams];
        if (need > w.bytes || !w.p) {
          hip_check(hipStreamSynchronize(aux_st_[bi % kAuxStreams]), "rocBLAS workspace");
          w.reserve(std::max<size_t>(need, 1 << 20));
          if (rocblas_set_workspace(hb, w.p, w.bytes) != rocblas_status_success)
            throw Error(ST_EHIP, "rocblas_set_workspace");
        }
      }
      rocblas_status rs = call();
      if (rs != rocblas_status_success) throw Error(ST_EHIP, "rocsolver_dsyevd_strided_batched failed");
      info_off += (long)bk_.second.size();
      ++bi;
    }
  }
  for (int i = 0; i < kAuxStreams; ++i) {
    hip_check(hipEventRecord(aux_ev_[i], aux_st_[i]), "join");
    hip_check(hipStreamWaitEvent(st, aux_ev_[i], 0), "join");
  }
  std::vector<double> E(etot);
  std::vector<rocblas_int> einfo(mids.size());
  hip_check(hipMemcpyAsync(E.data(), evals.p, etot * 8, hipMemcpyDeviceToHost, st), "eigenvalues");
  hip_check(hipMemcpyAsync(einfo.data(), info.p, mids.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost, st),
            "eigensolve info");
  hip_check(hipStreamSynchronize(st), "eigensolve");
  for (size_t i = 0; i < mids.size(); ++i)
    if (einfo[i] != 0)
      throw Error(ST_EHIP, "rocsolver_dsyevd did not converge for a density matrix (info " +
                               std::to_string(einfo[i]) + ")");
  // singular values per sector, descending: the largest gd eigenvalues of each padded block
  std::vector<long> oS(mids.size());
  std::vector<int> kk(mids.size());
  std::vector<double> S;
  for (size_t i = 0; i < mids.size(); ++i) {
    kk[i] = (mids[i].R == 0 || mids[i].C == 0) ? 0 : std::min(gd[i], l2r ? nr * mids[i].C : nr * mids[i].R);
    oS[i] = (long)S.size();
    for (int t = 0; t < kk[i]; ++t) S.push_back(std::sqrt(std::max(0.0, E[eoff[i] + gb[i] - 1 - t])));
  }
  const long sS = (long)S.size();
  // global truncation with the cluster rule
  struct SV { double s; int mid, j; };
  std::vector<SV> all_sv;
  for (size_t i = 0; i < mids.size(); ++i)
    for (int j = 0; j < kk[i]; ++j) all_sv.push_back({S[oS[i] + j], (int)i, j});
  std::stable_sort(all_sv.begin(), all_sv.end(), [](const SV& a, const SV& b) { return a.s > b.s; });
  double s1 = all_sv.empty() ? 0.0 : all_sv[0].s;
  long keep = std::min<long>((long)all_sv.size(), opt_.M);
  // Adaptive bond dimension (dynamic block-state selection): the fewest states
  // whose discarded weight is at most trunc_tol of the total, at least m_min,
  // at most M; a cluster at such a cut is kept whole while M allows.
  if (opt_.trunc_tol > 0 && !all_sv.empty()) {
    double total = 0, tail = 0;
    for (const SV& v : all_sv) total += v.s * v.s;
    long kt = (long)all_sv.size();
    while (kt > 1 && tail + all_sv[kt - 1].s * all_sv[kt - 1].s <= opt_.trunc_tol * total) {
      tail += all_sv[kt - 1].s * all_sv[kt - 1].s;
      --kt;
    }
    kt = std::max<long>(kt, opt_.m_min);
    if (kt < keep) {
      keep = kt;
      while (keep < std::min<long>((long)all_sv.size(), opt_.M) &&
             all_sv[keep - 1].s - all_sv[keep].s <= opt_.tie_rtol * s1)
        ++keep;
    }
  }
  // Nothing is dropped while every state fits (the exact regime: singular values
  // from density-matrix eigenvalues resolve only down to ~1e-8 s_1, so a small
  // one cannot be told from a zero one, and keeping both is exact).  When states
  // must go, those at or below cut_rtol s_1 go first and a near-degenerate
  // cluster is never split.
  if (keep < (long)all_sv.size()) {
    while (keep > 0 && all_sv[keep - 1].s <= opt_.cut_rtol * s1) --keep;
    while (keep > 1 && all_sv[keep - 1].s - all_sv[keep].s <= opt_.tie_rtol * s1) --keep;
  }
  if (keep < 1) keep = 1;
  last_kept_sv_.resize(keep);
  for (long i = 0; i < keep; ++i) last_kept_sv_[i] = all_sv[i].s;
  tau = 0;
  for (size_t i = keep; i < all_sv.size(); ++i) tau += all_sv[i].s * all_sv[i].s;
  std::vector<int> kept(mids.size(), 0);
  for (long i = 0; i < keep; ++i) kept[all_sv[i].mid]++;
  // singular values within a sector are descending, so the kept ones are the first kept[i]
  Bond nb;
  std::vector<int> new_index(mids.size(), -1);
  for (size_t i = 0; i < mids.size(); ++i)
    if (kept[i] > 0) {
      new_index[i] = (int)nb.sec.size();
      nb.sec.push_back({mids[i].q, kept[i]});
    }
  st_.max_bond = std::max(st_.max_bond, nb.total());
  // Every buffer the new tensors need is reserved before the bond table and the
  // MPS change, so a failed allocation (DMRG_ENOMEM in a workspace) leaves the
  // state as it was.
  TensorLayout clay;  // center layout
  const long fixed_size = l2r ? make_tensor_layout(bonds_[k], nb, site_phys_qn()).size
                              : make_tensor_layout(nb, bonds_[k + 2], site_phys_qn()).size;
  clay = l2r ? make_tensor_layout(nb, bonds_[k + 2], site_phys_qn()) : make_tensor_layout(bonds_[k], nb, site_phys_qn());
  DevMem fresh_fixed;  // used when the tensor being replaced has too small an allocation
  if (mps_[l2r ? k : k + 1].buf.bytes < (size_t)std::max<long>(fixed_size, 1) * 8)
    fresh_fixed.reserve(std::max<long>(fixed_size, 1) * 8);
  centers_.resize(nr);
  for (int r = 0; r < nr; ++r) centers_[r].reserve(std::max<long>(clay.size, 1) * 8);
  {
    long su = 0;
    for (size_t i = 0; i < mids.size(); ++i)
      if (kept[i] > 0) su += (long)(l2r ? mids[i].R : mids[i].C) * kept[i];
    (l2r ? Uv : Vv).reserve(std::max<long>(su, 1) * 8);
  }
  DevMem fresh_center;  // the centre site's new tensor, when its allocation is too small
  {
    const long other = make_tensor_layout(l2r ? nb : bonds_[k], l2r ? bonds_[k + 2] : nb, site_phys_qn()).size;
    if (mps_[l2r ? k + 1 : k].buf.bytes < (size_t)std::max<long>(other, 1) * 8)
      fresh_center.reserve(std::max<long>(other, 1) * 8);
  }
  // commit: from here on the bond table and the MPS change
  if (fresh_center.p) mps_[l2r ? k + 1 : k].buf = std::move(fresh_center);
  bonds_[k + 1] = nb;
  // kept singular vectors in descending order: U (R x nm, column-major) moving
  // right, V^T (nm x C, column-major) moving left
  std::vector<long> oU(mids.size(), 0), oV(mids.size(), 0);
  std::vector<int> mm(mids.size(), 0);
  {
    long su = 0;
    std::vector<int64_t> vdesc;
    for (size_t i = 0; i < mids.size(); ++i) {
      if (kept[i] == 0) continue;
      int d = gd[i], nm = kept[i];
      long top = goff[i] + (long)(gb[i] - 1) * gb[i];  // column of the largest eigenvalue
      if (l2r) {
        oU[i] = su;
        mm[i] = d;
        vdesc.insert(vdesc.end(), {top, 1, -(int64_t)gb[i], su, 1, d, d, nm, dbits(1.0)});
      } else {
        oV[i] = su;
        kk[i] = nm;
        vdesc.insert(vdesc.end(), {top, 1, -(int64_t)gb[i], su, nm, 1, d, nm, dbits(1.0)});
      }
      su += (long)d * nm;
    }
    DevMem& dst = l2r ? Uv : Vv;
    dst.reserve(std::max<long>(su, 1) * 8);
    check_desc(vdesc, 0, vdesc.size(), gtot, su);
    DevMem vd;
    vd.reserve(vdesc.size() * 8 + 8);
    hip_check(hipMemcpyAsync(vd.p, vdesc.data(), vdesc.size() * 8, hipMemcpyHostToDevice, st), "vdesc");
    launch_copy_blocks(vd.as<int64_t>(), (int)(vdesc.size() / 9), gram.as<double>(), dst.as<double>(), st);
    hip_check(hipStreamSynchronize(st), "vdesc");
    sU_total_ = su;
  }
  // new tensors
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  std::vector<int64_t> cdesc;
  SiteTensor fixed;  // the orthonormal side
  // it takes over the allocation of the tensor it replaces (no longer read from
  // here on): a stable address keeps the cached environment-update plan resolved
  // and saves an allocation and a free per step
  fixed.buf = fresh_fixed.p ? std::move(fresh_fixed) : std::move(mps_[l2r ? k : k + 1].buf);
  fixed.lay = l2r ? make_tensor_layout(bonds_[k], nb, site_phys_qn()) : make_tensor_layout(nb, bonds_[k + 2], site_phys_qn());
  launch_fill(fixed.buf.as<double>(), fixed.lay.size, 0.0, st);
  for (int r = 0; r < nr; ++r) launch_fill(centers_[r].as<double>(), clay.size, 0.0, st);
  for (size_t i = 0; i < mids.size(); ++i) {
    if (kept[i] == 0) continue;
    const Mid& m = mids[i];
    int nm = kept[i];
    int qi = new_index[i];
    if (l2r) {
      // A_k[(li, s1), q_m] = U rows; center_r = U^T Psi_r
      for (int s1 = 0; s1 < 4; ++s1) {
        const Part& rp = m.rows[s1];
        if (rp.dim == 0) continue;
        const Slab& as = fixed.lay.slabs[fixed.lay.slab_of_left[rp.idx]];
        int b = as.block_of(s1, qi);
        cdesc.insert(cdesc.end(), {oU[i] + rp.off, 1, mm[i], as.off + as.blocks[b].col0, as.width, 1, rp.dim, nm,
                                   dbits(1.0)});
      }
      const Slab& cs = clay.slabs[clay.slab_of_left[qi]];
      for (int r = 0; r < nr; ++r) {
        int ib = (int)items.size();
        items.push_back({Uv.as<double>() + oU[i], plain.as<double>() + off_plain[i] + (long)r * m.R * m.C, mm[i],
                         m.R, m.R, 0, 1.0});
        tile_units(units, centers_[r].as<double>() + cs.off, cs.width, nm, m.C, ib, ib + 1);
      }
    } else {
      // B_{k+1}[q_m, (s2, ri)] = Vt rows; center_r = Psi_r Vt^T
      const Slab& bs = fixed.lay.slabs[fixed.lay.slab_of_left[qi]];
      cdesc.insert(cdesc.end(), {oV[i], 1, kk[i], bs.off, bs.width, 1, nm, m.C, dbits(1.0)});
      for (int s1 = 0; s1 < 4; ++s1) {
        const Part& rp = m.rows[s1];
        if (rp.dim == 0) continue;
        const Slab& cs = clay.slabs[clay.slab_of_left[rp.idx]];
        int b = cs.block_of(s1, qi);
        for (int r = 0; r < nr; ++r) {
          int ib = (int)items.size();
          items.push_back({plain.as<double>() + off_plain[i] + (long)r * m.R * m.C + rp.off,
                           Vv.as<double>() + oV[i], m.R, kk[i], m.C, 0, 1.0});
          tile_units(units, centers_[r].as<double>() + cs.off + cs.blocks[b].col0, cs.width, rp.dim, nm, ib, ib + 1);
        }
      }
    }
  }
  check_desc(cdesc, 0, cdesc.size(), sU_total_, fixed.lay.size);
  if (!cdesc.empty()) {
    DevMem cd;
    cd.reserve(cdesc.size() * 8);
    hip_check(hipMemcpyAsync(cd.p, cdesc.data(), cdesc.size() * 8, hipMemcpyHostToDevice, st), "cdesc");
    launch_copy_blocks(cd.as<int64_t>(), (int)(cdesc.size() / 9), l2r ? Uv.as<double>() : Vv.as<double>(),
                       fixed.buf.as<double>(), st);
    hip_check(hipStreamSynchronize(st), "cdesc");
  }
  gemm_once(l2r ? GEMM_NT : GEMM_TN, items, units);
  center_lay_ = clay;
  if (l2r) {
    mps_[k] = std::move(fixed);
    mps_[k + 1].lay = clay;
    mps_[k + 1].buf.reserve(std::max<long>(clay.size, 1) * 8);
    launch_copy(mps_[k + 1].buf.as<double>(), centers_[0].as<double>(), clay.size, st);
    center_site_ = k + 1;
  } else {
    mps_[k + 1] = std::move(fixed);
    mps_[k].lay = clay;
    mps_[k].buf.reserve(std::max<long>(clay.size, 1) * 8);
    launch_copy(mps_[k].buf.as<double>(), centers_[0].as<double>(), clay.size, st);
    center_site_ = k;
  }
  hip_check(hipStreamSynchronize(st), "svd step");
  // next guesses
  next_guess.clear();
  next_guess.resize(nr);
  if (l2r && k + 2 < L_) {
    long sz = make_tensor_layout(bonds_[k + 1], bonds_[k + 3], twosite_phys_qn()).size;
    SiteTensor c;
    c.lay = clay;
    for (int r = 0; r < nr; ++r) {
      next_guess[r].reserve(std::max<long>(sz, 1) * 8);
      std::swap(c.buf, centers_[r]);
      form_twosite(k + 1, c, mps_[k + 2], next_guess[r].as<double>());
      std::swap(c.buf, centers_[r]);
    }
  } else if (!l2r && k >= 1) {
    long sz = make_tensor_layout(bonds_[k - 1], bonds_[k + 1], twosite_phys_qn()).size;
    SiteTensor c;
    c.lay = clay;
    for (int r = 0; r < nr; ++r) {
      next_guess[r].reserve(std::max<long>(sz, 1) * 8);
      std::swap(c.buf, centers_[r]);
      form_twosite(k - 1, mps_[k - 1], c, next_guess[r].as<double>());
      std::swap(c.buf, centers_[r]);
    }
  }
}

// ------------------------------------------------------------------- sweeps --
// Two-site guesses for step k: the truncation's next-step guesses when they
// were made for this step, else the per-root centers when the last truncation
// left them on site k or k+1, else the MPS itself (root 0) and seeded random
// vectors (further roots).
void Solver::make_guess(int k, bool l2r) {
  const int nr = opt_.n_states;
  if (guess_k_ == k && guess_l2r_ == l2r && (int)guess_.size() == nr) return;
  guess_.clear();
  guess_.resize(nr);
  long sz = twosite_size(k);
  for (int r = 0; r < nr; ++r) guess_[r].reserve(std::max<long>(sz, 1) * 8);
  bool have = (int)centers_.size() == nr && (center_site_ == k || center_site_ == k + 1);
  Rng rng(opt_.seed + 7919);
  for (int r = 0; r < nr; ++r) {
    if (have) {
      SiteTensor c;
      c.lay = center_lay_;
      std::swap(c.buf, centers_[r]);
      if (center_site_ == k) form_twosite(k, c, mps_[k + 1], guess_[r].as<double>());
      else form_twosite(k, mps_[k], c, guess_[r].as<double>());
      std::swap(c.buf, centers_[r]);
    } else if (r == 0) {
      form_twosite(k, mps_[k], mps_[k + 1], guess_[0].as<double>());
    } else {
      std::vector<double> h(sz);
      for (auto& x : h) x = rng.normal();
      hip_check(hipMemcpy(guess_[r].p, h.data(), sz * 8, hipMemcpyHostToDevice), "guess");
    }
  }
  guess_k_ = k;
  guess_l2r_ = l2r;
}

// One two-site step (Fig. 2 of the paper): solve H_eff on sites (k, k+1) with
// Davidson, decimate with the SVD, move the center, update the environment.
double Solver::step(int k, bool l2r, std::vector<double>& energies) {
  DMRG_REQUIRE(k >= 0 && k + 1 < L_, ST_EINVAL, "two-site step out of range");
  // the environments are orthonormal bases only when the orthogonality centre is on the two sites
  DMRG_REQUIRE(center_site_ < 0 || center_site_ == k || center_site_ == k + 1, ST_ESTATE,
               "two-site step away from the orthogonality centre (site " + std::to_string(center_site_) + ")");
  make_guess(k, l2r);
  prepare(k);
  std::vector<double> ev;
  davidson(k, guess_, ev);
  energies = ev;
  for (auto& e : energies) e += prob_->e_core;
  double tau = 0;
  auto t0 = std::chrono::steady_clock::now();
  svd_step(k, l2r, opt_.n_states, guess_, tau);
  guess_k_ = l2r ? k + 1 : k - 1;
  guess_l2r_ = l2r;
  if (guess_k_ < 0 || guess_k_ + 1 >= L_) guess_k_ = -1;
  st_.svd_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  after_truncation(k, l2r);
  st_.tau = tau;
  if (opt_.verbose)
    fprintf(stderr, "%s k=%d E=%.12f tau=%.2e M=%d\n", l2r ? "L->R" : "R->L", k, energies[0], tau,
            bonds_[k + 1].total());
  return tau;
}

// Environment of the new orthonormal site (its factors were built for the step)
// and invalidation of every environment the changed sites enter.
void Solver::after_truncation(int k, bool l2r) {
  auto t1 = std::chrono::steady_clock::now();
  if (l2r) {
    env_update_left(k, lf_);
    // sites k, k+1 changed: left envs beyond k+1 and right envs up to k+1 are stale
    for (int c = k + 2; c <= L_; ++c) left_[c].valid = false;
    for (int c = 0; c <= k + 1; ++c) right_[c].valid = false;
  } else {
    env_update_right(k + 1, rf_);
    for (int c = 0; c <= k; ++c) right_[c].valid = false;
    for (int c = k + 1; c <= L_; ++c) left_[c].valid = false;
  }
  hip_check(hipStreamSynchronize(st), "env");
  st_.env_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  plan_k_ = -1;
  ovl_invalidate(k + 1, k + 1);  // overlaps through site k (left) or site k+1 (right)
}

double Solver::truncate(int k, bool l2r, const double* psi) {
  DMRG_REQUIRE(k >= 0 && k + 1 < L_, ST_EINVAL, "two-site step out of range");
  DMRG_REQUIRE(center_site_ < 0 || center_site_ == k || center_site_ == k + 1, ST_ESTATE,
               "truncation away from the orthogonality centre (site " + std::to_string(center_site_) + ")");
  prepare(k);
  const long n = psi_lay_.size;
  const int nr = opt_.n_states;
  dv_X_.reserve((size_t)nr * n * 8);
  launch_copy(dv_X_.as<double>(), psi, (long)nr * n, st);
  double tau = 0;
  auto t0 = std::chrono::steady_clock::now();
  svd_step(k, l2r, nr, guess_, tau);
  guess_k_ = l2r ? k + 1 : k - 1;
  guess_l2r_ = l2r;
  if (guess_k_ < 0 || guess_k_ + 1 >= L_) guess_k_ = -1;
  st_.svd_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  after_truncation(k, l2r);
  st_.tau = tau;
  return tau;
}

std::vector<double> Solver::export_mps() const {
  if (!pending_mps_.empty()) return pending_mps_;
  long total = 0;
  for (int k = 0; k < L_; ++k) total += mps_[k].lay.size;
  std::vector<double> out(total);
  long off = 0;
  for (int k = 0; k < L_; ++k) {
    const long sz = mps_[k].lay.size;
    if (sz > 0)
      hip_check(hipMemcpyAsync(out.data() + off, mps_[k].buf.p, sz * sizeof(double), hipMemcpyDeviceToHost, st),
                "mps export");
    off += sz;
  }
  hip_check(hipStreamSynchronize(st), "mps export");
  return out;
}

double Solver::sweep(int n_sweeps, std::vector<double>& energies) {
  double tau_max = 0;
  bool all_ok = true;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    tau_max = 0;
    for (int k = 0; k + 1 < L_; ++k) {
      tau_max = std::max(tau_max, step(k, true, energies));
      all_ok = all_ok && last_converged_;
    }
    for (int k = L_ - 2; k >= 0; --k) {
      tau_max = std::max(tau_max, step(k, false, energies));
      all_ok = all_ok && last_converged_;
    }
  }
  last_converged_ = all_ok;
  st_.tau = tau_max;
  return tau_max;
}

// x <- P x for the one-site space of the step: with site k+1 frozen (F,
// right-orthonormal) X = x F^T over (s2, bond k+2) and x = X F; with site k
// frozen (left-orthonormal) Y = F^T x over (bond k, s1) and x = F Y.
void Solver::onesite_project(int k, double* x) {
  const TensorLayout P = make_tensor_layout(bonds_[k], bonds_[k + 2], twosite_phys_qn());
  std::vector<GemmItem> items;
  std::vector<GemmUnit> units;
  if (onesite_ > 0) {
    const SiteTensor& F = mps_[k + 1];
    os_tmp_.lay = make_tensor_layout(bonds_[k], bonds_[k + 1], site_phys_qn());
    os_tmp_.buf.reserve(std::max<long>(os_tmp_.lay.size, 1) * 8);
    for (const Slab& xs : os_tmp_.lay.slabs) {
      const int pi = P.slab_of_left[xs.li];
      for (const SlabBlock& xb : xs.blocks) {  // X[a, s1, m]
        const int ib = (int)items.size();
        const int fi = F.lay.slab_of_left[xb.ri];
        if (pi >= 0 && fi >= 0) {
          const Slab& ps = P.slabs[pi];
          const Slab& fs = F.lay.slabs[fi];
          for (const SlabBlock& fb : fs.blocks) {  // F[m, s2, b]
            const int pb = ps.block_of(4 * xb.phys + fb.phys, fb.ri);
            if (pb < 0) continue;
            items.push_back({x + ps.off + ps.blocks[pb].col0, F.buf.as<double>() + fs.off + fb.col0, ps.width,
                             fs.width, fb.mr, 0, 1.0});
          }
        }
        tile_units(units, os_tmp_.buf.as<double>() + xs.off + xb.col0, xs.width, xs.ml, xb.mr, ib,
                   (int)items.size());
      }
    }
    gemm_once(GEMM_NT, items, units);
    form_twosite(k, os_tmp_, F, x);
  } else {
    const SiteTensor& F = mps_[k];
    os_tmp_.lay = make_tensor_layout(bonds_[k + 1], bonds_[k + 2], site_phys_qn());
    os_tmp_.buf.reserve(std::max<long>(os_tmp_.lay.size, 1) * 8);
    for (const Slab& ys : os_tmp_.lay.slabs) {
      for (const SlabBlock& yb : ys.blocks) {  // Y[m, s2, b]
        const int ib = (int)items.size();
        for (const Slab& fs : F.lay.slabs) {  // F[a, s1, m]
          const int pi = P.slab_of_left[fs.li];
          if (pi < 0) continue;
          const Slab& ps = P.slabs[pi];
          for (const SlabBlock& fb : fs.blocks) {
            if (fb.ri != ys.li) continue;
            const int pb = ps.block_of(4 * fb.phys + yb.phys, yb.ri);
            if (pb < 0) continue;
            items.push_back({F.buf.as<double>() + fs.off + fb.col0, x + ps.off + ps.blocks[pb].col0, fs.width,
                             ps.width, fs.ml, 0, 1.0});
          }
        }
        tile_units(units, os_tmp_.buf.as<double>() + ys.off + yb.col0, ys.width, ys.ml, yb.mr, ib,
                   (int)items.size());
      }
    }
    gemm_once(GEMM_TN, items, units);
    form_twosite(k, F, os_tmp_, x);
  }
}

// One-site sweeps at fixed bond dimensions (Sec. II.E: a truncated two-site
// fixed point is not stationary on the tangent space of its own bond
// dimension).  Each two-site step optimises one site inside the two-site space
// (the projected Davidson above) and the SVD moves the centre without
// truncation, so the bond dimensions stay (only numerically zero singular
// values can go).  At a fixed point every one-site tensor is the lowest
// eigenvector of its effective Hamiltonian: the gauge-free tangent gradient,
// whose blocks are the first-iteration residuals of the steps, vanishes, and
// the Hellmann-Feynman gradient is the exact derivative of the variational
// energy at this bond dimension.
double Solver::stationarize(int n_sweeps, std::vector<double>& energies) {
  DMRG_REQUIRE(opt_.n_states == 1, ST_EINVAL, "one-site sweeps take one state");
  DMRG_REQUIRE(center_site_ <= 0, ST_ESTATE, "one-site sweeps start with the centre on site 0");
  struct Reset {
    int& f;
    ~Reset() { f = 0; }
  } reset{onesite_};
  bool all_ok = true;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    first_res_ = 0;
    for (int k = 0; k + 1 < L_; ++k) {
      onesite_ = 1;
      guess_k_ = -1;
      step(k, true, energies);
      all_ok = all_ok && last_converged_;
    }
    for (int k = L_ - 2; k >= 0; --k) {
      onesite_ = -1;
      guess_k_ = -1;
      step(k, false, energies);
      all_ok = all_ok && last_converged_;
    }
  }
  last_converged_ = all_ok;
  return first_res_;
}

// <Psi_r|H|Psi_r>/<Psi_r|Psi_r> of the current MPS (root r via its center tensor).
std::vector<double> Solver::mps_energy() {
  const int nr = (center_site_ == 0 && (int)centers_.size() == opt_.n_states) ? opt_.n_states : 1;
  prepare(0);
  const long n = psi_lay_.size;
  DevMem psi, sig, part, sc;
  psi.reserve(n * 8);
  sig.reserve(n * 8);
  part.reserve(512 * 8 * 4);
  sc.reserve(64);
  std::vector<double> out;
  for (int r = 0; r < nr; ++r) {
    if (nr > 1) {
      SiteTensor c;
      c.lay = center_lay_;
      std::swap(c.buf, centers_[r]);
      form_twosite(0, c, mps_[1], psi.as<double>());
      std::swap(c.buf, centers_[r]);
    } else {
      form_twosite(0, mps_[0], mps_[1], psi.as<double>());
    }
    sigma(0, PREC_F64, psi.as<double>(), sig.as<double>());
    launch_dots(psi.as<double>(), n, 1, sig.as<double>(), n, part.as<double>(), sc.as<double>(), st);
    launch_dots(psi.as<double>(), n, 1, psi.as<double>(), n, part.as<double>(), sc.as<double>() + 1, st);
    double h[2];
    hip_check(hipMemcpyAsync(h, sc.p, 16, hipMemcpyDeviceToHost, st), "energy");
    hip_check(hipStreamSynchronize(st), "energy");
    // psi . H_eff psi = <Psi|H|Psi> in any gauge (the left block of step 0 is the
    // vacuum); psi . psi is <Psi|Psi> only for right-orthonormal sites 2.. (the
    // centre on site 0 or 1), so otherwise a single state takes its norm from the
    // whole chain
    if (nr == 1 && center_site_ != 0 && center_site_ != 1) {
      const MPSView me{&bonds_, &mps_};
      h[1] = chain_overlap(me, me);
    }
    out.push_back(h[0] / h[1] + prob_->e_core);
  }
  return out;
}

}  // namespace dmrg
