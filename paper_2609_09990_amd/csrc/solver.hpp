// Two-site DMRG solver: device-resident MPS, environments, step plans, Davidson,
// SVD truncation and the sweep (the paper's decimation step, Fig. 2).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <array>
#include <map>
#include <memory>
#include <vector>

#include "kernels.hpp"
#include "layout.hpp"
#include "problem.hpp"

namespace dmrg {

struct Options {
  int M = 256;
  int n_states = 1;
  std::vector<double> weights;
  double davidson_tol = 1e-10;
  int max_iter = 200;
  int max_subspace = 32;
  int precision = PREC_F64;
  int precond = 0;
  unsigned long long seed = 1;
  double tie_rtol = 1e-10;
  double cut_rtol = 1e-14;
  int verbose = 0;
  long long sigma_chunk_bytes = 0;  // 0: all left factors in one chunk
  int pcg_steps = 5;                // shift-and-invert correction: inner CG steps ...
  double pcg_rtol = 0.1;            // ... and relative residual at which they stop
  double trunc_tol = 0;             // adaptive bond dimension: discarded weight per bond (0: fixed M)
  int m_min = 1;                    // ... never fewer states than this
};

// A caller-provided slab of device memory that the library carves into its
// buffers (the single preallocated arena of the paper's device engine, Sec. III):
// first fit over free ranges, 256-byte granules, neighbouring free ranges merged.
class Arena {
 public:
  Arena(void* base, size_t bytes);
  void* alloc(size_t bytes);  // Error(ST_ENOMEM) when no free range fits
  void free(void* p);
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t failed_request() const { return failed_; }  // bytes of the last request that did not fit (0: none)
  bool contains(const void* p) const { return (const char*)p >= base_ && (const char*)p < base_ + size_; }

 private:
  char* base_;
  size_t size_;
  std::map<size_t, size_t> free_, used_;  // offset -> length
  size_t in_use_ = 0, peak_ = 0, failed_ = 0;
};

// Buffers reserved while an arena is current (thread-local, set around every
// call on a solver that has a workspace) come from it; otherwise from hipMalloc.
Arena*& current_arena();
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};
// Number of hipMalloc calls the library's buffers have made (process-wide).
long library_device_allocations();

// Grow-only pinned host buffer (staging of plan tables for their uploads).
struct PinnedStage {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedStage() = default;
  PinnedStage(const PinnedStage&) = delete;
  PinnedStage& operator=(const PinnedStage&) = delete;
  ~PinnedStage();
  void* reserve(size_t b);
  template <class T> T* get(long n) { return (T*)reserve((size_t)std::max<long>(n, 1) * sizeof(T)); }
};

// Grow-only device buffer.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;  // the arena the memory came from (nullptr: hipMalloc)
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes), arena(o.arena) {
    o.p = nullptr;
    o.bytes = 0;
    o.arena = nullptr;
  }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      arena = o.arena;
      o.p = nullptr;
      o.bytes = 0;
      o.arena = nullptr;
    }
    return *this;
  }
  ~DevMem();
  void reserve(size_t b);
  void release();
  template <class T> T* as() const { return (T*)p; }
};

void hip_check(hipError_t e, const char* what);
bool same_sectors(const std::vector<Sector>& a, const std::vector<Sector>& b);

// Environment at one cut: channels grouped by quantum-number shift.
struct Env {
  bool valid = false;
  std::vector<EnvClass> classes;
  std::vector<int> chan_class, chan_slot;
  std::vector<long> class_base;
  long size = 0;
  DevMem buf;
  long chan_off(int ch) const {
    return class_base[chan_class[ch]] + (long)chan_slot[ch] * classes[chan_class[ch]].nnz;
  }
};

struct SiteTensor {
  TensorLayout lay;
  DevMem buf;
};

// Buffer ids used by the relocatable plans.
enum BufId : int {
  B_PSI = 0,   // two-site input vector (or site tensor for env updates)
  B_OUT,       // sigma output / new environment
  B_T,         // intermediates X psi (or X A, B Y)
  B_XMIX,      // premixed left factors
  B_YMIX,      // premixed right factors
  B_ENVL,      // left environment at cut k
  B_ENVR,      // right environment at cut k+2
  B_SITE2,     // second site tensor (right env update: B_j itself)
  B_YPAIR,     // merged right-factor blocks of sigma phase B
  B_NBUF
};

struct PItem {
  int abuf; long aoff; int bbuf; long boff;
  int lda, ldb, K;
  double coef;
};
struct PUnit {
  int cbuf; long coff;
  int ldc, M, N, m0, n0, ib, ie, acc;
};

// A relocatable grouped GEMM: one launch, pointers resolved per precision.
struct Phase {
  int mode = GEMM_NN;
  int tag = 0;  // kernel instantiation name tag (profiling only)
  hipEvent_t gemm_done = nullptr;  // if set, recorded between the GEMM and the split-K reduction
  std::vector<PItem> items;
  std::vector<PUnit> units;
  double flops = 0.0;       // algorithmic flops (see build_sigma_plan for sigma)
  double flops_exec = -1;   // flops the launch executes, unpadded (-1: same as flops)
  // device copies per precision
  DevMem d_items[3], d_units[3];
  DevMem d_tiles[3];                 // split-K tile table per precision slot
  const void* slot_base[3] = {};     // split-K scratch the units were resolved against
  int n_units[3] = {0, 0, 0}, n_tiles[3] = {0, 0, 0};
  const void* last_bases[3][B_NBUF] = {};
  bool uploaded[3] = {false, false, false};
  bool buf_ok[3] = {false, false, false};  // every item fits the buffer-load kernels
  bool wg = false;                         // may take the fp64 workgroup block kernel (NT)
  double split_work = 0;                   // > 0: split-K granularity from this work, not the phase's own
  bool wg_used[3] = {false, false, false};
};

// One side's factors for a middle cut: X_{beta,op} = sum_alpha c L[alpha] (left)
// or Y_{beta,op} = sum_gamma c R[gamma] (right), deduplicated.
struct Factor {
  int cls;        // class index in the env
  bool alias;     // true: a single env channel (off into env), else premixed
  long off;       // element offset (env buffer if alias, premix buffer otherwise)
};
struct FactorUse {
  int op;
  int f;
  double scale;
};
struct FactorSide {
  int cut = -1;
  std::vector<Factor> fac;
  std::vector<std::vector<FactorUse>> by_mid;  // per middle-cut channel
  // premix program
  std::vector<int> ptr;
  std::vector<long> src_off;
  std::vector<double> coef;
  std::vector<long> out_off;  // per premixed output (element offset in premix buffer)
  std::vector<long> out_nnz;
  long premix_size = 0;
  bool left = true;
  DevMem* mix = nullptr;  // the solver's premix buffer of this side (shared by every plan of the side)
  DevMem d_srcs, d_ptr, d_coef;
  std::vector<const double*> h_srcs;
};

// Sigma phase B: items of one output block that share their A slice (the same
// T_X columns) form one product with the coefficient-weighted sum of their
// right-factor blocks, sum_j c_j T Y_j^T = T (sum_j c_j Y_j)^T.  The sums are
// formed once per step, after the premix, into `mix`.
struct PairMix {
  std::vector<int> ptr;       // sources of group g: [ptr[g], ptr[g + 1])
  std::vector<int> src_buf;   // B_YMIX or B_ENVR
  std::vector<long> src_off;  // element offset of an N x K source block
  std::vector<double> coef;
  std::vector<long> out_off;  // per group: element offset in mix
  std::vector<int> nnz;       // per group: N x K
  long size = 0;
  DevMem* mix = nullptr;  // the solver's merged-block buffer
  DevMem d_srcs, d_ptr, d_coef, d_out_off, d_nnz;
  std::vector<const double*> h_srcs;
};

struct Stats {
  int matvecs = 0;
  int davidson_iters = 0;
  double sigma_ms = 0, env_ms = 0, svd_ms = 0, davidson_other_ms = 0, premix_ms = 0;
  double sigma_flops = 0;
  double sigma_a_ms = 0, sigma_b_ms = 0, sigma_a_flops = 0, sigma_b_flops = 0, env_flops = 0;
  double sigma_a_flops_exec = 0, sigma_b_flops_exec = 0;  // executed (merged / trimmed plan)
  double sigma_b_gemm_ms = 0;  // phase-B GEMM kernel alone (without the split-K reduction)
  double tau = 0;
  int max_bond = 0;
  int fallbacks = 0;
  int converged = 1;
  int refinements = 0;
  double grad_ms = 0, grad_flops = 0;  // integral-gradient passes
  double prepare_ms = 0, resolve_ms = 0, davidson_ms = 0;  // host wall times
  int plan_hits = 0;  // step plans reused from the cache
  int lowp_matvecs = 0;  // sigma products in fp32 / bf16
  double plan_build_ms = 0;  // host: sigma step plans built (factor sides and items)
  double env_plan_ms = 0;    // host: environment-update plans built
};

class MLP;

// What a solver carries over when its device memory moves to a new workspace.
struct SolverState {
  std::vector<Bond> bonds;
  std::vector<double> mps;  // all site tensors in slab layout
  int center_site = -1;
  std::vector<std::vector<double>> centers;  // per-root centre tensors of the last truncation
  std::vector<Sector> center_bond_l, center_bond_r;
  Options opt;
  int precond = 0;
  void* net = nullptr;
  int rec_cap = 0, rec_sample = 0;
  int kernel_tag = 0;
  Stats stats;
  struct Lower {
    std::vector<Bond> bonds;
    std::vector<double> mps;
    double w;
  };
  std::vector<Lower> lower;  // states held for penalty deflation
};

// A lower state held on the device for penalty deflation (Sec. II.F), with its
// overlap environments against the state being optimised: per cut, one
// block-diagonal matrix <basis of Psi | part of Phi>, block per common sector
// (the left one over the sites before the cut, the right one over the rest).
struct Deflated {
  double w = 0;     // penalty weight (energy units)
  double norm = 1;  // ||Phi||
  std::vector<Bond> bonds;
  std::vector<SiteTensor> sites;
  std::vector<DevMem> ol, orr;
  std::vector<char> ol_ok, orr_ok;
};
// An MPS as the overlap contractions see it.
struct MPSView {
  const std::vector<Bond>* bonds;
  const std::vector<SiteTensor>* sites;
};

class Solver {
 public:
  // The initial MPS is made on the host; it reaches the device on the first
  // call that needs device state (materialize), so creating a solver allocates
  // no device memory.
  Solver(const Problem* p, const Options& o, hipStream_t s);
  ~Solver();
  void materialize();
  SolverState save_state();
  void restore_state(const SolverState& s);
  // Device bytes a sweep at the current bonds is expected to need (environments
  // of every cut, the largest step's sigma intermediates and Davidson basis, the
  // MPS, plans); an estimate, see dmrg_workspace_query.
  size_t workspace_estimate() const;

  // MPS management
  void init_random_mps();
  void set_mps(const std::vector<Bond>& bonds, const std::vector<const double*>& sites_host);
  const std::vector<Bond>& bonds() const { return bonds_; }

  // prepare environments and plans for the two-site step at sites (k, k+1)
  void prepare(int k);
  long twosite_size(int k) const;
  void sigma(int k, int prec, const double* psi, double* out);
  void diag(int k, double* out);
  double sweep(int n_sweeps, std::vector<double>& energies);
  // One-site sweeps at the current bond dimensions (the stationarity of the
  // truncated MPS, Sec. II.E); returns the largest local tangent gradient of the
  // last sweep.  Needs one state, sites 1.. right-orthonormal (as after a sweep).
  double stationarize(int n_sweeps, std::vector<double>& energies);
  double step(int k, bool left_to_right, std::vector<double>& energies);
  std::vector<double> mps_energy();
  // Host copy of the current MPS: all site tensors concatenated in slab layout.
  std::vector<double> export_mps() const;
  // Truncation of step k applied to caller-given two-site vectors (device,
  // n_states x n, root-major) instead of Davidson's: new bond k+1, sites k and
  // k+1, the centre moved as a step moves it; returns tau.
  double truncate(int k, bool left_to_right, const double* psi);
  // Kept singular values of the last truncation, descending over all sectors.
  const std::vector<double>& last_kept_sv() const { return last_kept_sv_; }
  // Penalty deflation (Sec. II.F): the Davidson operator of every later step is
  // H_eff + sum_j w_j |phi_j><phi_j| / ||Phi_j||^2, phi_j the projection of the
  // lower state Phi_j (held on the device) into the step's two-site space.
  void deflate_add(const std::vector<Bond>& bonds, const std::vector<const double*>& sites, double w);
  void deflate_clear();
  int n_deflated() const { return (int)defl_.size(); }
  // Projection of lower state j into step k's two-site space, times `scale`
  // (device out of twosite_size(k) doubles).
  void deflate_project(int k, int j, double scale, double* out);
  // <Psi|Phi_j> / (||Psi|| ||Phi_j||) over the whole chain, in fp64.
  double overlap(int j);
  // Per-root <S^2> of the current MPS (orthogonality centre at site 0).
  std::vector<double> s_squared();
  // Device copy of another solver's MPS (same active space and sector).
  void adopt_mps(const Solver& o);
  // Energies of the roots w refers to and sum_r w_r dE_r/dh (n*n), dE_r/dB (nq*n*n).
  void grad(const std::vector<double>& w, std::vector<double>& dh, std::vector<double>& dB,
            std::vector<double>& energies);
  const Stats& stats() const { return st_; }
  int n_states() const { return opt_.n_states; }
  bool last_converged() const { return last_converged_; }  // the last step / sweep call
  void set_precision(int prec) {
    DMRG_REQUIRE(prec == PREC_F64 || prec == PREC_F32 || prec == PREC_BF16, ST_EINVAL, "unknown precision");
    opt_.precision = prec;
  }

  // Davidson preconditioner: 0 diagonal, 1 learned (net borrowed, must outlive its use)
  void set_precond(int mode, MLP* net);
  // Record (features, projected target) training triples of root 0 in later
  // Davidson solves: up to `capacity` triples of `sample` amplitudes each.
  void record_triples(int capacity, int sample);
  // Copies up to cap recorded triples to device arrays X[cap][sample][8],
  // T[cap][sample] (stream-ordered) and clears the store; returns the count.
  int take_triples(float* X, float* T, int cap);
  int triple_sample() const { return rec_sample_; }
  // Features of the prepared step k for device vectors r, d and a host theta.
  // CI vector (row-major c[I_a][I_b], colex strings) of this MPS (state 0) or of
  // held state `state` (1..n_deflated), as stored
  void mps_to_ci(int state, double* c);
  // two-orbital density matrices of the stored MPS for every pair i < j (host
  // [pair][16][16], determinant convention, trace 1)
  std::vector<double> pair_rdm_mps();
  int correction_host_theta(int k, int mode, const double* x, const double* r, const double* d, double theta,
                            double* t);
  void features_host_theta(int k, const double* r, const double* d, double theta, float* X);
  std::vector<double> env_host(int cut, int side);
  const Problem* prob() const { return prob_; }

  // sigma phase timing helpers for measurement
  double last_sigma_flops() const;       // algorithmic (every block product of the factorisation)
  double last_sigma_flops_exec() const;  // executed by the launches (merged / trimmed plan, unpadded)
  // 0: sigma phases launch the tag-1/2 kernel instantiations, 1: tag-3/4
  void set_kernel_tag(int t) { kernel_tag_ = t ? 1 : 0; }
  int kernel_tag_ = 0;
  double sigma_phase_ms(int which) const { return sigma_phase_ms_[which]; }

 private:
  const Problem* prob_;
  Options opt_;
  hipStream_t st;
  // the truncation's batched eigensolves run one size bucket per stream (each
  // bucket is a latency-bound chain of small kernels); default priority
  static constexpr int kAuxStreams = 4;
  hipStream_t aux_st_[kAuxStreams] = {};
  rocblas_handle aux_rb_[kAuxStreams] = {};
  DevMem rb_work_[kAuxStreams];  // rocBLAS workspaces when the solver runs in an arena
  std::vector<double> pending_mps_;  // host copy of the initial MPS until materialize()
  hipEvent_t aux_ev_[kAuxStreams + 1] = {};
  int L_;
  std::vector<Bond> bonds_;
  std::vector<SiteTensor> mps_;
  std::vector<Env> left_, right_;  // left_[c]: env of cut c built from sites < c; right_[c]: sites >= c
  Stats st_;
  double sigma_phase_ms_[4] = {0, 0, 0, 0};

  // step plan (cached for the prepared step)
  int plan_k_ = -1;
  FactorSide lf_, rf_;
  PairMix pm_;
  TensorLayout psi_lay_;
  std::vector<Phase> phA_, phB_;  // per chunk of left factors (build_sigma_plan)
  long t_size_ = 0;               // T_X doubles of the largest chunk
  std::vector<hipEvent_t> sig_ev_;  // phase boundaries of one sigma call (timing)
  DevMem psi_in_, out_buf_, t_buf_;
  // split-K partial tiles of whichever phase is running: phases run one after
  // another on the solver stream, so one scratch serves every cached plan
  DevMem splitk_;
  // premixed factors of the step being solved (left, right) and its merged right
  // blocks; filled at every prepare, grow-only, so their addresses (and the
  // resolved plans) stay put from one step to the next
  DevMem lmix_, rmix_, pmix_;
  DevMem env_t_buf_;  // intermediates of environment updates (kept apart so t_buf_ stays put)
  // Step plans by step k, reused when the outer bonds k and k+2 are unchanged
  // (the plan depends on them and the MPO only; values come from the buffers).
  struct StepPlan {
    std::vector<Sector> key_l, key_r;
    FactorSide lf, rf;
    PairMix pm;
    TensorLayout psi_lay;
    std::vector<Phase> phA, phB;
    long t_size = 0;
  };
  std::map<int, StepPlan> plan_cache_;
  // environment-update plans by (site, side), reused while bonds site, site+1 hold
  struct EnvPlan {
    std::vector<Sector> key_a, key_b;
    Phase pa, pb;
    long zsize = 0;
  };
  std::map<std::pair<int, int>, EnvPlan> env_plans_;
  int plan_built_k_ = -1;  // step whose plan is in lf_, rf_, psi_lay_, phA_, phB_
  std::vector<Sector> bonds_at_build_l_, bonds_at_build_r_;
  DevMem lowp_[B_NBUF];  // low-precision copies per buffer id
  int lowp_prec_ = -1;
  // Shift of the low-precision operator (precision form): the block
  // Hamiltonians of the step (left environment channel H at cut k, right channel
  // I at cut k+2) enter the low-precision copies as L_H - a 1 and R_I - b 1, so
  // their rounding error scales with their spread, not with the energy; the
  // product then gets (a + b) psi back in fp64.  Only with orthonormal outer
  // bases (centre on the two sites), where the partner channels are identities.
  bool shift_on_ = false;
  double shift_a_ = 0, shift_b_ = 0;
  DevMem shift_idx_[3], shift_w_[3];
  long shift_n_[3] = {0, 0, 0};
  void setup_lowp_shift(int k);
  long lowp_size_[B_NBUF] = {0};
  // diag plan
  std::vector<DiagBlock> dblocks_;
  std::vector<DiagTerm> dterms_host_;
  DevMem d_dblocks_, d_dterms_, diagvec_;
  bool diag_ready_ = false;
  std::vector<long> dterm_x_off_, dterm_y_off_;
  std::vector<int64_t> diag_desc_;

  // internals
  void ensure_left(int c);
  void ensure_right(int c);
  void make_env_layout(Env& e, int cut, const Bond& b);
  void build_factor_side(FactorSide& fs, bool left, int site);
  void run_premix(FactorSide& fs, const Env& env);
  void run_pairmix(int k);
  void env_update_left(int k, const FactorSide& fs);
  void env_update_right(int j, const FactorSide& fs);
  void build_sigma_plan(int k);
  void build_diag_plan(int k);
  void run_phase(Phase& ph, int prec, void* const* bases, size_t const* esz, const long* sizes);
  void launch_resolved(Phase& ph, int prec, int slot);
  void ensure_lowp(int prec);
  void svd_step(int k, bool left_to_right, int nr, std::vector<DevMem>& next_guess, double& tau);
  void form_twosite(int k, const SiteTensor& a, const SiteTensor& b, double* out);
  int davidson(int k, std::vector<DevMem>& guess, std::vector<double>& evals);
  void olsen(const double* x, const double* D, const double* theta, double* t);
  template <class Apply>
  int shift_invert(const double* x, const double* r, const double* D, const double* theta, double rnorm, double* t,
                   int prec, Apply& apply);
  DevMem dv_pcg_;  // work vectors of the Olsen and shift-and-invert corrections
  // one-site mode of a two-site step: +1 optimises site k with site k+1 frozen
  // (right-orthonormal), -1 optimises site k+1 with site k frozen (left-
  // orthonormal); the Davidson then works on P H_eff P, P the projector on that
  // one-site space inside the two-site space
  int onesite_ = 0;
  double first_res_ = 0;  // largest first-iteration residual of one-site steps
  SiteTensor os_tmp_;
  void onesite_project(int k, double* x);
  void gemm_once(int mode, std::vector<GemmItem>& items, std::vector<GemmUnit>& units);
  void grad_site(int k, std::vector<double>& g, double* norm);
  DevMem grad_P_, grad_Q_, grad_G_;

  // learned preconditioner and training-triple store
  bool last_converged_ = true;
  std::vector<double> last_kept_sv_;
  void after_truncation(int k, bool left_to_right);
  int precond_ = 0;
  MLP* net_ = nullptr;
  std::vector<int64_t> fblocks_host_;  // feature blocks of the prepared step: off, ld, rows, cols
  DevMem d_fblocks_, fstats_, feat_, nety_, dv_L_, feat_t_;
  int nfb_ = 0;
  int rec_cap_ = 0, rec_sample_ = 0, rec_count_ = 0;
  unsigned long long rec_seed_ = 0;
  DevMem rec_X_, rec_T_, rec_hist_, rec_idx_;
  void features(const double* r, const double* d, const double* theta, const double* t, float* X);

  // Davidson workspace
  DevMem dv_V_, dv_AV_, dv_G_, dv_evals_, dv_evecs_, dv_X_, dv_R_, dv_C_, dv_t_, dv_diag_, dv_part_,
      dv_sc_;
  std::vector<DevMem> centers_;    // per-root center tensors after the last truncation
  std::vector<DevMem> guess_;      // Davidson start vectors for step guess_k_
  int guess_k_ = -1;
  bool guess_l2r_ = true;
  void make_guess(int k, bool l2r);
  TensorLayout center_lay_;
  long sU_total_ = 0;  // size of the kept singular-vector buffer of the last truncation
  int center_site_ = -1;
  // penalty deflation
  std::vector<Deflated> defl_;
  DevMem defl_phi_, defl_t_, defl_a_, defl_b_;
  void ensure_ovl_left(int j, int c);
  void ensure_ovl_right(int j, int c);
  void ovl_invalidate(int first_left, int last_right);  // OL[c >= first_left], OR[c <= last_right]
  void ovl_update_left(const MPSView& bra, const MPSView& ket, int site, const double* in, double* out);
  void ovl_update_right(const MPSView& bra, const MPSView& ket, int site, const double* in, double* out);
  double chain_overlap(const MPSView& bra, const MPSView& ket);
  PinnedStage stage_items_, stage_units_, stage_tiles_;  // plan uploads (see run_phase)
  hipEvent_t stage_ev_ = nullptr;                        // recorded after the last upload from them
  bool stage_pending_ = false;
  DevMem scratch_items_, scratch_units_;
  std::vector<GemmItem> scratch_h_items_;
  std::vector<GemmUnit> scratch_h_units_;
};

// Determinant-space helpers (ci.cpp): the CI dimension C(n, n_a) C(n, n_b), and
// the (transition) 1-/2-RDMs of device CI vectors, times `scale`, to host arrays
// (gamma n^2, Gamma n^4, overlap <bra|ket> unscaled; each may be NULL).
long ci_dimension(int n, int na, int nb);
// Orbital entanglement from a device CI vector (2..16 orbitals): two-orbital
// density matrices of all pairs i < j (host, [pair][16][16], trace 1), the
// one-orbital entropies s1[n] and mutual information I[n][n]; and the ordering
// of orbitals by the Fiedler vector of I's graph Laplacian (host only).
void orbital_rdm2(int n, int na, int nb, hipStream_t st, const double* c, std::vector<double>& rho);
void mutual_information(int n, int na, int nb, hipStream_t st, const double* c, double* s1, double* I);
void mutual_information_of(int n, const std::vector<double>& rho, double* s1, double* I);
void fiedler_order(int n, const double* I, int* order, double* fiedler);
// V c for the all-active two-electron operator V = 1/2 sum (pq|rs) E_pq E_rs,
// streamed through the Cholesky factors Bh (host, nq x n x n); and the
// (transition) three-body density <bra|E_pq E_rs E_tu|ket> (host n^6) of device
// CI vectors.
void ci_apply_v(int n, int na, int nb, int nq, const double* Bh, hipStream_t st, const double* c, double* out);
void ci_rdm3(int n, int na, int nb, hipStream_t st, const double* bra, const double* ket, double scale, double* out);
void ci_rdm12(int n, int na, int nb, hipStream_t st, const double* bra, const double* ket, double scale,
              double* gamma, double* Gamma, double* overlap);

}  // namespace dmrg
