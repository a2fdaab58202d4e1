// Solver side of the learned Davidson preconditioner: selection, per-amplitude
// features of a correction, and the training-triple store.
#include <algorithm>

#include "mlp.hpp"
#include "solver.hpp"

namespace dmrg {

void Solver::set_precond(int mode, MLP* net) {
  DMRG_REQUIRE(mode >= 0 && mode <= 3, ST_EINVAL, "preconditioner must be DIAG, LEARNED, OLSEN or SHIFT_INVERT");
  DMRG_REQUIRE(mode != 1 || net, ST_EINVAL, "the learned preconditioner needs a network");
  DMRG_REQUIRE(!net || (net->n_in() == 8), ST_EINVAL, "the preconditioner network takes 8 features");
  precond_ = mode;
  net_ = net;
}

void Solver::record_triples(int capacity, int sample) {
  DMRG_REQUIRE(capacity >= 0 && sample >= 0, ST_EINVAL, "negative triple capacity");
  DMRG_REQUIRE(capacity == 0 || sample >= 16, ST_EINVAL, "triples need at least 16 amplitudes");
  rec_cap_ = capacity;
  rec_sample_ = sample;
  rec_count_ = 0;
  if (capacity > 0) {
    rec_X_.reserve((size_t)capacity * sample * 8 * 4);
    rec_T_.reserve((size_t)capacity * sample * 4);
  } else {
    rec_X_.release();
    rec_T_.release();
    rec_hist_.release();
  }
}

int Solver::take_triples(float* X, float* T, int cap) {
  DMRG_REQUIRE(cap >= 0, ST_EINVAL, "negative capacity");
  int m = std::min(cap, rec_count_);
  if (m > 0) {
    hip_check(hipMemcpyAsync(X, rec_X_.p, (size_t)m * rec_sample_ * 8 * 4, hipMemcpyDeviceToDevice, st), "triples X");
    hip_check(hipMemcpyAsync(T, rec_T_.p, (size_t)m * rec_sample_ * 4, hipMemcpyDeviceToDevice, st), "triples T");
    hip_check(hipStreamSynchronize(st), "triples");
  }
  rec_count_ = 0;
  return m;
}

// X[n][8] for the prepared step; r, d, t = diagonal candidate, theta: device arrays.
void Solver::features(const double* r, const double* d, const double* theta, const double* t, float* X) {
  const long n = psi_lay_.size;
  double* sc = dv_sc_.as<double>();
  double* part = dv_part_.as<double>();
  fstats_.reserve((size_t)std::max(nfb_, 1) * 4 * 8);
  launch_dots(r, n, 1, r, n, part, sc + 200, st);
  launch_dots(t, n, 1, t, n, part, sc + 201, st);
  launch_feat_stats(d, theta, d_fblocks_.as<int64_t>(), nfb_, fstats_.as<double>(), st);
  launch_feat_fill(r, d, theta, t, d_fblocks_.as<int64_t>(), nfb_, fstats_.as<double>(), sc + 200, sc + 201, n,
                   (float)plan_k_ / (float)L_, X, st);
}

void Solver::features_host_theta(int k, const double* r, const double* d, double theta, float* X) {
  if (plan_k_ != k) prepare(k);
  const long n = psi_lay_.size;
  dv_sc_.reserve(256 * 8);
  dv_part_.reserve((size_t)512 * 64 * 8);
  feat_t_.reserve((size_t)n * 8);
  double* sc = dv_sc_.as<double>();
  hip_check(hipMemcpyAsync(sc + 202, &theta, 8, hipMemcpyHostToDevice, st), "theta");
  launch_precond_diag(r, d, sc + 202, feat_t_.as<double>(), n, st);
  features(r, d, sc + 202, feat_t_.as<double>(), X);
  hip_check(hipStreamSynchronize(st), "features");
}

}  // namespace dmrg
