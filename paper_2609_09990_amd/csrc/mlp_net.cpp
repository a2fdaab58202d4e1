// The preconditioner network on the GPU: parameters, forward (fp32 or bf16
// hidden layer on the matrix cores), cosine loss with backward, and Adam.
#include <algorithm>
#include <cmath>

#include "mlp.hpp"

namespace dmrg {

namespace {
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double normal() {
    double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};
constexpr long kRowChunk = 512;  // rows per partial of the column reductions and split-K chunks
}  // namespace

MLP::MLP(int n_in, int width, unsigned long long seed, hipStream_t s) : nin_(n_in), w_(width), st_(s) {
  DMRG_REQUIRE(n_in >= 1 && n_in <= 64 && width >= 1 && width <= 1024, ST_EINVAL, "network shape out of range");
  oW1_ = 0;
  ob1_ = oW1_ + (long)w_ * nin_;
  oW2_ = ob1_ + w_;
  ob2_ = oW2_ + (long)w_ * w_;
  oW3_ = ob2_ + w_;
  ob3_ = oW3_ + w_;
  np_ = ob3_ + 1;
  // He-normal weights, zero biases
  std::vector<float> h(np_, 0.f);
  SplitMix rng{seed};
  for (long i = 0; i < (long)w_ * nin_; ++i) h[oW1_ + i] = (float)(rng.normal() * std::sqrt(2.0 / nin_));
  for (long i = 0; i < (long)w_ * w_; ++i) h[oW2_ + i] = (float)(rng.normal() * std::sqrt(2.0 / w_));
  for (long i = 0; i < w_; ++i) h[oW3_ + i] = (float)(rng.normal() * std::sqrt(1.0 / w_));
  p_.reserve(np_ * 4);
  m_.reserve(np_ * 4);
  v_.reserve(np_ * 4);
  grad_.reserve(np_ * 4);
  w2b_.reserve((size_t)w_ * w_ * 2);
  set_params(h.data());
}

void MLP::refresh_bf16() { launch_f32_to_bf16_rne(p_.as<float>() + oW2_, w2b_.as<uint16_t>(), (long)w_ * w_, st_); }

void MLP::set_params(const float* host) {
  hip_check(hipMemcpyAsync(p_.p, host, np_ * 4, hipMemcpyHostToDevice, st_), "mlp params");
  hip_check(hipMemsetAsync(m_.p, 0, np_ * 4, st_), "adam m");
  hip_check(hipMemsetAsync(v_.p, 0, np_ * 4, st_), "adam v");
  hip_check(hipMemsetAsync(grad_.p, 0, np_ * 4, st_), "grad");
  t_ = 0;
  refresh_bf16();
  hip_check(hipStreamSynchronize(st_), "mlp params");
}

void MLP::get_params(float* host) const {
  hip_check(hipMemcpyAsync(host, p_.p, np_ * 4, hipMemcpyDeviceToHost, st_), "mlp params");
  hip_check(hipStreamSynchronize(st_), "mlp params");
}

// Hidden-layer GEMMs on 64 x 64 tiles.  mode NT: C[rows x W] = A[rows x W] B^T (B = W2);
// NN: C = A B (B = W2); TN: per chunk of kRowChunk rows a W x W partial A_c^T B_c.
void MLP::gemm(Tables& t, int prec, int mode, const void* A, const void* B, void* C, long rows, hipStream_t s) {
  const bool same = t.key[0] == A && t.key[1] == B && t.key[2] == C && t.rows == rows && t.mode == mode &&
                    t.prec == prec;
  if (!same) {
    hip_check(hipStreamSynchronize(s), "mlp tables");  // earlier uploads of the staging vectors are done
    const size_t ea = prec == PREC_BF16 ? 2 : 4, ec = 4;
    t.hu.clear();
    t.hi.clear();
    if (mode == GEMM_TN) {
      const long nch = (rows + kRowChunk - 1) / kRowChunk;
      for (long c = 0; c < nch; ++c) {
        const long r0 = c * kRowChunk, nr = std::min(kRowChunk, rows - r0);
        int ib = (int)t.hi.size();
        t.hi.push_back({(const char*)A + r0 * w_ * ea, (const char*)B + r0 * w_ * ea, w_, w_, (int)nr, 0, 1.0});
        char* Cc = (char*)C + c * (long)w_ * w_ * ec;
        for (int m0 = 0; m0 < w_; m0 += 64)
          for (int n0 = 0; n0 < w_; n0 += 64) t.hu.push_back({Cc, w_, w_, w_, m0, n0, ib, ib + 1, 0});
      }
    } else {
      // one item per 64-row tile (the A operand moves with the tile), all W columns
      for (long m0 = 0; m0 < rows; m0 += 64) {
        int ib = (int)t.hi.size();
        t.hi.push_back({(const char*)A + m0 * w_ * ea, B, w_, w_, w_, 0, 1.0});
        char* Cm = (char*)C + m0 * w_ * ec;
        const int M = (int)std::min<long>(64, rows - m0);
        for (int n0 = 0; n0 < w_; n0 += 64) t.hu.push_back({Cm, w_, M, w_, 0, n0, ib, ib + 1, 0});
      }
    }
    t.du.reserve(t.hu.size() * sizeof(GemmUnit) + 64);
    t.di.reserve(t.hi.size() * sizeof(GemmItem) + 64);
    hip_check(hipMemcpyAsync(t.du.p, t.hu.data(), t.hu.size() * sizeof(GemmUnit), hipMemcpyHostToDevice, s), "mlp units");
    hip_check(hipMemcpyAsync(t.di.p, t.hi.data(), t.hi.size() * sizeof(GemmItem), hipMemcpyHostToDevice, s), "mlp items");
    t.key[0] = A;
    t.key[1] = B;
    t.key[2] = C;
    t.rows = rows;
    t.mode = mode;
    t.prec = prec;
    t.nu = (int)t.hu.size();
  }
  launch_gemm(prec, mode, t.du.as<GemmUnit>(), t.nu, t.di.as<GemmItem>(), s);
}

void MLP::forward(int prec, const float* X, long n, float* y, hipStream_t s) {
  DMRG_REQUIRE(prec == PREC_F32 || prec == PREC_BF16, ST_EINVAL, "network precision must be FP32 or BF16");
  if (n <= 0) return;
  if (!s) s = st_;
  const float* P = p_.as<float>();
  if (prec == PREC_BF16 && launch_mlp_infer_bf16(X, n, nin_, P + oW1_, P + ob1_, w_, w2b_.as<uint16_t>(), P + ob2_,
                                                 P + oW3_, P + ob3_, y, s))
    return;
  z2_.reserve((size_t)n * w_ * 4);
  if (prec == PREC_BF16) {
    a1b_.reserve((size_t)n * w_ * 2);
    launch_mlp_layer1(X, n, nin_, P + oW1_, P + ob1_, w_, nullptr, a1b_.as<uint16_t>(), s);
    gemm(ti_, PREC_BF16, GEMM_NT, a1b_.p, w2b_.p, z2_.p, n, s);
  } else {
    a1_.reserve((size_t)n * w_ * 4);
    launch_mlp_layer1(X, n, nin_, P + oW1_, P + ob1_, w_, a1_.as<float>(), nullptr, s);
    gemm(ti_, PREC_F32, GEMM_NT, a1_.p, P + oW2_, z2_.p, n, s);
  }
  launch_mlp_layer3(z2_.as<float>(), n, w_, P + ob2_, P + oW3_, P + ob3_, y, false, s);
}

double MLP::loss_grad(const float* X, const float* T, int nseg, int seglen) {
  DMRG_REQUIRE(nseg >= 1 && seglen >= 1, ST_EINVAL, "empty training batch");
  const long n = (long)nseg * seglen;
  const float* P = p_.as<float>();
  float* G = grad_.as<float>();
  a1_.reserve((size_t)n * w_ * 4);
  z2_.reserve((size_t)n * w_ * 4);
  da1_.reserve((size_t)n * w_ * 4);
  y_.reserve((size_t)n * 4);
  dy_.reserve((size_t)n * 4);
  stats_.reserve((size_t)nseg * 3 * 8);
  const int nch = (int)((n + kRowChunk - 1) / kRowChunk);
  part_.reserve((size_t)nch * std::max<long>(w_, 1) * 8);
  gpart_.reserve((size_t)nch * w_ * w_ * 4);
  // forward (fp32), keeping a1 and a2
  launch_mlp_layer1(X, n, nin_, P + oW1_, P + ob1_, w_, a1_.as<float>(), nullptr, st_);
  gemm(tz_, PREC_F32, GEMM_NT, a1_.p, P + oW2_, z2_.p, n, st_);
  launch_mlp_layer3(z2_.as<float>(), n, w_, P + ob2_, P + oW3_, P + ob3_, y_.as<float>(), true, st_);
  // loss and dL/dy
  launch_seg_stats(y_.as<float>(), T, nseg, seglen, stats_.as<double>(), st_);
  launch_cos_grad(y_.as<float>(), T, stats_.as<double>(), nseg, seglen, dy_.as<float>(), st_);
  // layer 3: dW3 = sum_i dy_i a2_i, db3 = sum_i dy_i
  launch_colsum_partial(z2_.as<float>(), n, w_, dy_.as<float>(), 1, kRowChunk, part_.as<double>(), st_);
  launch_sum_partials(part_.as<double>(), nch, w_, G + oW3_, 1, st_);
  launch_colsum_partial(dy_.as<float>(), n, 1, nullptr, 1, kRowChunk, part_.as<double>(), st_);
  launch_sum_partials(part_.as<double>(), nch, 1, G + ob3_, 1, st_);
  // dz2 (in place over a2), dW2 = dz2^T a1, db2 = colsum dz2
  launch_mlp_back3(z2_.as<float>(), dy_.as<float>(), P + oW3_, n, w_, st_);
  gemm(tgw_, PREC_F32, GEMM_TN, z2_.p, a1_.p, gpart_.p, n, st_);
  launch_sum_partials_f32(gpart_.as<float>(), nch, (long)w_ * w_, G + oW2_, st_);
  launch_colsum_partial(z2_.as<float>(), n, w_, nullptr, 1, kRowChunk, part_.as<double>(), st_);
  launch_sum_partials(part_.as<double>(), nch, w_, G + ob2_, 1, st_);
  // da1 = dz2 W2, dz1 = da1 * (a1 > 0); dW1[j][f] = sum_i dz1[i][j] X[i][f], db1 = colsum dz1
  gemm(tda_, PREC_F32, GEMM_NN, z2_.p, P + oW2_, da1_.p, n, st_);
  launch_relu_mask(da1_.as<float>(), a1_.as<float>(), n * w_, st_);
  for (int f = 0; f < nin_; ++f) {
    launch_colsum_partial(da1_.as<float>(), n, w_, X + f, nin_, kRowChunk, part_.as<double>(), st_);
    launch_sum_partials(part_.as<double>(), nch, w_, G + oW1_ + f, nin_, st_);
  }
  launch_colsum_partial(da1_.as<float>(), n, w_, nullptr, 1, kRowChunk, part_.as<double>(), st_);
  launch_sum_partials(part_.as<double>(), nch, w_, G + ob1_, 1, st_);
  std::vector<double> hs((size_t)nseg * 3);
  hip_check(hipMemcpyAsync(hs.data(), stats_.p, hs.size() * 8, hipMemcpyDeviceToHost, st_), "loss");
  hip_check(hipStreamSynchronize(st_), "loss");
  double loss = 0.0;
  for (int s = 0; s < nseg; ++s) {
    double yt = hs[3 * s], yy = hs[3 * s + 1], tt = hs[3 * s + 2];
    double c = (yy > 0 && tt > 0) ? yt / std::sqrt(yy * tt) : 0.0;
    loss += (1.0 - c) / nseg;
  }
  return loss;
}

void MLP::adam(float lr, float beta1, float beta2, float eps) {
  ++t_;
  const float c1 = 1.f - std::pow(beta1, (float)t_), c2 = 1.f - std::pow(beta2, (float)t_);
  launch_adam(p_.as<float>(), m_.as<float>(), v_.as<float>(), grad_.as<float>(), np_, lr, beta1, beta2, eps, c1, c2,
              st_);
  refresh_bf16();
  hip_check(hipStreamSynchronize(st_), "adam");
}

}  // namespace dmrg
