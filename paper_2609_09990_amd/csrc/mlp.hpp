// Learned Davidson preconditioner: a per-amplitude 3-layer ReLU network
// F -> W -> W -> 1 (fp32 master weights; bf16 inference on the matrix cores),
// its training (loss, backward, Adam) on the GPU, and the feature and
// training-triple kernels that feed it from the solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "solver.hpp"

namespace dmrg {

// ---- kernels (mlp.hip) ----
// a1[i][j] = max(0, b1[j] + sum_f X[i][f] W1[j][f]); fp32 out and/or bf16 bits out.
// Fused bf16 inference of a width-256 network (n_in <= 16), no activations in
// memory; returns false (nothing launched) for other shapes.
bool launch_mlp_infer_bf16(const float* X, long n, int nin, const float* W1, const float* b1, int width,
                           const uint16_t* W2b, const float* b2, const float* W3, const float* b3, float* y,
                           hipStream_t s);
void launch_mlp_layer1(const float* X, long n, int nin, const float* W1, const float* b1, int width,
                       float* a1, uint16_t* a1b, hipStream_t s);
// y[i] = b3 + sum_j max(0, z2[i][j] + b2[j]) W3[j]; if store, z2 <- max(0, z2 + b2).
void launch_mlp_layer3(float* z2, long n, int width, const float* b2, const float* W3, const float* b3,
                       float* y, bool store, hipStream_t s);
// per segment: [sum y t, sum y y, sum t t] (fp64)
void launch_seg_stats(const float* y, const float* t, int nseg, int seglen, double* stats, hipStream_t s);
// d(mean over segments of 1 - cos(y_seg, t_seg))/dy
void launch_cos_grad(const float* y, const float* t, const double* stats, int nseg, int seglen, float* dy,
                     hipStream_t s);
// partial[c][j] = sum_{i in chunk c} A[i][j] * (w ? w[i * wstride] : 1)  (fp64 accumulation)
void launch_colsum_partial(const float* A, long rows, int cols, const float* w, int wstride, long chunk,
                           double* partial, hipStream_t s);
// out[j * ostride] = sum_c partial[c][j] (in chunk order)
void launch_sum_partials(const double* partial, int nchunks, long cols, float* out, int ostride, hipStream_t s);
void launch_sum_partials_f32(const float* partial, int nchunks, long cols, float* out, hipStream_t s);
// dz2[i][j] = a2[i][j] > 0 ? dy[i] W3[j] : 0 (in place over a2)
void launch_mlp_back3(float* a2, const float* dy, const float* W3, long n, int width, hipStream_t s);
// x[i] = mask[i] > 0 ? x[i] : 0
void launch_relu_mask(float* x, const float* mask, long n, hipStream_t s);
void launch_adam(float* w, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s);
void launch_f32_to_bf16_rne(const float* x, uint16_t* y, long n, hipStream_t s);

// Feature blocks of a two-site vector: {element offset, row stride, rows, cols}.
// stats per block: {s_b, mean(e/s_b), min(e/s_b), log(size)/10}
void launch_feat_stats(const double* d, const double* theta, const int64_t* blocks, int nb, double* stats,
                       hipStream_t s);
// X[i][0..7] (fp32) from r, d, theta, the diagonal candidate t, the block stats and
// the squared norms nrm2[0] = |r|^2, nrm2[1] = |t|^2.
void launch_feat_fill(const double* r, const double* d, const double* theta, const double* t,
                      const int64_t* blocks, int nb, const double* stats, const double* nrr, const double* ntt,
                      long n, float kpos, float* X, hipStream_t s);
// out[j][f] = X[idx[j]][f]
void launch_gather_rows(const float* X, int nf, const int64_t* idx, int m, float* out, hipStream_t s);
// out[j] = sign(c) psi_star[idx[j]] - |c| psi_i[idx[j]], c = cdev[0]
void launch_triple_target(const double* psi_i, const double* psi_star, const double* cdev, const int64_t* idx,
                          int m, float* out, hipStream_t s);

// ---- the network ----
class MLP {
 public:
  MLP(int n_in, int width, unsigned long long seed, hipStream_t s);
  int n_in() const { return nin_; }
  int width() const { return w_; }
  long n_params() const { return np_; }
  void set_params(const float* host);   // resets the Adam state
  void get_params(float* host) const;
  // y[n] = net(X[n][n_in]) with fp32 (PREC_F32) or bf16 (PREC_BF16) hidden GEMM.
  void forward(int prec, const float* X, long n, float* y, hipStream_t s = nullptr);
  // Mean over segments of 1 - cos(net(X_seg), T_seg); gradient kept for adam().
  double loss_grad(const float* X, const float* T, int nseg, int seglen);
  const float* grad() const { return grad_.as<float>(); }
  void adam(float lr, float beta1 = 0.9f, float beta2 = 0.999f, float eps = 1e-8f);
  hipStream_t stream() const { return st_; }

 private:
  int nin_, w_;
  long np_;
  long oW1_, ob1_, oW2_, ob2_, oW3_, ob3_;
  hipStream_t st_;
  DevMem p_, m_, v_, grad_, w2b_;
  DevMem a1_, a1b_, z2_, da1_, y_, dy_, stats_, part_, gpart_;
  int t_ = 0;
  // cached GEMM tables of the hidden layer
  struct Tables {
    const void* key[3] = {nullptr, nullptr, nullptr};
    long rows = -1;
    int mode = -1, prec = -1;
    DevMem du, di;
    std::vector<GemmUnit> hu;
    std::vector<GemmItem> hi;
    int nu = 0;
  } tz_, tda_, tgw_, ti_;
  void gemm(Tables& t, int prec, int mode, const void* A, const void* B, void* C, long rows, hipStream_t s);
  void refresh_bf16();
};

}  // namespace dmrg
