// Device kernels (gfx950) and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmrg {

// One product term of a grouped block GEMM: acc += coef * op(A) * op(B), K deep.
struct GemmItem {
  const void* A;
  const void* B;
  int lda, ldb, K, pad;
  double coef;
};

// One output tile (rows m0.., cols n0.., at most 64 x 64) of an M x N output
// block; it accumulates items [ib, ie) in order (no atomics: deterministic).
// shape (fp64 one-wave kernel only): 8 RB + CB for a (16 RB) x (16 CB) tile,
// RB in 1..4, CB in 1..2 (0 = 32 x 32).
struct GemmUnit {
  void* C;
  int ldc, M, N, m0, n0, ib, ie, accumulate;
  int shape;
};

enum GemmMode : int {
  GEMM_NN = 0,  // A: M x K row-major, B: K x N row-major
  GEMM_NT = 1,  // A: M x K row-major, B: N x K row-major (B transposed)
  GEMM_TN = 2,  // A: K x M row-major (A transposed), B: K x N row-major
};

// Element precision of A and B (C is fp64 for FP64, fp32 otherwise).
enum GemmPrec : int { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

void launch_gemm(int prec, int mode, const GemmUnit* units, int n_units, const GemmItem* items,
                 hipStream_t s);

// fp64 one-wave variant (one wave per unit, tile of 16..64 rows by 16 or 32
// columns from the unit's shape, operands from global memory).  Units with accumulate == 2 write
// the full tile, row-major (tile rows x tile cols), to a partial slot (split-K).
// buf: NN / NT launch whose items all pass buffer_reach_ok (raw buffer loads);
// otherwise plain loads (and any mode).
void launch_gemm_w32(int mode, int tag, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                     hipStream_t s);
// Whether one item may take the buffer-load path: every element offset a tile
// forms from the operand starts (up to 32 past the last row's K, NN rows of B up
// to K + 32) stays below 1 GiB in bytes, so offsets fit 32-bit arithmetic.
inline bool buffer_reach_ok(int mode, int M, int N, int K, int lda, int ldb, size_t esz_a, size_t esz_b) {
  if (mode != GEMM_NN && mode != GEMM_NT) return false;
  const long lim = 1L << 30;
  const long ra = ((long)(M - 1) * lda + K + 32) * (long)esz_a;
  const long rb = (mode == GEMM_NT ? (long)(N - 1) * ldb + K + 32 : (long)(K + 32) * ldb + N) * (long)esz_b;
  return ra < lim && rb < lim;
}

// Output tile (rows m0.., cols n0.. of an M x N block, tm x tn <= 96 x 64
// elements) = sum of ns partial tiles (row-major tm x tn each) stored one after
// another from element s0 of the slot buffer, summed in order; acc = 1 adds
// that sum to the tile instead.
struct SplitTile {
  void* C;
  long s0;
  int ldc, M, N, m0, n0, ns, tm, tn;
  int acc, pad;
};
void launch_splitk_reduce(const SplitTile* tiles, int n, const double* slots, hipStream_t s);
// NT block kernel (prec PREC_F64 or PREC_F32: operands, accumulation and
// outputs in that type): one 256-thread workgroup per unit, tile (16 RB) x
// (16 CB) with RB = shape >> 3 in 1..6 and CB = shape & 7 in 1..4; every item
// must pass buffer_reach_ok.  Partial tiles (accumulate == 2) are 16 CB wide.
void launch_gemm_wg(int prec, int tag, const GemmUnit* units, int n_units, const GemmItem* items, hipStream_t s);
// The same for fp32 operands, fp32 accumulation and fp32 outputs and slots.
void launch_gemm_w32_f32(int mode, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                         hipStream_t s);
void launch_splitk_reduce_f32(const SplitTile* tiles, int n, const float* slots, hipStream_t s);
// bf16 one-wave variant: A bf16 bits (a_f32 = false) or fp32 rounded to bf16,
// B bf16 bits, fp32 accumulation and fp32 outputs / slots.
void launch_gemm_w32_bf16(int mode, bool a_f32, bool buf, const GemmUnit* units, int n_units, const GemmItem* items,
                          hipStream_t s);

// out[f][j] = sum_{i in [ptr[f], ptr[f+1])} coef[i] * src[idx[i]][j], j < nnz.
void launch_premix(double* out, const double* const* srcs, const int* ptr, const double* coef,
                   int n_out, long nnz, hipStream_t s);

// Device ceilings: a register-only fp64 MFMA loop (out: n_blocks * 256 doubles;
// returns the flops launched) and a streaming copy of bytes (multiple of 16,
// 16-byte aligned buffers).
long launch_mfma_f64_peak(double* out, int n_blocks, int iters, hipStream_t s);
void launch_stream_copy(const void* src, void* dst, long bytes, hipStream_t s);
// Per group g: out[out_off[g] + j] = sum_{i in [ptr[g], ptr[g+1])} coef[i] * srcs[i][j], j < nnz[g].
void launch_pairmix(double* out, const double* const* srcs, const int* ptr, const double* coef, const long* out_off,
                    const int* nnz, int n_groups, hipStream_t s);
void launch_fill(double* x, long n, double v, hipStream_t s);
// desc per block (9 x int64): src_off, src_row_stride, src_col_stride, dst_off,
// dst_row_stride, dst_col_stride, rows, cols, scale (bits of a double)
void launch_copy_blocks(const int64_t* desc, int n_blocks, const double* src, double* dst,
                        hipStream_t s);
void launch_axpy_dev(double* y, const double* x, const double* a, double sign, long n, hipStream_t s);
void launch_copy(double* dst, const double* src, long n, hipStream_t s);

// Davidson helpers (all fp64, deterministic two-pass reductions).
void launch_dots(const double* V, long ldv, int k, const double* x, long n, double* partial,
                 double* out, hipStream_t s);
void launch_fill_f32(float* x, long n, hipStream_t s);
void launch_gemv(const double* V, long ldv, int k, const double* coef, double alpha,
                 double* out, double beta, long n, hipStream_t s);
void launch_scale_by_norm(double* x, long n, const double* nrm2, hipStream_t s);
void launch_precond_diag(const double* r, const double* diag, const double* theta, double* out,
                         long n, hipStream_t s);
// dst[idx[i]] = round(src[idx[i]] - w[i] * shift) into an fp32 (bf16 = false) or bf16 copy.
void launch_shift_entries(const double* src, void* dst, bool bf16, const long* idx, const double* w, long n,
                          double shift, hipStream_t s);
// y += a x
void launch_axpy(double* y, const double* x, double a, long n, hipStream_t s);
// y += sign * (num[0] / den[0]) x and p = z + (num[0] / den[0]) p (device scalars)
void launch_axpy_ratio(double* y, const double* x, const double* num, const double* den, double sign, long n,
                       hipStream_t s);
void launch_xpby_ratio(double* p, const double* z, const double* num, const double* den, long n, hipStream_t s);
// d[i] += sum_{j<k} V[j ldv + i]^2.
void launch_add_squares(double* d, const double* V, long ldv, int k, long n, hipStream_t s);
// In place: V[:, i] = sum_{j<k} V[:, j] Y[i k + j] for i < keep (k <= 64, keep <= 16).
void launch_subspace_rotate(double* V, long ldv, int k, const double* Y, int keep, long n, hipStream_t s);
void launch_jacobi_eig(const double* G, int ldg, int k, double* evals, double* evecs,
                       hipStream_t s);

// precision conversions
void launch_f64_to_f32(const double* x, float* y, long n, hipStream_t s);
void launch_f64_to_bf16(const double* x, uint16_t* y, long n, hipStream_t s);
void launch_f32_to_f64(const float* x, double* y, long n, hipStream_t s);

// H_eff diagonal: out[e] = sum_t w_t * xd[tx_t][ia] * yd[ty_t][ib] per block.
struct DiagBlock {
  long out_off;
  int ld, rows, cols, t0, t1;  // rows x cols block at out_off with row stride ld; terms [t0,t1)
};
struct DiagTerm {
  const double* x;  // diagonal of the left factor restricted to the block's row sector
  const double* y;  // diagonal of the right factor restricted to the block's col sector
  double w;
};
void launch_diag(double* out, const DiagBlock* blocks, int n_blocks, const DiagTerm* terms,
                 hipStream_t s);
// diag of each env block: out[j] = blk[j*(ld+1)], used to extract factor diagonals.
void launch_extract_diag(const int64_t* desc, int n, const double* src, double* dst,
                         hipStream_t s);

}  // namespace dmrg
