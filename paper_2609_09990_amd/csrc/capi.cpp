// C ABI over the solver: argument checks, exception-to-status translation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "../../include/dmrg_mi355x.h"
#include "capi_guard.hpp"
#include "mlp.hpp"
#include "solver.hpp"

using namespace dmrg;

struct dmrg_problem {
  Problem p;
};
struct dmrg_solver {
  std::unique_ptr<Arena> arena;  // the attached workspace (outlives s)
  Solver* s = nullptr;
  const dmrg_problem* prob = nullptr;
  Options opt;
  hipStream_t stream = nullptr;
  long allocs_at_attach = -1;
};

namespace {
// Body of a call on a solver: buffers come from its workspace when one is
// attached, and the initial MPS reaches the device on the first such call.
template <class F>
dmrg_status solver_call(dmrg_solver* s, F&& f) {
  return guard([&] {
    DMRG_REQUIRE(s && s->s, ST_EINVAL, "NULL solver");
    ArenaScope scope(s->arena.get());
    s->s->materialize();
    f();
  });
}
}  // namespace
struct dmrg_mlp {
  MLP* m = nullptr;
};

namespace dmrg {
std::string& last_error_slot() {
  thread_local std::string msg;
  return msg;
}
}  // namespace dmrg

extern "C" {

const char* dmrg_last_error(void) { return last_error_slot().c_str(); }

void dmrg_options_default(dmrg_options* o) {
  if (!o) return;
  o->M = 256;
  o->n_states = 1;
  o->weights = nullptr;
  o->davidson_tol = 1e-10;
  o->max_iter = 200;
  o->max_subspace = 32;
  o->precision = DMRG_FP64;
  o->precond = DMRG_PRECOND_DIAG;
  o->seed = 1;
  o->tie_rtol = 1e-10;
  o->cut_rtol = 1e-14;
  o->verbose = 0;
  o->sigma_chunk_bytes = 0;
  o->pcg_steps = 5;
  o->pcg_rtol = 0.1;
  o->trunc_tol = 0;
  o->m_min = 1;
}

dmrg_status dmrg_problem_create(int n, int na, int nb, int nq, const double* h, const double* B,
                                double e_core, dmrg_problem** out) {
  return guard([&] {
    DMRG_REQUIRE(out, ST_EINVAL, "out is NULL");
    *out = nullptr;
    DMRG_REQUIRE(n >= 2 && n <= 64, ST_EINVAL, "n_orb must be in [2, 64]");
    DMRG_REQUIRE(na >= 0 && nb >= 0 && na <= n && nb <= n, ST_ESECTOR, "electron counts outside [0, n_orb]");
    DMRG_REQUIRE(nq >= 0, ST_EINVAL, "n_chol must be >= 0");
    DMRG_REQUIRE(h && (nq == 0 || B), ST_EINVAL, "h or B is NULL");
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        DMRG_REQUIRE(std::isfinite(h[p * n + q]), ST_EINVAL, "h has a non-finite entry");
        DMRG_REQUIRE(std::fabs(h[p * n + q] - h[q * n + p]) <= 1e-12, ST_EINVAL, "h is not symmetric");
      }
    for (int Q = 0; Q < nq; ++Q)
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
          double x = B[((size_t)Q * n + p) * n + q], y = B[((size_t)Q * n + q) * n + p];
          DMRG_REQUIRE(std::isfinite(x), ST_EINVAL, "B has a non-finite entry");
          DMRG_REQUIRE(std::fabs(x - y) <= 1e-12, ST_EINVAL, "B^Q is not symmetric");
        }
    auto* P = new dmrg_problem;
    P->p.n = n;
    P->p.n_alpha = na;
    P->p.n_beta = nb;
    P->p.nq = nq;
    P->p.e_core = e_core;
    P->p.h.assign(h, h + (size_t)n * n);
    if (nq) P->p.B.assign(B, B + (size_t)nq * n * n);
    try {
      P->p.mpo = build_mpo(n, nq, P->p.h.data(), P->p.B.data());
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
  });
}

void dmrg_problem_destroy(dmrg_problem* p) { delete p; }

dmrg_status dmrg_mpo_dims(const dmrg_problem* p, int* dims) {
  return guard([&] {
    DMRG_REQUIRE(p && dims, ST_EINVAL, "NULL argument");
    for (int c = 0; c <= p->p.n; ++c) dims[c] = p->p.mpo.dim(c);
  });
}

dmrg_status dmrg_mpo_site_nnz(const dmrg_problem* p, int site, int* nnz) {
  return guard([&] {
    DMRG_REQUIRE(p && nnz, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(site >= 0 && site < p->p.n, ST_EINVAL, "site out of range");
    *nnz = (int)p->p.mpo.W[site].size();
  });
}

dmrg_status dmrg_mpo_site(const dmrg_problem* p, int site, int* a, int* b, double* c, double* op) {
  return guard([&] {
    DMRG_REQUIRE(p && a && b && c && op, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(site >= 0 && site < p->p.n, ST_EINVAL, "site out of range");
    const auto& W = p->p.mpo.W[site];
    for (size_t i = 0; i < W.size(); ++i) {
      a[i] = W[i].a;
      b[i] = W[i].b;
      c[i] = W[i].c;
      std::memcpy(op + 16 * i, p->p.mpo.ops[W[i].op].data(), 16 * sizeof(double));
    }
  });
}

dmrg_status dmrg_solver_create(const dmrg_problem* p, const dmrg_options* o, void* stream,
                               dmrg_solver** out) {
  return guard([&] {
    DMRG_REQUIRE(p && out, ST_EINVAL, "NULL argument");
    *out = nullptr;
    Options op;
    dmrg_options d;
    dmrg_options_default(&d);
    if (!o) o = &d;
    op.M = o->M;
    op.n_states = o->n_states;
    if (o->weights) op.weights.assign(o->weights, o->weights + std::max(o->n_states, 0));
    op.davidson_tol = o->davidson_tol;
    op.max_iter = o->max_iter;
    op.max_subspace = o->max_subspace;
    op.precision = o->precision;
    op.precond = o->precond;
    op.seed = o->seed;
    op.tie_rtol = o->tie_rtol;
    op.cut_rtol = o->cut_rtol;
    op.verbose = o->verbose;
    DMRG_REQUIRE(o->sigma_chunk_bytes >= 0, ST_EINVAL, "sigma_chunk_bytes must be >= 0");
    if (o->sigma_chunk_bytes > 0) op.sigma_chunk_bytes = o->sigma_chunk_bytes;
    DMRG_REQUIRE(o->pcg_steps >= 1 && o->pcg_rtol >= 0, ST_EINVAL, "pcg_steps must be >= 1 and pcg_rtol >= 0");
    op.pcg_steps = o->pcg_steps;
    op.pcg_rtol = o->pcg_rtol;
    DMRG_REQUIRE(o->trunc_tol >= 0 && o->trunc_tol < 1 && o->m_min >= 1, ST_EINVAL,
                 "trunc_tol must be in [0, 1) and m_min >= 1");
    op.trunc_tol = o->trunc_tol;
    op.m_min = o->m_min;
    DMRG_REQUIRE(op.precision >= 0 && op.precision <= 2, ST_EINVAL, "unknown precision");
    DMRG_REQUIRE(op.davidson_tol > 0, ST_EINVAL, "davidson_tol must be positive");
    DMRG_REQUIRE(op.max_iter >= 1, ST_EINVAL, "max_iter must be >= 1");
    auto* S = new dmrg_solver;
    S->prob = p;
    S->opt = op;
    S->stream = (hipStream_t)stream;
    try {
      S->s = new Solver(&p->p, op, (hipStream_t)stream);
    } catch (...) {
      delete S;
      throw;
    }
    *out = S;
  });
}

void dmrg_solver_destroy(dmrg_solver* s) {
  if (!s) return;
  try {
    delete s->s;  // buffers return to the workspace, which is dropped after it
  } catch (...) {
  }
  delete s;
}

dmrg_status dmrg_set_mps(dmrg_solver* s, const int* n_sec, const int* sec, const double* data) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && n_sec && sec && data, ST_EINVAL, "NULL argument");
    int L = s->prob->p.n;
    std::vector<Bond> bonds(L + 1);
    long idx = 0;
    for (int c = 0; c <= L; ++c) {
      DMRG_REQUIRE(n_sec[c] >= 1, ST_EINVAL, "every bond needs at least one sector");
      for (int i = 0; i < n_sec[c]; ++i, ++idx)
        bonds[c].sec.push_back({{sec[3 * idx], sec[3 * idx + 1]}, sec[3 * idx + 2]});
    }
    std::vector<const double*> sites(L);
    long off = 0;
    for (int k = 0; k < L; ++k) {
      sites[k] = data + off;
      off += make_tensor_layout(bonds[k], bonds[k + 1], site_phys_qn()).size;
    }
    s->s->set_mps(bonds, sites);
  });
}

dmrg_status dmrg_get_bonds(const dmrg_solver* s, int* n_sec, int* sec, int cap) {
  return guard([&] {
    DMRG_REQUIRE(s && n_sec && sec, ST_EINVAL, "NULL argument");
    const auto& b = s->s->bonds();
    int idx = 0;
    for (size_t c = 0; c < b.size(); ++c) {
      n_sec[c] = (int)b[c].sec.size();
      for (auto& x : b[c].sec) {
        DMRG_REQUIRE(idx < cap, ST_EINVAL, "sector capacity too small");
        sec[3 * idx] = x.q.n;
        sec[3 * idx + 1] = x.q.sz;
        sec[3 * idx + 2] = x.dim;
        ++idx;
      }
    }
  });
}

dmrg_status dmrg_prepare(dmrg_solver* s, int k, int64_t* n) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL solver");
    s->s->prepare(k);
    if (n) *n = s->s->twosite_size(k);
  });
}

dmrg_status dmrg_sigma(dmrg_solver* s, int k, int precision, int64_t n, const double* psi, double* sigma,
                       double* flops) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && psi && sigma, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(precision >= 0 && precision <= 2, ST_EINVAL, "unknown precision");
    const long len = s->s->twosite_size(k);
    DMRG_REQUIRE(n == len, ST_EINVAL,
                 "vector length " + std::to_string(n) + " is not the two-site length " + std::to_string(len));
    s->s->sigma(k, precision, psi, sigma);
    if (flops) *flops = s->s->last_sigma_flops_exec();
  });
}

dmrg_status dmrg_diag(dmrg_solver* s, int k, int64_t n, double* diag) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && diag, ST_EINVAL, "NULL argument");
    const long len = s->s->twosite_size(k);
    DMRG_REQUIRE(n == len, ST_EINVAL,
                 "vector length " + std::to_string(n) + " is not the two-site length " + std::to_string(len));
    s->s->diag(k, diag);
    hip_check(hipDeviceSynchronize(), "diag");
  });
}

dmrg_status dmrg_export_mps(dmrg_solver* s, int* n_sec, int* sec, int sec_cap, double* data, int64_t data_cap,
                            int64_t* data_size) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && n_sec && data_size, ST_EINVAL, "NULL argument");
    const auto& b = s->s->bonds();
    int total_sec = 0;
    for (size_t c = 0; c < b.size(); ++c) {
      n_sec[c] = (int)b[c].sec.size();
      total_sec += n_sec[c];
    }
    if (sec) {
      DMRG_REQUIRE(sec_cap >= total_sec, ST_EINVAL, "sector capacity too small");
      int idx = 0;
      for (const auto& bond : b)
        for (const auto& x : bond.sec) {
          sec[3 * idx] = x.q.n;
          sec[3 * idx + 1] = x.q.sz;
          sec[3 * idx + 2] = x.dim;
          ++idx;
        }
    }
    long total = 0;
    for (size_t c = 0; c + 1 < b.size(); ++c)
      total += make_tensor_layout(b[c], b[c + 1], site_phys_qn()).size;
    *data_size = total;
    if (data) {
      DMRG_REQUIRE(data_cap >= total, ST_EINVAL, "data capacity too small");
      std::vector<double> v = s->s->export_mps();
      std::memcpy(data, v.data(), v.size() * sizeof(double));
    }
  });
}

dmrg_status dmrg_truncate(dmrg_solver* s, int k, int direction, int64_t n, const double* psi, double* tau,
                          double* sv, int sv_cap, int* n_kept) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && psi && tau && n_kept, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(direction == 0 || direction == 1, ST_EINVAL, "direction must be 0 or 1");
    const long len = s->s->twosite_size(k);
    DMRG_REQUIRE(n == len, ST_EINVAL,
                 "vector length " + std::to_string(n) + " is not the two-site length " + std::to_string(len));
    *tau = s->s->truncate(k, direction == 0, psi);
    const auto& kept = s->s->last_kept_sv();
    *n_kept = (int)kept.size();
    if (sv)
      for (int i = 0; i < sv_cap && i < (int)kept.size(); ++i) sv[i] = kept[i];
  });
}

dmrg_status dmrg_stationarize(dmrg_solver* s, int n_sweeps, double* energy, double* tangent_residual) {
  dmrg_status st = solver_call(s, [&] {
    DMRG_REQUIRE(s && energy, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(n_sweeps >= 1, ST_EINVAL, "n_sweeps must be >= 1");
    std::vector<double> e;
    const double r = s->s->stationarize(n_sweeps, e);
    *energy = e.empty() ? 0.0 : e[0];
    if (tangent_residual) *tangent_residual = r;
  });
  if (st == DMRG_OK && s && !s->s->last_converged()) {
    last_error_slot() = "Davidson did not reach the tolerance in at least one step";
    return DMRG_ENOCONV;
  }
  return st;
}

dmrg_status dmrg_sweep(dmrg_solver* s, int n_sweeps, double* energies, double* tau) {
  dmrg_status st = solver_call(s, [&] {
    DMRG_REQUIRE(s && energies, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(n_sweeps >= 1, ST_EINVAL, "n_sweeps must be >= 1");
    std::vector<double> e;
    double t = s->s->sweep(n_sweeps, e);
    for (size_t i = 0; i < e.size(); ++i) energies[i] = e[i];
    if (tau) *tau = t;
  });
  if (st == DMRG_OK && s && !s->s->last_converged()) {
    last_error_slot() = "Davidson did not reach the tolerance in at least one step";
    return DMRG_ENOCONV;
  }
  return st;
}

dmrg_status dmrg_step(dmrg_solver* s, int k, int direction, double* energies, double* tau) {
  dmrg_status st = solver_call(s, [&] {
    DMRG_REQUIRE(s && energies, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(direction == 0 || direction == 1, ST_EINVAL, "direction must be 0 or 1");
    std::vector<double> e;
    double t = s->s->step(k, direction == 0, e);
    for (size_t i = 0; i < e.size(); ++i) energies[i] = e[i];
    if (tau) *tau = t;
  });
  if (st == DMRG_OK && s && !s->s->last_converged()) {
    last_error_slot() = "Davidson did not reach the tolerance";
    return DMRG_ENOCONV;
  }
  return st;
}

dmrg_status dmrg_energy(dmrg_solver* s, double* energies) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && energies, ST_EINVAL, "NULL argument");
    auto e = s->s->mps_energy();
    for (size_t i = 0; i < e.size(); ++i) energies[i] = e[i];
  });
}

dmrg_status dmrg_deflate_add(dmrg_solver* s, const int* n_sec, const int* sec, const double* data, double weight) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && n_sec && sec && data, ST_EINVAL, "NULL argument");
    int L = s->prob->p.n;
    std::vector<Bond> bonds(L + 1);
    long idx = 0;
    for (int c = 0; c <= L; ++c) {
      DMRG_REQUIRE(n_sec[c] >= 1, ST_EINVAL, "every bond needs at least one sector");
      for (int i = 0; i < n_sec[c]; ++i, ++idx)
        bonds[c].sec.push_back({{sec[3 * idx], sec[3 * idx + 1]}, sec[3 * idx + 2]});
    }
    std::vector<const double*> sites(L);
    long off = 0;
    for (int k = 0; k < L; ++k) {
      sites[k] = data + off;
      off += make_tensor_layout(bonds[k], bonds[k + 1], site_phys_qn()).size;
    }
    s->s->deflate_add(bonds, sites, weight);
  });
}

dmrg_status dmrg_deflate_clear(dmrg_solver* s) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    s->s->deflate_clear();
  });
}

dmrg_status dmrg_deflate_project(dmrg_solver* s, int k, int j, int64_t n, double* phi) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && phi, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(n == s->s->twosite_size(k), ST_EINVAL, "length does not match the two-site space of step k");
    s->s->deflate_project(k, j, 1.0, phi);
  });
}

dmrg_status dmrg_overlap(dmrg_solver* s, int j, double* overlap) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && overlap, ST_EINVAL, "NULL argument");
    *overlap = s->s->overlap(j);
  });
}

dmrg_status dmrg_s_squared(dmrg_solver* s, double* s2) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && s2, ST_EINVAL, "NULL argument");
    auto v = s->s->s_squared();
    for (size_t i = 0; i < v.size(); ++i) s2[i] = v[i];
  });
}

dmrg_status dmrg_ci_dims(const dmrg_problem* p, int64_t* n_alpha_strings, int64_t* n_beta_strings) {
  return guard([&] {
    DMRG_REQUIRE(p && n_alpha_strings && n_beta_strings, ST_EINVAL, "NULL argument");
    *n_alpha_strings = ci_dimension(p->p.n, p->p.n_alpha, 0);
    *n_beta_strings = ci_dimension(p->p.n, p->p.n_beta, 0);
  });
}

dmrg_status dmrg_mps_to_ci(dmrg_solver* s, int state, double* c, int64_t n) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && c, ST_EINVAL, "NULL argument");
    const Problem& P = s->prob->p;
    DMRG_REQUIRE(n == ci_dimension(P.n, P.n_alpha, P.n_beta), ST_EINVAL, "n must be the CI dimension");
    s->s->mps_to_ci(state, c);
  });
}

static void require_ci_length(const dmrg_problem* p, int64_t n) {
  const long len = ci_dimension(p->p.n, p->p.n_alpha, p->p.n_beta);
  DMRG_REQUIRE(n == len, ST_EINVAL, "vector length " + std::to_string(n) + " is not the CI dimension " +
                                        std::to_string(len));
}

dmrg_status dmrg_ci_rdm12(const dmrg_problem* p, int64_t n, const double* bra, const double* ket, double* gamma,
                          double* Gamma, double* overlap, void* stream) {
  return guard([&] {
    DMRG_REQUIRE(p && bra && ket, ST_EINVAL, "NULL argument");
    require_ci_length(p, n);
    ci_rdm12(p->p.n, p->p.n_alpha, p->p.n_beta, (hipStream_t)stream, bra, ket, 1.0, gamma, Gamma, overlap);
  });
}

dmrg_status dmrg_ci_apply_v(const dmrg_problem* p, int64_t n, const double* c, double* out, void* stream) {
  return guard([&] {
    DMRG_REQUIRE(p && c && out, ST_EINVAL, "NULL argument");
    require_ci_length(p, n);
    DMRG_REQUIRE(c != out, ST_EINVAL, "out must not alias c");
    ci_apply_v(p->p.n, p->p.n_alpha, p->p.n_beta, p->p.nq, p->p.B.data(), (hipStream_t)stream, c, out);
  });
}

dmrg_status dmrg_ci_rdm3(const dmrg_problem* p, int64_t n, const double* bra, const double* ket, double* Gamma3,
                         void* stream) {
  return guard([&] {
    DMRG_REQUIRE(p && bra && ket && Gamma3, ST_EINVAL, "NULL argument");
    require_ci_length(p, n);
    ci_rdm3(p->p.n, p->p.n_alpha, p->p.n_beta, (hipStream_t)stream, bra, ket, 1.0, Gamma3);
  });
}

dmrg_status dmrg_orbital_rdm2(const dmrg_problem* p, int64_t n, const double* c, double* rho, void* stream) {
  return guard([&] {
    DMRG_REQUIRE(p && c && rho, ST_EINVAL, "NULL argument");
    require_ci_length(p, n);
    std::vector<double> r;
    orbital_rdm2(p->p.n, p->p.n_alpha, p->p.n_beta, (hipStream_t)stream, c, r);
    std::copy(r.begin(), r.end(), rho);
  });
}

dmrg_status dmrg_mutual_information(const dmrg_problem* p, int64_t n, const double* c, double* s1, double* I,
                                    void* stream) {
  return guard([&] {
    DMRG_REQUIRE(p && c && s1 && I, ST_EINVAL, "NULL argument");
    require_ci_length(p, n);
    mutual_information(p->p.n, p->p.n_alpha, p->p.n_beta, (hipStream_t)stream, c, s1, I);
  });
}

dmrg_status dmrg_mps_orbital_rdm2(dmrg_solver* s, double* rho, double* s1, double* I) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    const std::vector<double> r = s->s->pair_rdm_mps();
    if (rho) std::copy(r.begin(), r.end(), rho);
    if (s1 && I) mutual_information_of(s->prob->p.n, r, s1, I);
  });
}

dmrg_status dmrg_fiedler_order(int n, const double* I, int* order, double* fiedler) {
  return guard([&] {
    DMRG_REQUIRE(I && order, ST_EINVAL, "NULL argument");
    fiedler_order(n, I, order, fiedler);
  });
}

dmrg_status dmrg_rdm12(dmrg_solver* s, int bra_state, int ket_state, double* gamma, double* Gamma, double* overlap) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    const Problem& P = s->prob->p;
    const long N = ci_dimension(P.n, P.n_alpha, P.n_beta);
    DevMem cb, ck, part, nrm;
    cb.reserve((size_t)N * 8);
    s->s->mps_to_ci(bra_state, cb.as<double>());
    const bool same = bra_state == ket_state;
    if (!same) {
      ck.reserve((size_t)N * 8);
      s->s->mps_to_ci(ket_state, ck.as<double>());
    }
    const double* kv = same ? cb.as<double>() : ck.as<double>();
    part.reserve((size_t)512 * 64 * 8);
    nrm.reserve(16);
    launch_dots(cb.as<double>(), N, 1, cb.as<double>(), N, part.as<double>(), nrm.as<double>(), s->stream);
    launch_dots(kv, N, 1, kv, N, part.as<double>(), nrm.as<double>() + 1, s->stream);
    double h[2];
    hip_check(hipMemcpyAsync(h, nrm.p, 16, hipMemcpyDeviceToHost, s->stream), "norms");
    hip_check(hipStreamSynchronize(s->stream), "norms");
    DMRG_REQUIRE(h[0] > 0 && h[1] > 0, ST_ESTATE, "a state has zero norm");
    const double scale = 1.0 / std::sqrt(h[0] * h[1]);
    double ov = 0;
    ci_rdm12(P.n, P.n_alpha, P.n_beta, s->stream, cb.as<double>(), kv, scale, gamma, Gamma, &ov);
    if (overlap) *overlap = ov * scale;
  });
}

dmrg_status dmrg_grad(dmrg_solver* s, const double* state_weights, double* dE_dh, double* dE_dB,
                      double* energies) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && dE_dh && (dE_dB || s->prob->p.nq == 0), ST_EINVAL, "NULL argument");
    const Problem& P = s->prob->p;
    int ns = s->s->n_states();
    std::vector<double> w(ns, 0.0);
    if (state_weights) w.assign(state_weights, state_weights + ns);
    else w[0] = 1.0;
    std::vector<double> dh, dB, e;
    s->s->grad(w, dh, dB, e);
    std::memcpy(dE_dh, dh.data(), (size_t)P.n * P.n * sizeof(double));
    if (P.nq > 0) std::memcpy(dE_dB, dB.data(), (size_t)P.nq * P.n * P.n * sizeof(double));
    if (energies) std::memcpy(energies, e.data(), e.size() * sizeof(double));
  });
}

dmrg_status dmrg_mlp_create(int n_in, int width, unsigned long long seed, void* hip_stream, dmrg_mlp** out) {
  return guard([&] {
    DMRG_REQUIRE(out, ST_EINVAL, "NULL argument");
    *out = nullptr;
    auto* m = new dmrg_mlp;
    try {
      m->m = new MLP(n_in, width, seed, (hipStream_t)hip_stream);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

void dmrg_mlp_destroy(dmrg_mlp* m) {
  if (!m) return;
  delete m->m;
  delete m;
}

dmrg_status dmrg_mlp_num_params(const dmrg_mlp* m, int64_t* n) {
  return guard([&] {
    DMRG_REQUIRE(m && n, ST_EINVAL, "NULL argument");
    *n = m->m->n_params();
  });
}

dmrg_status dmrg_mlp_set_params(dmrg_mlp* m, const float* host, int64_t n) {
  return guard([&] {
    DMRG_REQUIRE(m && host, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(n == m->m->n_params(), ST_EINVAL, "parameter count mismatch");
    m->m->set_params(host);
  });
}

dmrg_status dmrg_mlp_get_params(const dmrg_mlp* m, float* host, int64_t n) {
  return guard([&] {
    DMRG_REQUIRE(m && host, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(n == m->m->n_params(), ST_EINVAL, "parameter count mismatch");
    m->m->get_params(host);
  });
}

dmrg_status dmrg_mlp_forward(dmrg_mlp* m, int precision, const float* X, int64_t rows, float* y) {
  return guard([&] {
    DMRG_REQUIRE(m && (rows == 0 || (X && y)), ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(rows >= 0, ST_EINVAL, "negative row count");
    m->m->forward(precision, X, rows, y);
    hip_check(hipStreamSynchronize(m->m->stream()), "mlp forward");
  });
}

dmrg_status dmrg_mlp_loss_grad(dmrg_mlp* m, const float* X, const float* target, int n_seg, int seg_len,
                               double* loss, float* grad) {
  return guard([&] {
    DMRG_REQUIRE(m && X && target && loss, ST_EINVAL, "NULL argument");
    *loss = m->m->loss_grad(X, target, n_seg, seg_len);
    if (grad) {
      hip_check(hipMemcpyAsync(grad, m->m->grad(), m->m->n_params() * 4, hipMemcpyDeviceToHost, m->m->stream()),
                "mlp grad");
      hip_check(hipStreamSynchronize(m->m->stream()), "mlp grad");
    }
  });
}

dmrg_status dmrg_mlp_adam_step(dmrg_mlp* m, double lr) {
  return guard([&] {
    DMRG_REQUIRE(m, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(lr > 0 && std::isfinite(lr), ST_EINVAL, "learning rate must be positive");
    m->m->adam((float)lr);
  });
}

dmrg_status dmrg_set_precision(dmrg_solver* s, int precision) {
  return guard([&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    s->s->set_precision(precision);
  });
}

dmrg_status dmrg_set_precond(dmrg_solver* s, int precond, dmrg_mlp* net) {
  return guard([&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    s->s->set_precond(precond, net ? net->m : nullptr);
  });
}

dmrg_status dmrg_record_triples(dmrg_solver* s, int capacity, int sample) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s, ST_EINVAL, "NULL argument");
    s->s->record_triples(capacity, sample);
  });
}

dmrg_status dmrg_take_triples(dmrg_solver* s, float* X, float* target, int cap, int* count) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && count && (cap == 0 || (X && target)), ST_EINVAL, "NULL argument");
    *count = s->s->take_triples(X, target, cap);
  });
}

dmrg_status dmrg_precond_features(dmrg_solver* s, int k, int64_t n, const double* r, const double* d, double theta,
                                  float* X) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && r && d && X, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(k >= 0 && k + 1 < s->prob->p.n, ST_EINVAL, "two-site step out of range");
    DMRG_REQUIRE(n == s->s->twosite_size(k), ST_EINVAL, "vector length is not the two-site length");
    s->s->features_host_theta(k, r, d, theta, X);
  });
}

dmrg_status dmrg_correction(dmrg_solver* s, int k, int mode, int64_t n, const double* x, const double* r,
                            const double* d, double theta, double* t, int* products) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && x && r && d && t, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(k >= 0 && k + 1 < s->prob->p.n, ST_EINVAL, "two-site step out of range");
    DMRG_REQUIRE(n == s->s->twosite_size(k), ST_EINVAL, "vector length is not the two-site length");
    DMRG_REQUIRE(mode == DMRG_PRECOND_DIAG || mode == DMRG_PRECOND_OLSEN || mode == DMRG_PRECOND_SHIFT_INVERT,
                 ST_EINVAL, "mode must be DIAG, OLSEN or SHIFT_INVERT");
    int mv = s->s->correction_host_theta(k, mode, x, r, d, theta, t);
    if (products) *products = mv;
  });
}

dmrg_status dmrg_get_env(dmrg_solver* s, int cut, int side, double* host, int64_t cap, int64_t* size) {
  return solver_call(s, [&] {
    DMRG_REQUIRE(s && size && (host || cap == 0), ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(cut >= 0 && cut <= s->prob->p.n && (side == 0 || side == 1), ST_EINVAL, "bad cut/side");
    std::vector<double> v = s->s->env_host(cut, side);
    *size = (int64_t)v.size();
    std::memcpy(host, v.data(), std::min<int64_t>(cap, (int64_t)v.size()) * sizeof(double));
  });
}

dmrg_status dmrg_block_gemm(int precision, int mode, int M, int N, int K, const void* A, int lda,
                            const void* B, int ldb, void* C, int ldc, double coef, void* stream) {
  return guard([&] {
    DMRG_REQUIRE(A && B && C, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(M > 0 && N > 0 && K > 0, ST_EINVAL, "sizes must be positive");
    DMRG_REQUIRE(mode >= 0 && mode <= 2 && precision >= 0 && precision <= 2, ST_EINVAL, "bad mode/precision");
    DMRG_REQUIRE(!(precision == 2 && mode == 2), ST_EINVAL, "bf16 has no transposed-A mode");
    DMRG_REQUIRE(lda >= (mode == 2 ? M : K) && ldb >= (mode == 1 ? K : N) && ldc >= N, ST_EINVAL,
                 "leading dimension too small");
    hipStream_t st = (hipStream_t)stream;
    GemmItem it{A, B, lda, ldb, K, 0, coef};
    std::vector<GemmUnit> units;
    for (int m0 = 0; m0 < M; m0 += 64)
      for (int n0 = 0; n0 < N; n0 += 64) units.push_back({C, ldc, M, N, m0, n0, 0, 1, 0});
    DevMem di, du;
    di.reserve(sizeof(GemmItem));
    du.reserve(units.size() * sizeof(GemmUnit));
    hip_check(hipMemcpyAsync(di.p, &it, sizeof(GemmItem), hipMemcpyHostToDevice, st), "gemm item");
    hip_check(hipMemcpyAsync(du.p, units.data(), units.size() * sizeof(GemmUnit), hipMemcpyHostToDevice, st), "gemm units");
    launch_gemm(precision, mode, du.as<GemmUnit>(), (int)units.size(), di.as<GemmItem>(), st);
    hip_check(hipStreamSynchronize(st), "gemm");
  });
}

dmrg_status dmrg_workspace_query(const dmrg_solver* s, size_t* bytes) {
  return guard([&] {
    DMRG_REQUIRE(s && s->s && bytes, ST_EINVAL, "NULL argument");
    size_t est = s->s->workspace_estimate();
    if (const Arena* a = s->arena.get()) {
      size_t need = a->peak();
      if (a->failed_request()) need = std::max(a->size(), a->in_use() + a->failed_request());
      est = std::max(est, need + need / 4);
    }
    *bytes = est;
  });
}

dmrg_status dmrg_workspace_attach(dmrg_solver* s, void* dev_ptr, size_t bytes) {
  return guard([&] {
    DMRG_REQUIRE(s && s->s && dev_ptr, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(bytes >= (size_t(1) << 20), ST_EINVAL, "a workspace needs at least 1 MiB");
    auto arena = std::make_unique<Arena>(dev_ptr, bytes);
    SolverState state;
    {
      ArenaScope old_scope(s->arena.get());
      state = s->s->save_state();
    }
    Solver* fresh = nullptr;
    {
      ArenaScope scope(arena.get());
      fresh = new Solver(&s->prob->p, s->opt, s->stream);
      try {
        fresh->restore_state(state);
      } catch (...) {
        delete fresh;
        throw;
      }
    }
    {
      ArenaScope old_scope(s->arena.get());
      delete s->s;  // its buffers go back to the old workspace (or hipFree) before that one is dropped
    }
    s->s = fresh;
    s->arena = std::move(arena);
    s->allocs_at_attach = library_device_allocations();
  });
}

dmrg_status dmrg_set_kernel_tag(dmrg_solver* s, int tag) {
  return guard([&] {
    DMRG_REQUIRE(s && (tag == 0 || tag == 1), ST_EINVAL, "tag must be 0 or 1");
    s->s->set_kernel_tag(tag);
  });
}

dmrg_status dmrg_get_stats(const dmrg_solver* s, double* out, int n) {
  return guard([&] {
    DMRG_REQUIRE(s && out, ST_EINVAL, "NULL argument");
    const Stats& t = s->s->stats();
    double v[30] = {(double)t.matvecs, (double)t.davidson_iters, t.sigma_ms, t.env_ms, t.svd_ms,
                    t.sigma_flops, t.tau, (double)t.max_bond, (double)t.fallbacks, (double)t.converged,
                    t.sigma_a_ms, t.sigma_b_ms, t.sigma_a_flops, t.sigma_b_flops, t.env_flops,
                    (double)t.refinements, t.sigma_b_gemm_ms, t.grad_ms, t.grad_flops, t.prepare_ms,
                    t.resolve_ms, t.davidson_ms, (double)t.plan_hits, t.sigma_a_flops_exec,
                    t.sigma_b_flops_exec, (double)t.lowp_matvecs,
                    s->arena ? (double)s->arena->peak() : 0.0,
                    s->allocs_at_attach >= 0 ? (double)(library_device_allocations() - s->allocs_at_attach) : -1.0,
                    t.plan_build_ms, t.env_plan_ms};
    for (int i = 0; i < n && i < 30; ++i) out[i] = v[i];
  });
}

}  // extern "C"

dmrg_status dmrg_measure_peaks(void* stream, const void* src, void* dst, size_t bytes, double* fp64_tflops,
                               double* copy_gbs) {
  return guard([&] {
    DMRG_REQUIRE(src && dst && fp64_tflops && copy_gbs, ST_EINVAL, "NULL argument");
    DMRG_REQUIRE(bytes >= (size_t(1) << 22) && bytes % 16 == 0, ST_EINVAL,
                 "bytes must be a multiple of 16 and at least 4 MiB");
    DMRG_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, ST_EINVAL, "buffers must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    // best of three timed runs after one warm-up, for each ceiling
    const int n_blocks = 2048, iters = 2000;  // 8 waves per SIMD on 256 CUs; out = 4 MiB of dst
    double best_f = 0.0, best_c = 0.0;
    for (int rep = 0; rep < 4; ++rep) {
      float ms = 0.f;
      hip_check(hipEventRecord(e0, st), "event");
      const long flops = launch_mfma_f64_peak((double*)dst, n_blocks, iters, st);
      hip_check(hipEventRecord(e1, st), "event");
      hip_check(hipEventSynchronize(e1), "mfma peak");
      hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
      if (rep > 0 && ms > 0.f) best_f = std::max(best_f, flops / (ms * 1e-3) / 1e12);
    }
    for (int rep = 0; rep < 4; ++rep) {
      float ms = 0.f;
      hip_check(hipEventRecord(e0, st), "event");
      launch_stream_copy(src, dst, (long)bytes, st);
      hip_check(hipEventRecord(e1, st), "event");
      hip_check(hipEventSynchronize(e1), "stream copy");
      hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
      if (rep > 0 && ms > 0.f) best_c = std::max(best_c, 2.0 * (double)bytes / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *fp64_tflops = best_f;
    *copy_gbs = best_c;
  });
}
