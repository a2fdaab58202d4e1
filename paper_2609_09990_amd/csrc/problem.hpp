// The active-space problem: integrals, electron counts and the MPO built from them.
#pragma once

#include <vector>

#include "mpo.hpp"

namespace dmrg {

struct Problem {
  int n = 0, n_alpha = 0, n_beta = 0, nq = 0;
  double e_core = 0.0;
  std::vector<double> h, B;
  MPO mpo;
  QN target() const { return {n_alpha + n_beta, n_alpha - n_beta}; }
};

}  // namespace dmrg
