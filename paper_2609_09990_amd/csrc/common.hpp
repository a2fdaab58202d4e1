// Shared host-side definitions: quantum numbers, status handling, small helpers.
#pragma once

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace dmrg {

// Sector label of a bond or site state: particle number and twice S_z.
struct QN {
  int n = 0;
  int sz = 0;
  bool operator==(const QN& o) const { return n == o.n && sz == o.sz; }
  bool operator!=(const QN& o) const { return !(*this == o); }
  bool operator<(const QN& o) const { return n != o.n ? n < o.n : sz < o.sz; }
  QN operator+(const QN& o) const { return {n + o.n, sz + o.sz}; }
  QN operator-(const QN& o) const { return {n - o.n, sz - o.sz}; }
  QN operator-() const { return {-n, -sz}; }
};

// Site states |0>, |alpha>, |beta>, |alpha beta>: index s = n_alpha + 2 n_beta.
inline QN site_qn(int s) {
  static const QN q[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};
  return q[s];
}

// Library error carrying a status code (converted to a return code at the C ABI).
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum StatusCode {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_ENOMEM = -2,
  ST_EHIP = -3,
  ST_ENOCONV = -4,
  ST_ESECTOR = -5,
  ST_ESTATE = -6,
};

#define DMRG_REQUIRE(cond, code, msg)                                   \
  do {                                                                  \
    if (!(cond)) throw ::dmrg::Error((code), std::string(msg));         \
  } while (0)

}  // namespace dmrg
