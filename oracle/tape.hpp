// Reverse-mode scalars for the oracle (test infrastructure only).
//
// An RV holds a value and, when it depends on the differentiated inputs, the
// index of its node on the thread's tape.  Every operation on variables
// appends one node with its parents and the local partial derivative with
// respect to each; constants (index -1) record nothing.  The adjoint sweep
// walks the tape from the last node to the first and adds each node's
// adjoint, times the partials, to its parents.  Comparisons look at the value
// only, so branches are taken as in a double run.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace orc {

struct Tape {
  std::vector<int64_t> first;   // node i's parents are [first[i], first[i + 1]) of par / dpar
  std::vector<int32_t> par;
  std::vector<double> dpar;
  std::vector<double> adj;
  Tape() { first.push_back(0); }
  int64_t size() const { return (int64_t)first.size() - 1; }
  int32_t add(int n, const int32_t* p, const double* d) {
    for (int k = 0; k < n; ++k) { par.push_back(p[k]); dpar.push_back(d[k]); }
    first.push_back((int64_t)par.size());
    return (int32_t)(first.size() - 2);
  }
  // Adjoint of node i into its parents.
  void back(int64_t i) {
    const double a = adj[(size_t)i];
    if (a == 0.0) return;
    for (int64_t k = first[(size_t)i]; k < first[(size_t)i + 1]; ++k) adj[(size_t)par[(size_t)k]] += a * dpar[(size_t)k];
  }
};

inline Tape*& active_tape() {
  static thread_local Tape* t = nullptr;
  return t;
}

struct RV {
  double v;
  int32_t i;
  RV() : v(0.0), i(-1) {}
  RV(double x) : v(x), i(-1) {}  // NOLINT: implicit on purpose
  // A new independent variable (an input of the differentiated function).
  static RV input(double x) {
    RV r(x);
    r.i = active_tape()->add(0, nullptr, nullptr);
    return r;
  }
  // A node of value x depending on up to n parents with partials d.
  static RV node(double x, int n, const RV* const* p, const double* d) {
    RV r(x);
    int32_t ip[16];
    double dp[16];
    int m = 0;
    for (int k = 0; k < n; ++k)
      if (p[k]->i >= 0) { ip[m] = p[k]->i; dp[m] = d[k]; ++m; }
    if (m) r.i = active_tape()->add(m, ip, dp);
    return r;
  }
  static RV unary(double x, const RV& a, double da) {
    const RV* p[1] = {&a};
    return node(x, 1, p, &da);
  }
  static RV binary(double x, const RV& a, double da, const RV& b, double db) {
    const RV* p[2] = {&a, &b};
    const double d[2] = {da, db};
    return node(x, 2, p, d);
  }

  RV& operator+=(const RV& o) { *this = *this + o; return *this; }
  RV& operator-=(const RV& o) { *this = *this - o; return *this; }
  RV& operator*=(const RV& o) { *this = *this * o; return *this; }
  RV& operator/=(const RV& o) { *this = *this / o; return *this; }

  friend RV operator+(const RV& a, const RV& b) { return binary(a.v + b.v, a, 1.0, b, 1.0); }
  friend RV operator-(const RV& a, const RV& b) { return binary(a.v - b.v, a, 1.0, b, -1.0); }
  friend RV operator-(const RV& a) { return unary(-a.v, a, -1.0); }
  friend RV operator*(const RV& a, const RV& b) { return binary(a.v * b.v, a, b.v, b, a.v); }
  friend RV operator/(const RV& a, const RV& b) {
    const double q = a.v / b.v;
    return binary(q, a, 1.0 / b.v, b, -q / b.v);
  }
  friend bool operator<(const RV& a, const RV& b) { return a.v < b.v; }
  friend bool operator>(const RV& a, const RV& b) { return a.v > b.v; }
  friend bool operator<=(const RV& a, const RV& b) { return a.v <= b.v; }
  friend bool operator>=(const RV& a, const RV& b) { return a.v >= b.v; }
};

inline RV sqrt(const RV& a) { const double s = std::sqrt(a.v); return RV::unary(s, a, 0.5 / s); }
inline RV log(const RV& a) { return RV::unary(std::log(a.v), a, 1.0 / a.v); }
inline RV exp(const RV& a) { const double e = std::exp(a.v); return RV::unary(e, a, e); }
inline RV sin(const RV& a) { return RV::unary(std::sin(a.v), a, std::cos(a.v)); }
inline RV cos(const RV& a) { return RV::unary(std::cos(a.v), a, -std::sin(a.v)); }
inline RV fabs(const RV& a) { return a.v < 0.0 ? -a : a; }
inline double val(const RV& x) { return x.v; }

}  // namespace orc
