// Forward-mode dual numbers for the oracle (test infrastructure only).
//
// Dual<K> carries a value and K tangents; every operation applies the chain
// rule to each tangent.  Comparisons look at the value only, so branches of the
// method are taken on the primal value exactly as in a double run.
#pragma once
#include <cmath>

namespace orc {

template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { for (int k = 0; k < K; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0.0; }  // NOLINT: implicit on purpose
  static Dual var(double x, int k) { Dual r(x); r.d[k] = 1.0; return r; }

  Dual& operator+=(const Dual& o) { v += o.v; for (int k = 0; k < K; ++k) d[k] += o.d[k]; return *this; }
  Dual& operator-=(const Dual& o) { v -= o.v; for (int k = 0; k < K; ++k) d[k] -= o.d[k]; return *this; }
  Dual& operator*=(const Dual& o) { *this = *this * o; return *this; }
  Dual& operator/=(const Dual& o) { *this = *this / o; return *this; }

  friend Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
  friend Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
  friend Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
  friend Dual operator*(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v * b.v;
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
  }
  friend Dual operator/(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v / b.v;
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
  }
  friend bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
  friend bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
  friend bool operator<=(const Dual& a, const Dual& b) { return a.v <= b.v; }
  friend bool operator>=(const Dual& a, const Dual& b) { return a.v >= b.v; }
};

// Elementary functions: value f(x), tangent f'(x) * dx.
template <int K> Dual<K> chain(const Dual<K>& a, double fv, double dfdx) {
  Dual<K> r; r.v = fv;
  for (int k = 0; k < K; ++k) r.d[k] = dfdx * a.d[k];
  return r;
}
template <int K> Dual<K> sqrt(const Dual<K>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int K> Dual<K> log(const Dual<K>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int K> Dual<K> exp(const Dual<K>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int K> Dual<K> sin(const Dual<K>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int K> Dual<K> cos(const Dual<K>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int K> Dual<K> fabs(const Dual<K>& a) { return a.v < 0.0 ? -a : a; }

inline double val(double x) { return x; }
template <int K> double val(const Dual<K>& x) { return x.v; }

using std::sqrt; using std::log; using std::exp; using std::sin; using std::cos; using std::fabs;

}  // namespace orc
