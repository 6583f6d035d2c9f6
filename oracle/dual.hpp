// Forward-mode dual numbers for the oracle (test infrastructure only).
//
// Dual<K> carries a value and K tangents; every operation applies the chain
// rule to each tangent.  Comparisons look at the value only, so branches of the
// method are taken on the primal value exactly as in a double run.  The real
// type R is double unless stated (long double: x87 extended precision, 64-bit
// significand).
#pragma once
#include <cmath>

namespace orc {

template <int K, class R = double>
struct Dual {
  R v;
  R d[K];
  Dual() : v(0.0) { for (int k = 0; k < K; ++k) d[k] = 0.0; }
  Dual(R x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0.0; }  // NOLINT: implicit on purpose
  static Dual var(R x, int k) { Dual r(x); r.d[k] = 1.0; return r; }

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
template <int K, class R> Dual<K, R> chain(const Dual<K, R>& a, R fv, R dfdx) {
  Dual<K, R> r; r.v = fv;
  for (int k = 0; k < K; ++k) r.d[k] = dfdx * a.d[k];
  return r;
}
template <int K, class R> Dual<K, R> sqrt(const Dual<K, R>& a) { R s = std::sqrt(a.v); return chain(a, s, R(0.5) / s); }
template <int K, class R> Dual<K, R> log(const Dual<K, R>& a) { return chain(a, R(std::log(a.v)), R(1) / a.v); }
template <int K, class R> Dual<K, R> exp(const Dual<K, R>& a) { R e = std::exp(a.v); return chain(a, e, e); }
template <int K, class R> Dual<K, R> sin(const Dual<K, R>& a) { return chain(a, R(std::sin(a.v)), R(std::cos(a.v))); }
template <int K, class R> Dual<K, R> cos(const Dual<K, R>& a) { return chain(a, R(std::cos(a.v)), R(-std::sin(a.v))); }
template <int K, class R> Dual<K, R> fabs(const Dual<K, R>& a) { return a.v < 0.0 ? -a : a; }

inline double val(double x) { return x; }
inline double val(long double x) { return (double)x; }
template <int K, class R> double val(const Dual<K, R>& x) { return (double)x.v; }

using std::sqrt; using std::log; using std::exp; using std::sin; using std::cos; using std::fabs;

}  // namespace orc
