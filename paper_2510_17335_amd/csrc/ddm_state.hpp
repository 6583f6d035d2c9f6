// Device views of the particle state and of its adjoint (structure of arrays,
// rows x[D], v[D], C[D*D], G[D*D] of stride ntot), shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddm_kernels.hpp"

namespace ddm {

// Position storage: 32-bit fixed point in FP32 (resolution 2^-32 of the unit
// domain, 60x finer than float near x = 0.5, and cell indices come out of
// integer arithmetic), plain double in FP64.
template <typename T> struct Pos;
template <> struct Pos<float> {
  using X = uint32_t;
  static __device__ __forceinline__ bool cell(X xr, const KCfg& c, int& base, float& f) {
    const uint64_t q = (uint64_t)xr << c.nlog2;          // x n in units of 2^-32
    if (q < 0x80000000ull) return false;
    const uint64_t s = q - 0x80000000ull;                // x n - 1/2
    const uint64_t b = s >> 32;
    if (b > (uint64_t)(c.n - 3)) return false;
    base = (int)b;
    f = 0.5f + (float)(uint32_t)(s & 0xFFFFFFFFull) * 2.3283064365386963e-10f;
    return true;
  }
  static __device__ __forceinline__ double real(X xr) { return (double)xr * 2.3283064365386963e-10; }
  static __device__ __forceinline__ X advance(X xr, float d, bool& ok) {
    const float q = rintf(d * 4294967296.0f);
    ok = fabsf(q) < 1073741824.0f;
    return ok ? xr + (uint32_t)(int32_t)q : xr;
  }
  static __device__ __forceinline__ X from_real(double x) {
    const double q = rint(x * 4294967296.0);
    return q <= 0.0 ? 0u : (q >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)q);
  }
  static __device__ __forceinline__ unsigned long long key(X xr) { return (unsigned long long)xr; }
  static __device__ __forceinline__ double unkey(unsigned long long k) { return (double)k * 2.3283064365386963e-10; }
};
template <> struct Pos<double> {
  using X = double;
  static __device__ __forceinline__ bool cell(X xr, const KCfg& c, int& base, double& f) {
    const double xs = xr * c.inv_dx;
    const double bf = floor(xs - 0.5);
    if (!(bf >= 0.0 && bf <= (double)(c.n - 3))) return false;
    base = (int)bf;
    f = xs - bf;
    return true;
  }
  static __device__ __forceinline__ double real(X xr) { return xr; }
  static __device__ __forceinline__ X advance(X xr, double d, bool& ok) { ok = true; return xr + d; }
  static __device__ __forceinline__ X from_real(double x) { return x; }
  static __device__ __forceinline__ unsigned long long key(X xr) { return (unsigned long long)__double_as_longlong(xr); }
  static __device__ __forceinline__ double unkey(unsigned long long k) { return __longlong_as_double((long long)k); }
};

template <typename T, int D> struct P {
  T* s;
  int64_t ntot;
  using X = typename Pos<T>::X;
  __device__ __forceinline__ X& xr(int a, int64_t p) const { return reinterpret_cast<X*>(s)[(int64_t)a * ntot + p]; }
  __device__ __forceinline__ T& v(int a, int64_t p) const { return s[(int64_t)(D + a) * ntot + p]; }
  __device__ __forceinline__ T& C(int a, int b, int64_t p) const { return s[(int64_t)(2 * D + a * D + b) * ntot + p]; }
  __device__ __forceinline__ T& G(int a, int b, int64_t p) const {
    return s[(int64_t)(2 * D + D * D + a * D + b) * ntot + p];
  }
};
// Adjoint states hold plain T in every row.
template <typename T, int D> struct Adj {
  T* s;
  int64_t ntot;
  __device__ __forceinline__ T& x(int a, int64_t p) const { return s[(int64_t)a * ntot + p]; }
  __device__ __forceinline__ T& v(int a, int64_t p) const { return s[(int64_t)(D + a) * ntot + p]; }
  __device__ __forceinline__ T& C(int a, int b, int64_t p) const { return s[(int64_t)(2 * D + a * D + b) * ntot + p]; }
  __device__ __forceinline__ T& G(int a, int b, int64_t p) const {
    return s[(int64_t)(2 * D + D * D + a * D + b) * ntot + p];
  }
};

template <typename T, int D>
__device__ __forceinline__ P<T, D> pv(const void* s, int64_t ntot) {
  return P<T, D>{const_cast<T*>(static_cast<const T*>(s)), ntot};
}
template <typename T, int D>
__device__ __forceinline__ Adj<T, D> av(const void* s, int64_t ntot) {
  return Adj<T, D>{const_cast<T*>(static_cast<const T*>(s)), ntot};
}

}  // namespace ddm
