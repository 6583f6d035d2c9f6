// Device math of the MLS-MPM sub-step for gfx950: small fixed-size matrix
// helpers, the SVD of F, the Drucker-Prager return map with its adjoint, the
// isotropic-function adjoint that carries gradients through the SVD, and the
// shovel contact with its adjoint.  Everything lives in registers; T is float
// or double, D is 2 or 3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddm {

template <typename T> struct Lim;
template <> struct Lim<float> {
  static constexpr int sweeps = 6;
  static __device__ __forceinline__ float tol() { return 1e-6f; }
};
template <> struct Lim<double> {
  static constexpr int sweeps = 12;
  static __device__ __forceinline__ double tol() { return 1e-16; }
};

template <typename T> __device__ __forceinline__ T dsqrt(T x) { return sqrt(x); }
// Square root of an argument that is never subnormal (at least 1e-12): the
// hardware v_sqrt_f32 (about 1 ulp, no rescaling or rounding fix-up) in
// float, the library routine in double.
template <typename T> __device__ __forceinline__ T fsqrt(T x) { return sqrt(x); }
template <> __device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// a[i] for a run-time i in {0, 1, 2} by selects, so that a loop counter used
// as the index does not move a register array to scratch memory.
template <typename T> __device__ __forceinline__ T sel3(const T (&a)[3], int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}
template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }

// Reciprocal and reciprocal square root: the hardware approximations
// (v_rcp_f32, v_rsq_f32, about 1 ulp) in float, exact division in double.
template <typename T> __device__ __forceinline__ T frcp(T x);
template <> __device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ T frsq(T x);
template <> __device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }

// log(1 + x) and exp(x) - 1 for small x.  In float: the hardware base-2
// logarithm and exponential (v_log_f32, v_exp_f32) with the classical
// corrections that cancel the rounding of 1 + x and of exp(x):
//   log1p(x) = log(u) x / (u - 1), u = 1 + x (u == 1: x)   (Goldberg 1991, Thm. 4)
//   expm1(x) = (u - 1) x / log(u), u = exp(x) (u == 1: x)  (Kahan; Higham 2002, 1.14.1)
// A few ulp (the GPU accuracy test bounds them), about a quarter of the
// instructions of the library routines.
// In double: the library routines.
template <typename T> __device__ __forceinline__ T flog1p(T x) { return log1p(x); }
template <> __device__ __forceinline__ float flog1p(float x) {
  const float u = 1.0f + x;
  if (u == 1.0f) return x;
  if (!(u < __builtin_inff())) return u;     // +inf and NaN as they come
  return __builtin_amdgcn_logf(u) * 0.693147180559945f * (x * __builtin_amdgcn_rcpf(u - 1.0f));
}
template <typename T> __device__ __forceinline__ T fexpm1(T x) { return expm1(x); }
template <> __device__ __forceinline__ float fexpm1(float x) {
  // x log2(e) as t + e exactly enough (two-part constant, FMA for the
  // product's rounding), so that exp(x) = 2^t (1 + e ln 2) keeps about an ulp
  // for large |x| as well; the correction below then handles small x.
  // Beyond the range of the float result: +inf and -1 (NaN passes through).
  if (x > 88.8f) return __builtin_inff();
  if (x < -104.0f) return -1.0f;
  const float t = x * 1.44269502162933350f;
  const float e = __builtin_fmaf(x, 1.44269502162933350f, -t) + x * 1.92596303350001e-8f;
  float u = __builtin_amdgcn_exp2f(t);
  u = __builtin_fmaf(u, e * 0.693147180559945f, u);
  if (u == 1.0f) return x;
  if (!(u < __builtin_inff())) return u;     // overflow (and NaN) as they come
  const float um1 = u - 1.0f;
  if (um1 == -1.0f) return -1.0f;
  return um1 * x * __builtin_amdgcn_rcpf(__builtin_amdgcn_logf(u) * 0.693147180559945f);
}

// Sigma below this is clamped before the logarithm (ln S must exist).
template <typename T> __device__ __forceinline__ T sigma_min() { return T(1e-6); }

// ---------------------------------------------------------------------------
// Eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations
// (stopped when the off-diagonal part is below tol relative to the diagonal),
// eigenvalues left on the diagonal of a and sorted in decreasing order, each
// column swap of V paired with a sign flip so that det V stays +1.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void jacobi_sym(T a[3][3], T V[3][3], T ev[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = T(i == j ? 1 : 0);
  for (int sweep = 0; sweep < Lim<T>::sweeps; ++sweep) {
    T off = T(0), dia = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      dia += a[i][i] * a[i][i];
#pragma unroll
      for (int j = i + 1; j < D; ++j) off += a[i][j] * a[i][j];
    }
    if (!(off > Lim<T>::tol() * Lim<T>::tol() * dia)) break;
#pragma unroll
    for (int pq = 0; pq < (D == 3 ? 3 : 1); ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const T apq = a[p][q];
      // a zero a_pq gives t = 0, the identity rotation (selected rather than
      // branched over: no merge of register copies in the unrolled sweeps)
      const T theta = (a[q][q] - a[p][p]) * frcp(T(2) * apq);
      const T tr = (theta >= T(0) ? T(1) : T(-1)) * frcp(dabs(theta) + fsqrt(theta * theta + T(1)));
      const T t = apq == T(0) ? T(0) : tr;
      const T c = frsq(t * t + T(1));
      const T sn = t * c;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = T(0);
      if (D == 3) {
        const int r = 3 - p - q;
        const T arp = a[r][p], arq = a[r][q];
        a[r][p] = a[p][r] = c * arp - sn * arq;
        a[r][q] = a[q][r] = sn * arp + c * arq;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const T vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - sn * vq;
        V[k][q] = sn * vp + c * vq;
      }
    }
  }
  ev[0] = a[0][0];
  ev[1] = a[1][1];
  ev[2] = D == 3 ? a[2][2] : T(0);
  auto swap_cols = [&](int i, int j) {
    const T t = ev[i]; ev[i] = ev[j]; ev[j] = t;
#pragma unroll
    for (int k = 0; k < D; ++k) { const T u = V[k][i]; V[k][i] = V[k][j]; V[k][j] = -u; }
  };
  if (ev[0] < ev[1]) swap_cols(0, 1);
  if (D == 3) {
    if (ev[0] < ev[2]) swap_cols(0, 2);
    if (ev[1] < ev[2]) swap_cols(1, 2);
  }
}

// ---------------------------------------------------------------------------
// Drucker-Prager return map on eps = ln s (Eq. DP), forward.
// Cases: 1 tension (tr eps > 0, or beyond the shifted apex with cohesion):
// eps' = apex; 2 inside the cone: eps' = eps; 3 projection onto the cone:
// eps' = (tr/D) 1 - beta n, n = dev(eps)/|dev(eps)|,
// beta = (alpha (D lam + 2 mu) tr - k_c) / (2 mu).
// Outputs g = exp(eps') (plastic singular values) and the principal Kirchhoff
// stresses h = 2 mu eps' + lam tr(eps').
// ---------------------------------------------------------------------------
template <typename T> struct DP {
  T eps[3], ep[3], g[3], h[3];
  T tr, nrm, beta, apex, stiff;
  int cs;
};

template <typename T, int D>
__device__ __forceinline__ void dp_forward(const T eps[3], T mu, T lam, T alpha, T kc, DP<T>& o) {
  o.tr = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) { o.eps[i] = eps[i]; o.tr += o.eps[i]; }
  T n2 = T(0), dev[3];
  const T mean = o.tr * T(1.0 / D);
#pragma unroll
  for (int i = 0; i < D; ++i) { dev[i] = o.eps[i] - mean; n2 += dev[i] * dev[i]; }
  o.nrm = n2 > T(0) ? dsqrt(n2) : T(0);
  o.stiff = T(D) * lam + T(2) * mu;
  o.beta = T(0);
  o.apex = T(0);
  const bool tension = (kc == T(0)) ? (o.tr > T(0)) : (alpha * o.stiff * o.tr > kc);
  if (tension) {
    o.cs = 1;
    o.apex = kc * frcp(T(D) * alpha * o.stiff);
#pragma unroll
    for (int i = 0; i < D; ++i) o.ep[i] = o.apex;
  } else {
    o.beta = (alpha * o.stiff * o.tr - kc) * frcp(T(2) * mu);
    const T dgam = o.nrm + o.beta;
    if (!(dgam > T(0))) {
      o.cs = 2;
#pragma unroll
      for (int i = 0; i < D; ++i) o.ep[i] = o.eps[i];
    } else {
      o.cs = 3;
      const T f = dgam * frcp(o.nrm);
#pragma unroll
      for (int i = 0; i < D; ++i) o.ep[i] = o.eps[i] - f * dev[i];
    }
  }
  T tre = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) tre += o.ep[i];
#pragma unroll
  for (int i = 0; i < D; ++i) { o.g[i] = exp(o.ep[i]); o.h[i] = T(2) * mu * o.ep[i] + lam * tre; }
#pragma unroll
  for (int i = D; i < 3; ++i) { o.g[i] = T(1); o.h[i] = T(0); o.eps[i] = o.ep[i] = T(0); }
}

// Adjoint of dp_forward: (gbar, hbar) -> sbar and material adjoints.
template <typename T, int D>
__device__ __forceinline__ void dp_backward(const DP<T>& o, const T s[3], T mu, T lam, T alpha, T kc,
                                            const T gbar[3], const T hbar[3], T sbar[3], T& mub, T& lamb,
                                            T& alb, T& kcb) {
  T hsum = T(0), tre = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) { hsum += hbar[i]; tre += o.ep[i]; }
  T epb[3];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    epb[i] = gbar[i] * o.g[i] + T(2) * mu * hbar[i] + lam * hsum;
    mub += T(2) * hbar[i] * o.ep[i];
  }
  lamb += hsum * tre;
  T eb[3] = {T(0), T(0), T(0)};
  if (o.cs == 2) {
#pragma unroll
    for (int i = 0; i < D; ++i) eb[i] = epb[i];
  } else if (o.cs == 1) {
    if (kc != T(0)) {
      T ab = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) ab += epb[i];
      // apex = kc / (D alpha stiff)
      kcb += ab * frcp(T(D) * alpha * o.stiff);
      alb -= ab * o.apex * frcp(alpha);
      const T sb = -ab * o.apex * frcp(o.stiff);
      lamb += T(D) * sb;
      mub += T(2) * sb;
    }
  } else {
    // eps' = (tr/D) 1 - beta n
    T nvec[3], trb = T(0), betab = T(0);
    const T inrm = frcp(o.nrm), mean = o.tr * T(1.0 / D);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      nvec[i] = (o.eps[i] - mean) * inrm;
      trb += epb[i] * T(1.0 / D);
      betab -= epb[i] * nvec[i];
    }
    T nb[3], nbn = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) { nb[i] = -o.beta * epb[i]; nbn += nb[i] * nvec[i]; }
    // beta = (alpha stiff tr - kc) / (2 mu)
    const T inv2mu = frcp(T(2) * mu);
    trb += betab * alpha * o.stiff * inv2mu;
    alb += betab * o.stiff * o.tr * inv2mu;
    kcb -= betab * inv2mu;
    const T sb = betab * alpha * o.tr * inv2mu;
    mub += T(2) * (sb - betab * o.beta * inv2mu);
    lamb += T(D) * sb;
    // n = dev / |dev|, dev = eps - tr/D
    T devb[3], devbs = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) { devb[i] = (nb[i] - nbn * nvec[i]) * inrm; devbs += devb[i]; }
#pragma unroll
    for (int i = 0; i < D; ++i) eb[i] = devb[i] - devbs * T(1.0 / D) + trb;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) sbar[i] = eb[i] * frcp(s[i]);
}

// Divided differences of g and h across a pair of singular values, without
// cancellation: eps'_i - eps'_j = k (eps_i - eps_j) with k = 1 (case 2),
// 0 (case 1) or -beta/|dev| (case 3), and eps_i - eps_j = log1p((s_i-s_j)/s_j);
// ds = s_i - s_j is passed in, computed from s - 1 without cancellation.
template <typename T>
__device__ __forceinline__ void divided(const DP<T>& o, T mu, T ds, T sj, T gj, T& ddg, T& ddh, T& y) {
  const T k = o.cs == 2 ? T(1) : (o.cs == 1 ? T(0) : -o.beta * frcp(o.nrm));
  const T isj = frcp(sj);
  const T de = flog1p(ds * isj);
  const T dl = ds != T(0) ? de * frcp(ds) : isj;        // (eps_i - eps_j) / (s_i - s_j)
  y = k * de;                                            // eps'_i - eps'_j
  const T em1 = y != T(0) ? fexpm1(y) * frcp(y) : T(1);
  ddg = gj * em1 * k * dl;
  ddh = T(2) * mu * k * dl;
}

// ---------------------------------------------------------------------------
// Constitutive update of one particle, on the displacement gradient G = F - I
// (kept instead of F so that small strains keep their relative precision).
// F = U diag(s) V^T = R S (polar): V and s^2 - 1 from the eigen-decomposition
// of F^T F - I = G + G^T + G^T G, eps = ln s = log1p(s^2 - 1)/2,
// R - I = (G - (S - I)) S^-1, U = R V.  Outputs, without cancellation:
//   G' = F' - I = (S' - I) + (R - I) + (R - I)(S' - I), S' - I = V diag(expm1(eps')) V^T
//   tau = U diag(h) U^T.
// ---------------------------------------------------------------------------
template <typename T, int D> struct Constit {
  T U[3][3], V[3][3], s[3], sm1[3], eps[3], RmI[3][3];
  bool clamped[3];
  int nclamp;
  DP<T> dp;
};

template <typename T, int D>
__device__ __forceinline__ void constit_forward(const T G[3][3], T mu, T lam, T alpha, T kc, Constit<T, D>& c) {
  T a[3][3];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = G[i][j] + G[j][i];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += G[k][i] * G[k][j];
      a[i][j] = acc;
    }
  T ev[3];
  jacobi_sym<T, D>(a, c.V, ev);
  // det F <= 0 (an inverted particle) has no logarithmic strain: flagged as a clamp.
  T detF;
  if (D == 2) {
    detF = (T(1) + G[0][0]) * (T(1) + G[1][1]) - G[0][1] * G[1][0];
  } else {
    const T f00 = T(1) + G[0][0], f11 = T(1) + G[1][1], f22 = T(1) + G[2][2];
    detF = f00 * (f11 * f22 - G[1][2] * G[2][1]) - G[0][1] * (G[1][0] * f22 - G[1][2] * G[2][0]) +
           G[0][2] * (G[1][0] * G[2][1] - f11 * G[2][0]);
  }
  c.nclamp = detF > T(0) ? 0 : 1;
  const T smin = sigma_min<T>();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c.clamped[i] = false;
    if (i >= D) { c.s[i] = T(1); c.sm1[i] = T(0); c.eps[i] = T(0); continue; }
    const T l = ev[i];                       // s^2 - 1
    if (!(T(1) + l > smin * smin)) {
      c.s[i] = smin; c.sm1[i] = smin - T(1); c.eps[i] = log(smin);
      c.clamped[i] = true; ++c.nclamp;
    } else {
      c.s[i] = fsqrt(T(1) + l);
      c.sm1[i] = l * frcp(T(1) + c.s[i]);
      c.eps[i] = T(0.5) * flog1p(l);
    }
  }
  // R - I = (G - (S - I)) S^-1; S - I = V diag(s - 1) V^T and S^-1 are
  // symmetric, so each entry pair is formed once
  T GmS[3][3], Sinv[3][3], is[3];
#pragma unroll
  for (int k = 0; k < D; ++k) is[k] = frcp(c.s[k]);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T smi = T(0), si = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const T vv = c.V[i][k] * c.V[j][k];
        smi += vv * c.sm1[k];
        si += vv * is[k];
      }
      GmS[i][j] = G[i][j] - smi;
      GmS[j][i] = G[j][i] - smi;
      Sinv[i][j] = Sinv[j][i] = si;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) acc += GmS[i][k] * Sinv[k][j];
      c.RmI[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = c.V[i][j];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += c.RmI[i][k] * c.V[k][j];
      c.U[i][j] = acc;
    }
  dp_forward<T, D>(c.eps, mu, lam, alpha, kc, c.dp);
}

template <typename T, int D>
__device__ __forceinline__ void constit_outputs(const Constit<T, D>& c, T Gn[3][3], T tau[3][3]) {
  T em[3], SpmI[3][3];
#pragma unroll
  for (int k = 0; k < D; ++k) em[k] = fexpm1(c.dp.ep[k]);
  // both are symmetric: the upper triangle is computed and mirrored
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T a = T(0), b = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        a += c.V[i][k] * em[k] * c.V[j][k];
        b += c.U[i][k] * c.dp.h[k] * c.U[j][k];
      }
      SpmI[i][j] = SpmI[j][i] = a;
      tau[i][j] = tau[j][i] = b;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = SpmI[i][j] + c.RmI[i][j];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += c.RmI[i][k] * SpmI[k][j];
      Gn[i][j] = acc;
    }
}

// The forward constitutive update alone (P2G), without the polar factors.
// Since eps' and eps share the eigenvectors V of F^T F,
//   F' = U diag(s') V^T = F V diag(exp(eps' - eps)) V^T,
// so G' = G + M + G M with M = V diag(expm1(d)) V^T, d = eps' - eps taken per
// case without cancellation (0 inside the cone, apex - eps in tension,
// -(dgam/|dev|) dev on projection): an elastic step leaves G' = G exactly.
// With U = F' V diag(1/s'), tau = U diag(h) U^T = F' N F'^T, N = V diag(h / s'^2) V^T,
// s'^2 = (1 + lambda'_i)(1 + expm1(d_i))^2.  The result equals
// constit_forward + constit_outputs up to rounding (clamped singular values
// aside, which are flagged).  Returns the number of clamps.
template <typename T, int D>
__device__ __forceinline__ int constit_step(const T G[3][3], T mu, T lam, T alpha, T kc, T Gn[3][3], T tau[3][3]) {
  T a[3][3], V[3][3], ev[3];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = G[i][j] + G[j][i];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += G[k][i] * G[k][j];
      a[i][j] = acc;
    }
  jacobi_sym<T, D>(a, V, ev);
  T detF;
  if (D == 2) {
    detF = (T(1) + G[0][0]) * (T(1) + G[1][1]) - G[0][1] * G[1][0];
  } else {
    const T f00 = T(1) + G[0][0], f11 = T(1) + G[1][1], f22 = T(1) + G[2][2];
    detF = f00 * (f11 * f22 - G[1][2] * G[2][1]) - G[0][1] * (G[1][0] * f22 - G[1][2] * G[2][0]) +
           G[0][2] * (G[1][0] * G[2][1] - f11 * G[2][0]);
  }
  int nclamp = detF > T(0) ? 0 : 1;
  const T smin = sigma_min<T>();
  T eps[3], s2[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= D) { eps[i] = T(0); s2[i] = T(1); continue; }
    const T l = ev[i];                       // s^2 - 1
    if (!(T(1) + l > smin * smin)) {
      eps[i] = log(smin); s2[i] = smin * smin; ++nclamp;
    } else {
      eps[i] = T(0.5) * flog1p(l); s2[i] = T(1) + l;
    }
  }
  DP<T> dp;
  dp_forward<T, D>(eps, mu, lam, alpha, kc, dp);
  T e[3] = {T(0), T(0), T(0)}, cn[3] = {T(0), T(0), T(0)};
  const T mean = dp.tr * T(1.0 / D);
  const T f = dp.cs == 3 ? (dp.nrm + dp.beta) * frcp(dp.nrm) : T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T d = dp.cs == 2 ? T(0) : (dp.cs == 1 ? dp.apex - eps[i] : -f * (eps[i] - mean));
    e[i] = fexpm1(d);
    const T g = T(1) + e[i];
    cn[i] = dp.h[i] * frcp(s2[i] * g * g);
  }
  // M and N share the products V_ik V_jk; both are symmetric
  T M[3][3], N[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { M[i][j] = T(0); N[i][j] = T(0); }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T m = T(0), n = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const T vv = V[i][k] * V[j][k];
        m += vv * e[k];
        n += vv * cn[k];
      }
      M[i][j] = M[j][i] = m;
      N[i][j] = N[j][i] = n;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = G[i][j] + M[i][j];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += G[i][k] * M[k][j];
      Gn[i][j] = acc;
    }
  // tau = F' N F'^T with F' = I + G': P = N + G' N, tau = P + P G'^T
  T P[3][3];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = N[i][j];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += Gn[i][k] * N[k][j];
      P[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T acc = P[i][j];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += P[i][k] * Gn[j][k];
      tau[i][j] = tau[j][i] = acc;
    }
  return nclamp;
}

// Adjoint of (F_tmp -> F', tau) for adjoints Fnb (of F', equally of G') and
// taub (of tau); the result is the adjoint of F_tmp (equally of G_tmp).
// In the SVD frame, with sym/skw the symmetric/skew parts of dF~ = U^T dF V,
// dG~_ij = ddg sym + cg skw, dG~_ji = ddg sym - cg skw, dT~_ij = dT~_ji =
// ddh sym + ch skw; the diagonal goes through s and the return map.
template <typename T, int D>
__device__ __forceinline__ void constit_backward(const Constit<T, D>& c, T mu, T lam, T alpha, T kc,
                                                 const T Fnb[3][3], const T taub[3][3], T Ftb[3][3], T& mub,
                                                 T& lamb, T& alb, T& kcb) {
  // Gb = U^T Fnb V and Tb = U^T taub U as two-step products.
  T Gb[3][3], Tb[3][3];
  {
    T UtF[3][3], UtT[3][3];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        T a = T(0), b = T(0);
#pragma unroll
        for (int p = 0; p < D; ++p) { a += c.U[p][i] * Fnb[p][q]; b += c.U[p][i] * taub[p][q]; }
        UtF[i][q] = a;
        UtT[i][q] = b;
      }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T a = T(0), b = T(0);
#pragma unroll
        for (int q = 0; q < D; ++q) { a += UtF[i][q] * c.V[q][j]; b += UtT[i][q] * c.U[q][j]; }
        Gb[i][j] = a;
        Tb[i][j] = b;
      }
  }
  T gb[3], hb[3], sb[3];
#pragma unroll
  for (int i = 0; i < D; ++i) { gb[i] = Gb[i][i]; hb[i] = Tb[i][i]; }
  dp_backward<T, D>(c.dp, c.s, mu, lam, alpha, kc, gb, hb, sb, mub, lamb, alb, kcb);
  T Fb[3][3];
#pragma unroll
  for (int i = 0; i < D; ++i) Fb[i][i] = c.clamped[i] ? T(0) : sb[i];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i + 1; j < D; ++j) {
      T ddg, ddh, y;
      divided<T>(c.dp, mu, c.sm1[i] - c.sm1[j], c.s[j], c.dp.g[j], ddg, ddh, y);
      const T isum = frcp(c.s[i] + c.s[j]);
      const T cg = (c.dp.g[i] + c.dp.g[j]) * isum;
      const T ch = -T(2) * mu * y * isum;
      const T tsym = Tb[i][j] + Tb[j][i];
      const T symb = ddg * (Gb[i][j] + Gb[j][i]) + ddh * tsym;
      const T skwb = cg * (Gb[i][j] - Gb[j][i]) + ch * tsym;
      Fb[i][j] = T(0.5) * (symb + skwb);
      Fb[j][i] = T(0.5) * (symb - skwb);
    }
  // Ftb = U Fb V^T
  T UF[3][3];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T a = T(0);
#pragma unroll
      for (int p = 0; p < D; ++p) a += c.U[i][p] * Fb[p][q];
      UF[i][q] = a;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < D; ++q) a += UF[i][q] * c.V[j][q];
      Ftb[i][j] = a;
    }
}

// ---------------------------------------------------------------------------
// Shovel: oriented box about the tip.  Axes e_w = z, e_n = (cos psi, -sin psi, 0),
// e_p = (-sin psi, -cos psi, 0) (pointing); centre = tip - half_p e_p.
// ---------------------------------------------------------------------------
template <typename T> struct Blade {
  T tip[3], psi, vel[3], omega;   // pose and velocity of the sub-step
  T sp, cp;                       // sin/cos psi
};

template <typename T> struct SDF {
  T loc[3], q[3], o[3], od;  // local coordinates, q = |loc| - half, outside offsets
  T n[3];                     // world normal
  T phi;
  int inside_axis;            // -1 when outside
};

template <typename T>
__device__ __forceinline__ void blade_axes(const Blade<T>& b, T e[3][3]) {
  e[0][0] = T(0); e[0][1] = T(0); e[0][2] = T(1);
  e[1][0] = b.cp; e[1][1] = -b.sp; e[1][2] = T(0);
  e[2][0] = -b.sp; e[2][1] = -b.cp; e[2][2] = T(0);
}

template <typename T>
__device__ __forceinline__ void sdf_eval(const Blade<T>& b, const T half[3], const T x[3], SDF<T>& f) {
  T e[3][3];
  blade_axes(b, e);
  T d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = x[k] - b.tip[k] + half[2] * e[2][k];
  bool outside = false;
  T o2 = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f.loc[a] = d[0] * e[a][0] + d[1] * e[a][1] + d[2] * e[a][2];
    f.q[a] = dabs(f.loc[a]) - half[a];
    const T sg = f.loc[a] >= T(0) ? T(1) : T(-1);
    f.o[a] = f.q[a] > T(0) ? sg * f.q[a] : T(0);
    if (f.q[a] > T(0)) { outside = true; o2 += f.q[a] * f.q[a]; }
  }
  T nl[3];
  if (outside) {
    f.od = dsqrt(o2);
    f.phi = f.od;
    f.inside_axis = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) nl[a] = f.o[a] / f.od;
  } else {
    int am = 0;
    if (f.q[1] > f.q[0]) am = 1;
    if (f.q[2] > sel3(f.q, am)) am = 2;
    f.phi = sel3(f.q, am);
    f.od = T(0);
    f.inside_axis = am;
    const T sg = sel3(f.loc, am) >= T(0) ? T(1) : T(-1);
#pragma unroll
    for (int a = 0; a < 3; ++a) nl[a] = a == am ? sg : T(0);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) f.n[k] = nl[0] * e[0][k] + nl[1] * e[1][k] + nl[2] * e[2][k];
}

// Adjoint of the normal with respect to the blade pose (tip, psi).
template <typename T>
__device__ __forceinline__ void sdf_normal_backward(const Blade<T>& b, const T half[3], const T x[3],
                                                    const SDF<T>& f, const T nb[3], T tipb[3], T& psib) {
  T e[3][3];
  blade_axes(b, e);
  T eb[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
  if (f.inside_axis >= 0) {
    const int am = f.inside_axis;
    const T sg = sel3(f.loc, am) >= T(0) ? T(1) : T(-1);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) eb[a][k] += a == am ? sg * nb[k] : T(0);
  } else {
    T nl[3], nlb[3], dotb = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      nl[a] = f.o[a] / f.od;
      nlb[a] = nb[0] * e[a][0] + nb[1] * e[a][1] + nb[2] * e[a][2];
#pragma unroll
      for (int k = 0; k < 3; ++k) eb[a][k] += nl[a] * nb[k];
      dotb += nlb[a] * nl[a];
    }
    T d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = x[k] - b.tip[k] + half[2] * e[2][k];
    T db[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!(f.q[a] > T(0))) continue;
      const T locb = (nlb[a] - dotb * nl[a]) / f.od;     // d o_a / d loc_a = 1 when outside
#pragma unroll
      for (int k = 0; k < 3; ++k) { db[k] += locb * e[a][k]; eb[a][k] += locb * d[k]; }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { tipb[k] -= db[k]; eb[2][k] += half[2] * db[k]; }
  }
  // de_n/dpsi = e_p, de_p/dpsi = -e_n, e_w constant.
  psib += eb[1][0] * e[2][0] + eb[1][1] * e[2][1] - eb[2][0] * e[1][0] - eb[2][1] * e[1][1];
}

// Coulomb contact (forward): returns the case (0 none/separating, 1 stick, 2 slip).
template <typename T>
__device__ __forceinline__ int coulomb_forward(const T vs[3], const T n[3], T mu_b, T v[3]) {
  T vr[3], vn = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) { vr[k] = v[k] - vs[k]; vn += vr[k] * n[k]; }
  if (vn >= T(0)) return 0;
  T vt[3], t2 = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) { vt[k] = vr[k] - vn * n[k]; t2 += vt[k] * vt[k]; }
  const T tn = dsqrt(t2);
  if (tn <= -mu_b * vn) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = vs[k];
    return 1;
  }
  const T sc = T(1) + mu_b * vn / tn;
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = vs[k] + sc * vt[k];
  return 2;
}

// Coulomb contact (adjoint): given the input velocity u and vb (adjoint of
// the output), returns ub and the adjoints of vs and n.
template <typename T>
__device__ __forceinline__ void coulomb_backward(const T vs[3], const T n[3], T mu_b, const T u[3], const T vb[3],
                                                 T ub[3], T vsb[3], T nb[3]) {
  T vr[3], vn = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) { vr[k] = u[k] - vs[k]; vn += vr[k] * n[k]; nb[k] = T(0); }
  if (vn >= T(0)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { ub[k] = vb[k]; vsb[k] = T(0); }
    return;
  }
  T vt[3], t2 = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) { vt[k] = vr[k] - vn * n[k]; t2 += vt[k] * vt[k]; }
  const T tn = dsqrt(t2);
  if (tn <= -mu_b * vn) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { ub[k] = T(0); vsb[k] = vb[k]; }
    return;
  }
  const T sc = T(1) + mu_b * vn / tn;
  T scb = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) scb += vb[k] * vt[k];
  T vtb[3];
  const T vnb0 = scb * mu_b / tn;
  const T tnb = -scb * mu_b * vn / (tn * tn);
#pragma unroll
  for (int k = 0; k < 3; ++k) vtb[k] = sc * vb[k] + tnb * vt[k] / tn;
  // vt = vr - vn n
  T vrb[3], vnb = vnb0;
#pragma unroll
  for (int k = 0; k < 3; ++k) { vrb[k] = vtb[k]; vnb -= vtb[k] * n[k]; nb[k] -= vn * vtb[k]; }
  // vn = vr . n
#pragma unroll
  for (int k = 0; k < 3; ++k) { vrb[k] += vnb * n[k]; nb[k] += vnb * vr[k]; }
#pragma unroll
  for (int k = 0; k < 3; ++k) { ub[k] = vrb[k]; vsb[k] = vb[k] - vrb[k]; }
}

// ---------------------------------------------------------------------------
// Quadratic B-spline stencil along one axis: base = floor(x/dx - 1/2),
// f = x/dx - base in [1/2, 3/2), weights and their derivatives in f.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void bspline(T f, T w[3], T dw[3]) {
  const T a = T(1.5) - f, b = f - T(1), c = f - T(0.5);
  w[0] = T(0.5) * a * a;
  w[1] = T(0.75) - b * b;
  w[2] = T(0.5) * c * c;
  dw[0] = -a;
  dw[1] = T(-2) * b;
  dw[2] = c;
}

}  // namespace ddm
