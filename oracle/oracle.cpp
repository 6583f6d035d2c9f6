// ============================================================================
//  ORACLE — test infrastructure only.
//
//  A plain, single-threaded FP64 implementation of the differentiable MLS-MPM
//  sub-step of DDBot (arXiv 2510.17335), written from the paper:
//    * the sub-step is Algorithm 1 (Sec. III-A, "System dynamics"), run in the
//      order printed there: F update, SVD, constitutive model, P2G, agent move,
//      gravity, grid collision, G2P, advection;
//    * elasticity: the SVK energy on the logarithmic singular values and its
//      Piola stress (Eqs. SVK, piola), Lame constants from (E, nu);
//    * plasticity: the Drucker-Prager return map on eps = ln S (Eq. DP) with
//      alpha_f from the friction angle;
//    * the stress passed to P2G is sigma = P' F'^T / det F' with det F' := 1
//      imposed, as the text after Eq. DP states;
//    * the digging skill: Eqs. d1 .. delta_d4 and Algorithm 2 (Sec. III-B),
//      optionally with the unrounded T_1^float, T_4^float in the per-action
//      displacements of phases 1 and 4 (the ablation variant of Sec. III-B);
//    * the particle-level collision of Algorithm 1 (optional);
//    * the height-map observation and loss (Eq. hm, Sec. III-A "Goal"), and
//      the earth mover's distance between the surface observation and a
//      target point cloud (Eq. emd) through an exact linear assignment.
//  Gradients are exact forward-mode tangents (Dual<9>) of all of the above with
//  respect to (E, nu, phi_f[deg], rho, insert depth, rotate angle[deg], push
//  distance, displacement d1, push angle phi3[deg]); the rounded phase lengths
//  T_i carry no tangent (Sec. III-B).
//
//  Arithmetic is FP64 throughout, except in the tangents of the SVD-based
//  update: the return map and its tangents run in x87 extended precision and
//  the divided differences of its outputs across pairs of singular values in
//  IEEE binary128 (libquadmath), so that near-equal singular values and small
//  deviators cost no digits (the quotient is evaluated as written, with no
//  threshold or rewrite).
//
//  Nothing in the product may include, link or call this file.  It shares no
//  source with the GPU path.  Readings of points the paper leaves open (grid,
//  walls, shovel shape, contact law, loss terms, cohesion) are listed at each
//  function and follow the build's design notes.
//
//  Parity-pinned pieces are tested from tests/test_oracle_*.py.
// ============================================================================
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include <quadmath.h>

#include "dual.hpp"
#include "tape.hpp"

namespace orc {

static const double kPi = 3.14159265358979323846;
static const double kSigmaMin = 1e-6;   // singular values are clamped before ln

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EDOMAIN = 6 };

// IEEE binary128 scalar (113-bit significand, libquadmath), used only to
// evaluate divided differences of the return map where its FP64 evaluation
// would cancel.
using quad = __float128;
inline quad log(quad x) { return logq(x); }
inline quad exp(quad x) { return expq(x); }
inline quad sqrt(quad x) { return sqrtq(x); }
inline double val(quad x) { return (double)x; }

}  // namespace orc

extern "C" {
// Field order must match oracle/__init__.py.
typedef struct orc_config {
  int32_t dim, n_grid, bound, n_sub;
  int32_t shovel, hm_res, region_sign, skill_unrounded;
  double dt, gravity, ppc;
  double half_w, half_n, half_p;   // shovel half extents along (width, normal, pointing)
  double skin, mu_b;               // contact skin and Coulomb coefficient
  double v_l, v_w, d_lift;         // skill speeds and lift distance
  double tip0[3];                  // initial shovel tip (build frame, y up)
  double hm_origin[2], hm_size, hm_offset;
  double region_depth, m_target, m_ref, w_mass, w_hm;
  double cohesion;
  int32_t particle_contact, pad1;  // Algorithm 1's particle collision on (1) or off (0)
  double w_emd;                    // weight of the EMD term (Eq. emd); 0 = off
} orc_config;
}

namespace orc {

// ---------------------------------------------------------------------------
// Small dense helpers (row-major 3x3, the 2D case uses the upper-left block)
// ---------------------------------------------------------------------------
template <class S> struct M3 { S a[3][3]; };

template <class S> static void set_identity(S A[3][3]) {
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) A[i][j] = S(i == j ? 1.0 : 0.0);
}

// ---------------------------------------------------------------------------
// Skill-to-action mapping (Sec. III-B, Eqs. d1 .. delta_d4, Algorithm 2).
// theta = (displace, rotate, insert_dist, push_dist, push_angle), each in [-1,1].
// Actions are 6-vectors [dx, dy, dz, drx, dry, drz] in the paper's z-up frame.
// Phase bounds are cumulative (the actions of phase i follow those of phase
// i-1), round() is half away from zero, and the T_i carry no derivative.
// unrounded: the per-action displacements of phases 1 and 4 divide by the
// real-valued T_1^float and T_4^float (a tangent flows through them), while
// the number of actions stays T_1, T_4 (Sec. III-B, the alternative mapping;
// max() takes its first argument on ties, as the case split of Appendix A).
// ---------------------------------------------------------------------------
static int round_half_away(double x) { return (int)std::llround(x); }

template <class S> static S max_first(const S& a, const S& b) { return val(a) >= val(b) ? a : b; }

template <class S>
static void skill_actions(const S th[5], double v_l, double v_w, double dta, double d4, bool unrounded,
                          int T[4], std::vector<std::array<S, 6>>* acts) {
  const S d1 = th[0] * 0.12;                          // Eq. d1
  const S phi1 = th[1] * (kPi / 3.0);
  const S Tf_d1 = fabs(d1) / (v_l * dta);             // Eq. Tf1
  const S Tf_phi1 = fabs(phi1) / (v_w * dta);
  const S Tf1 = max_first(Tf_d1, Tf_phi1);
  T[0] = round_half_away(val(Tf1));                   // Eq. Ti1
  const S div1 = unrounded ? Tf1 : S(double(T[0]));
  const S dx1 = T[0] > 0 ? d1 / div1 : S(0.0);        // Eq. delta_d1
  const S drx1 = T[0] > 0 ? phi1 / div1 : S(0.0);

  const S d2 = (th[2] + 1.0) * 0.03;                  // Eq. d2
  const S phi2 = phi1 + kPi / 2.0;
  T[1] = round_half_away(val(d2) / (v_l * dta));      // Eqs. Tf2, Ti2
  const S dx2 = T[1] > 0 ? d2 * cos(phi2) / double(T[1]) : S(0.0);    // Eq. delta_d2
  const S dz2 = T[1] > 0 ? -(d2 * sin(phi2)) / double(T[1]) : S(0.0);

  const S d3 = (th[3] + 1.0) * 0.1 + 0.04;            // Eq. d3
  const S phi3 = (th[4] + 3.0) * (kPi / 3.0);
  T[2] = round_half_away(std::fabs(val(d3) / (v_l * dta)));  // Eqs. Tf3, Ti3
  const S dx3 = T[2] > 0 ? d3 * cos(phi3) / double(T[2]) : S(0.0);    // Eq. delta_d3
  const S dz3 = T[2] > 0 ? d3 * sin(phi3) / double(T[2]) : S(0.0);

  const S Tf_d4 = S(d4 / (v_l * dta));                // Eq. Tf4
  const S Tf4 = max_first(Tf_phi1, Tf_d4);
  T[3] = round_half_away(val(Tf4));                   // Eq. Ti4
  const S div4 = unrounded ? Tf4 : S(double(T[3]));
  const S drx4 = T[3] > 0 ? -phi1 / div4 : S(0.0);    // Eq. delta_d4
  const S dz4 = T[3] > 0 ? d4 / div4 : S(0.0);

  acts->clear();
  const int total = T[0] + T[1] + T[2] + T[3];
  for (int t = 0; t < total; ++t) {
    std::array<S, 6> a;
    for (int k = 0; k < 6; ++k) a[k] = S(0.0);
    if (t < T[0]) { a[0] = dx1; a[3] = drx1; }
    else if (t < T[0] + T[1]) { a[0] = dx2; a[2] = dz2; }
    else if (t < T[0] + T[1] + T[2]) { a[0] = dx3; a[2] = dz3; }
    else { a[3] = drx4; a[2] = dz4; }
    acts->push_back(a);
  }
}

// Physical skill parameters (insert depth d2 [m], rotate angle phi1 [deg],
// push distance d3 [m], displacement d1 [m], push angle phi3 [deg]) to the
// paper's normalised theta, inverting Eqs. d1, d2 and d3.
template <class S>
static void theta_from_physical(const S sk[5], S th[5]) {
  th[0] = sk[3] / 0.12;
  th[1] = sk[1] * (kPi / 180.0) / (kPi / 3.0);
  th[2] = sk[0] / 0.03 - 1.0;
  th[3] = (sk[2] - 0.04) / 0.1 - 1.0;
  th[4] = sk[4] * (kPi / 180.0) / (kPi / 3.0) - 3.0;
}

// Agent pose per sub-step (Sec. III-A "Actions"; the agent move of Algorithm 1).  Build
// frame is y up: paper (x, y, z) maps to (x, z, y), and the paper's rotation
// about its x axis is a rotation psi about -z through the tip.  Entry n holds
// the pose used by the grid collision of sub-step n (after the agent moved)
// and the shovel velocity during that sub-step.
template <class S> struct Pose { S tip[3]; S psi; S vel[3]; S omega; };

template <class S>
static void pose_table(const orc_config& c, const S sk[5], double dt, int n_steps, std::vector<Pose<S>>* out) {
  S th[5];
  theta_from_physical(sk, th);
  int T[4];
  std::vector<std::array<S, 6>> acts;
  skill_actions(th, c.v_l, c.v_w, c.n_sub * dt, c.d_lift, c.skill_unrounded != 0, T, &acts);
  Pose<S> cur;
  for (int k = 0; k < 3; ++k) cur.tip[k] = S(c.tip0[k]);
  cur.psi = S(0.0);
  out->clear();
  for (int n = 0; n < n_steps; ++n) {
    const int t = n / c.n_sub;
    Pose<S> p = cur;
    if (t < (int)acts.size()) {
      const std::array<S, 6>& a = acts[t];
      const S inv_n = S(1.0 / c.n_sub);
      const S d[3] = {a[0] * inv_n, a[2] * inv_n, a[1] * inv_n};   // paper (x,y,z) -> build (x,z,y)
      for (int k = 0; k < 3; ++k) { p.tip[k] = cur.tip[k] + d[k]; p.vel[k] = d[k] / dt; }
      p.psi = cur.psi + a[3] * inv_n;
      p.omega = a[3] * inv_n / dt;
    } else {
      for (int k = 0; k < 3; ++k) p.vel[k] = S(0.0);
      p.omega = S(0.0);
    }
    out->push_back(p);
    cur = p;
  }
}

// ---------------------------------------------------------------------------
// SVD of a d x d matrix by one-sided (Hestenes) Jacobi rotations, iterated to
// full FP64 convergence.  Returns U, V in SO(d) and singular values S (the last
// one negated if det F < 0).  F = U diag(S) V^T.
// ---------------------------------------------------------------------------
static void svd(int d, const double F[3][3], double U[3][3], double S[3], double V[3][3]) {
  double W[3][3];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { W[i][j] = F[i][j]; V[i][j] = (i == j); }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < d; ++p) for (int q = p + 1; q < d; ++q) {
      double al = 0, be = 0, ga = 0;
      for (int k = 0; k < d; ++k) { al += W[k][p] * W[k][p]; be += W[k][q] * W[k][q]; ga += W[k][p] * W[k][q]; }
      if (ga == 0.0) continue;
      const double rel = std::fabs(ga) / std::sqrt(al * be);
      off = std::max(off, rel);
      if (rel < 1e-16) continue;
      const double zeta = (be - al) / (2.0 * ga);
      const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
      const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
      for (int k = 0; k < d; ++k) {
        const double wp = W[k][p], wq = W[k][q];
        W[k][p] = cs * wp - sn * wq; W[k][q] = sn * wp + cs * wq;
        const double vp = V[k][p], vq = V[k][q];
        V[k][p] = cs * vp - sn * vq; V[k][q] = sn * vp + cs * vq;
      }
    }
    if (off < 1e-15) break;
  }
  // Singular values are the column norms; U's columns the normalised columns.
  int order[3] = {0, 1, 2};
  for (int j = 0; j < d; ++j) {
    double n2 = 0;
    for (int k = 0; k < d; ++k) n2 += W[k][j] * W[k][j];
    S[j] = std::sqrt(n2);
  }
  std::sort(order, order + d, [&](int a, int b) { return S[a] > S[b]; });
  double Ss[3] = {0, 0, 0}, Ws[3][3] = {}, Vs[3][3] = {};
  for (int jj = 0; jj < d; ++jj) {
    Ss[jj] = S[order[jj]];
    for (int k = 0; k < d; ++k) { Ws[k][jj] = W[k][order[jj]]; Vs[k][jj] = V[k][order[jj]]; }
  }
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { U[i][j] = 0; V[i][j] = 0; }
  for (int j = 0; j < d; ++j) { S[j] = Ss[j]; for (int k = 0; k < d; ++k) V[k][j] = Vs[k][j]; }
  // Columns of U: normalised where the singular value is not negligible, else
  // completed to an orthonormal basis by Gram-Schmidt on the unit vectors.
  const double tiny = 1e-300;
  for (int j = 0; j < d; ++j) {
    if (S[j] > tiny && S[j] > 1e-14 * S[0]) {
      for (int k = 0; k < d; ++k) U[k][j] = Ws[k][j] / S[j];
    } else {
      for (int e = 0; e < d; ++e) {
        double u[3] = {0, 0, 0};
        u[e] = 1.0;
        for (int jj = 0; jj < j; ++jj) {
          double dp = 0;
          for (int k = 0; k < d; ++k) dp += U[k][jj] * u[k];
          for (int k = 0; k < d; ++k) u[k] -= dp * U[k][jj];
        }
        double nn = 0;
        for (int k = 0; k < d; ++k) nn += u[k] * u[k];
        if (nn > 1e-6) { nn = std::sqrt(nn); for (int k = 0; k < d; ++k) U[k][j] = u[k] / nn; break; }
      }
    }
  }
  // Make det U = det V = +1.  Sorting can leave det V = -1; flipping a column
  // of V together with the matching singular value's sign keeps F = U S V^T.
  auto det = [d](double A[3][3]) {
    if (d == 2) return A[0][0] * A[1][1] - A[0][1] * A[1][0];
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  };
  if (det(V) < 0) { for (int k = 0; k < d; ++k) V[k][d - 1] = -V[k][d - 1]; S[d - 1] = -S[d - 1]; }
  if (det(U) < 0) { for (int k = 0; k < d; ++k) U[k][d - 1] = -U[k][d - 1]; S[d - 1] = -S[d - 1]; }
}

// ---------------------------------------------------------------------------
// Constitutive model on the singular values (Eqs. SVK, piola, DP).
// Input: clamped singular values s; output: plastic singular values g = S_hat
// and principal Kirchhoff stresses h = 2 mu eps' + lambda tr(eps').
// With det F' := 1 imposed, sigma = P' F'^T = U diag(h) U^T.
// Cohesion c (not in the paper): the yield surface is shifted by
// k_c = sqrt(2/3) 6 c cos(phi) / (3 - sin(phi)); it reduces to Eq. DP at c = 0.
// ---------------------------------------------------------------------------
// forced_case (1, 2 or 3) takes that case without testing the conditions; 0
// decides as Eq. DP states.
template <class S>
static void return_map(int d, const S s[3], const S& mu, const S& lam, const S& alpha, const S& kc,
                       S g[3], S h[3], int* dp_case, int forced_case = 0) {
  S eps[3], tr = S(0.0);
  for (int i = 0; i < d; ++i) { eps[i] = log(s[i]); tr += eps[i]; }
  S eh[3], nrm2 = S(0.0);
  for (int i = 0; i < d; ++i) { eh[i] = eps[i] - tr / double(d); nrm2 += eh[i] * eh[i]; }
  const S stiff = double(d) * lam + 2.0 * mu;
  S ep[3];
  // Case 1 (tension: tr eps > 0 when c = 0): project to the cone apex.
  const bool tension = forced_case ? forced_case == 1
                                   : (val(kc) == 0.0 ? val(tr) > 0.0 : val(alpha * stiff * tr) > val(kc));
  if (tension) {
    const S apex = kc / (double(d) * alpha * stiff);
    for (int i = 0; i < d; ++i) ep[i] = apex;
    *dp_case = 1;
  } else {
    const S nrm = val(nrm2) > 0.0 ? sqrt(nrm2) : S(0.0);
    const S dgam = nrm + stiff / (2.0 * mu) * tr * alpha - kc / (2.0 * mu);
    if (forced_case ? forced_case == 2 : val(dgam) <= 0.0) {   // Case 2: inside the cone, unchanged
      for (int i = 0; i < d; ++i) ep[i] = eps[i];
      *dp_case = 2;
    } else {                          // Case 3: project onto the cone surface
      for (int i = 0; i < d; ++i) ep[i] = eps[i] - dgam * eh[i] / nrm;
      *dp_case = 3;
    }
  }
  S tre = S(0.0);
  for (int i = 0; i < d; ++i) tre += ep[i];
  for (int i = 0; i < d; ++i) { g[i] = exp(ep[i]); h[i] = 2.0 * mu * ep[i] + lam * tre; }
  for (int i = d; i < 3; ++i) { g[i] = S(1.0); h[i] = S(0.0); }
}

}  // namespace orc

namespace orc {

// ---------------------------------------------------------------------------
// Constitutive update of one particle (Algorithm 1, SVD and return map) in double.
// F' = U diag(S_hat) V^T and sigma = U diag(h) U^T.
// ---------------------------------------------------------------------------
static void constitutive(int d, const double Ft[3][3], double mu, double lam, double alpha, double kc,
                         double Fn[3][3], double tau[3][3], int* dp_case, int* clamped) {
  double U[3][3], sg[3], V[3][3];
  svd(d, Ft, U, sg, V);
  double s[3] = {1, 1, 1};
  *clamped = 0;
  for (int i = 0; i < d; ++i) {
    s[i] = sg[i];
    if (s[i] < kSigmaMin) { s[i] = kSigmaMin; ++*clamped; }
  }
  double g[3], h[3];
  return_map(d, s, mu, lam, alpha, kc, g, h, dp_case);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { Fn[i][j] = 0; tau[i][j] = 0; }
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) {
    double a = 0, b = 0;
    for (int k = 0; k < d; ++k) { a += U[i][k] * g[k] * V[j][k]; b += U[i][k] * h[k] * U[j][k]; }
    Fn[i][j] = a; tau[i][j] = b;
  }
}

// The same update with K forward tangents.  F' and sigma are isotropic
// functions of F_tmp: F' = U diag(g(s)) V^T and sigma = U diag(h(s)) U^T with g,
// h symmetric in s.  Their differentials in the SVD frame (dF~ = U^T dF V) are
//   diagonal:      dG~_ii = dg_i (chain rule through s_i = dF~_ii and the
//                  material parameters, done by the Dual arithmetic),
//   off-diagonal:  with sym = (dF~_ij + dF~_ji)/2, skw = (dF~_ij - dF~_ji)/2,
//                  dG~_ij = sym (g_i-g_j)/(s_i-s_j) + skw (g_i+g_j)/(s_i+s_j),
//                  dG~_ji = sym (g_i-g_j)/(s_i-s_j) - skw (g_i+g_j)/(s_i+s_j),
//                  dT~_ij = dT~_ji = sym (h_i-h_j)/(s_i-s_j) + skw (h_j-h_i)/(s_i+s_j)
//                  (sigma's frame is U on both sides).
// The divided differences (g_i - g_j)/(s_i - s_j) and (h_i - h_j)/(s_i - s_j)
// are those quotients as written, with g and h evaluated in binary128 at the
// same (double) singular values, parameters and return-map case: for s_i and
// s_j one ulp apart the subtraction still leaves about 18 significant digits,
// so no threshold, quadrature or closed-form rewrite is involved.  Only at an
// exact tie s_i == s_j is the quotient replaced by its limit
// dg_i/ds_i - dg_i/ds_j (Dual<3> derivative at s; g is symmetric).
// This follows from F = U S V^T and never differentiates the SVD iteration.
// ---------------------------------------------------------------------------
template <int K>
static void constitutive(int d, const Dual<K> Ft[3][3], const Dual<K>& mu, const Dual<K>& lam,
                         const Dual<K>& alpha, const Dual<K>& kc, Dual<K> Fn[3][3], Dual<K> tau[3][3],
                         int* dp_case, int* clamped) {
  double Fv[3][3] = {};
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Fv[i][j] = Ft[i][j].v;
  double U[3][3], sg[3], V[3][3];
  svd(d, Fv, U, sg, V);
  double sc[3] = {1, 1, 1};
  bool cl[3] = {false, false, false};
  *clamped = 0;
  for (int i = 0; i < d; ++i) {
    sc[i] = sg[i];
    if (sc[i] < kSigmaMin) { sc[i] = kSigmaMin; cl[i] = true; ++*clamped; }
  }
  // Tangents of F_tmp in the SVD frame.
  double Fk[K][3][3];
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) {
      double a = 0;
      for (int p = 0; p < d; ++p) for (int q = 0; q < d; ++q) a += U[p][i] * Ft[p][q].d[k] * V[q][j];
      Fk[k][i][j] = a;
    }
  Dual<K> s[3];
  for (int i = 0; i < 3; ++i) s[i] = Dual<K>(sc[i]);
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < K; ++k) s[i].d[k] = cl[i] ? 0.0 : Fk[k][i][i];
  // The return map and its tangents in extended precision: near the cone's
  // apex the deviator eps - tr/d is a small difference of logarithms.
  using XD = Dual<K, long double>;
  auto widen = [](const Dual<K>& a) { XD r((long double)a.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k]; return r; };
  auto narrow = [](const XD& a) { Dual<K> r((double)a.v); for (int k = 0; k < K; ++k) r.d[k] = (double)a.d[k]; return r; };
  XD sx[3], gx[3], hx[3];
  for (int q = 0; q < 3; ++q) sx[q] = widen(s[q]);
  return_map(d, sx, widen(mu), widen(lam), widen(alpha), widen(kc), gx, hx, dp_case);
  Dual<K> g[3], h[3];
  for (int q = 0; q < 3; ++q) { g[q] = narrow(gx[q]); h[q] = narrow(hx[q]); }
  // Divided differences of pair (i, j): the quotient of the binary128 return
  // map (evaluated once, at the first untied pair), or its limit at a tie.
  quad gq[3], hq[3];
  bool have_q = false;
  auto pair_dd = [&](int i, int j, double* ddg, double* ddh) {
    if (sc[i] != sc[j]) {
      if (!have_q) {
        const quad sq[3] = {(quad)sc[0], (quad)sc[1], (quad)sc[2]};
        int cq;
        return_map(d, sq, (quad)mu.v, (quad)lam.v, (quad)alpha.v, (quad)kc.v, gq, hq, &cq, *dp_case);
        have_q = true;
      }
      const quad ds = (quad)sc[i] - (quad)sc[j];
      *ddg = (double)((gq[i] - gq[j]) / ds);
      *ddh = (double)((hq[i] - hq[j]) / ds);
      return;
    }
    using X3 = Dual<3, long double>;
    X3 s3[3], g3[3], h3[3];
    for (int q = 0; q < 3; ++q) s3[q] = (q < d && !cl[q]) ? X3::var(sc[q], q) : X3(sc[q]);
    int c3;
    return_map(d, s3, X3(mu.v), X3(lam.v), X3(alpha.v), X3(kc.v), g3, h3, &c3, *dp_case);
    *ddg = (double)(g3[i].d[i] - g3[i].d[j]);
    *ddh = (double)(h3[i].d[i] - h3[i].d[j]);
  };
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { Fn[i][j] = Dual<K>(0.0); tau[i][j] = Dual<K>(0.0); }
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) {
    double a = 0, b = 0;
    for (int p = 0; p < d; ++p) { a += U[i][p] * g[p].v * V[j][p]; b += U[i][p] * h[p].v * U[j][p]; }
    Fn[i][j].v = a; tau[i][j].v = b;
  }
  double ddg[3][3] = {}, ddh[3][3] = {};
  for (int i = 0; i < d; ++i) for (int j = i + 1; j < d; ++j) pair_dd(i, j, &ddg[i][j], &ddh[i][j]);
  for (int k = 0; k < K; ++k) {
    double Gt[3][3] = {}, Tt[3][3] = {};
    for (int i = 0; i < d; ++i) { Gt[i][i] = g[i].d[k]; Tt[i][i] = h[i].d[k]; }
    for (int i = 0; i < d; ++i) for (int j = i + 1; j < d; ++j) {
      const double sym = 0.5 * (Fk[k][i][j] + Fk[k][j][i]);
      const double skw = 0.5 * (Fk[k][i][j] - Fk[k][j][i]);
      const double sgg = (g[i].v + g[j].v) / (sc[i] + sc[j]);
      const double shh = (h[j].v - h[i].v) / (sc[i] + sc[j]);
      Gt[i][j] = sym * ddg[i][j] + skw * sgg;
      Gt[j][i] = sym * ddg[i][j] - skw * sgg;
      Tt[i][j] = Tt[j][i] = sym * ddh[i][j] + skw * shh;
    }
    for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) {
      double a = 0, b = 0;
      for (int p = 0; p < d; ++p) for (int q = 0; q < d; ++q) {
        a += U[i][p] * Gt[p][q] * V[j][q];
        b += U[i][p] * Tt[p][q] * U[j][q];
      }
      Fn[i][j].d[k] = a; tau[i][j].d[k] = b;
    }
  }
}

// The same update on the reverse-mode tape: one node per output entry of F'
// and sigma, whose partials with respect to the entries of F_tmp and to
// (mu, lambda, alpha_f, k_c) are the forward-mode tangents of the update above
// (13 directions), so the tape carries exactly the derivative of the SVD-based
// update that the forward mode uses.
static void constitutive(int d, const RV Ft[3][3], const RV& mu, const RV& lam, const RV& alpha, const RV& kc,
                         RV Fn[3][3], RV tau[3][3], int* dp_case, int* clamped) {
  constexpr int K = 13;
  Dual<K> Fd[3][3], md(mu.v), ld(lam.v), ad(alpha.v), kd(kc.v);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    Fd[i][j] = Dual<K>(Ft[i][j].v);
    if (i < d && j < d) Fd[i][j].d[i * 3 + j] = 1.0;
  }
  md.d[9] = 1.0; ld.d[10] = 1.0; ad.d[11] = 1.0; kd.d[12] = 1.0;
  Dual<K> Fo[3][3], To[3][3];
  constitutive(d, Fd, md, ld, ad, kd, Fo, To, dp_case, clamped);
  const RV* in[K];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) in[i * 3 + j] = &Ft[i][j];
  in[9] = &mu; in[10] = &lam; in[11] = &alpha; in[12] = &kc;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    if (i < d && j < d) {
      Fn[i][j] = RV::node(Fo[i][j].v, K, in, Fo[i][j].d);
      tau[i][j] = RV::node(To[i][j].v, K, in, To[i][j].d);
    } else {
      Fn[i][j] = RV(0.0);
      tau[i][j] = RV(0.0);
    }
  }
}

// ---------------------------------------------------------------------------
// Shovel: an oriented box about the tip (width along z, thin along the digging
// normal, long along the pointing direction), exact box signed distance and
// its gradient.  e_p = (-sin psi, -cos psi, 0), e_n = (cos psi, -sin psi, 0),
// e_w = (0, 0, 1); the box centre is tip - half_p e_p.
// ---------------------------------------------------------------------------
template <class S> struct Frame { S c[3]; S e[3][3]; };   // e[0]=e_w, e[1]=e_n, e[2]=e_p

template <class S>
static Frame<S> shovel_frame(const orc_config& cf, const S tip[3], const S& psi) {
  Frame<S> f;
  const S sp = sin(psi), cp = cos(psi);
  f.e[0][0] = S(0.0); f.e[0][1] = S(0.0); f.e[0][2] = S(1.0);
  f.e[1][0] = cp;     f.e[1][1] = -sp;    f.e[1][2] = S(0.0);
  f.e[2][0] = -sp;    f.e[2][1] = -cp;    f.e[2][2] = S(0.0);
  for (int k = 0; k < 3; ++k) f.c[k] = tip[k] - cf.half_p * f.e[2][k];
  return f;
}

template <class S>
static S box_sdf(const orc_config& cf, const Frame<S>& f, const S x[3], S nrm[3]) {
  const double half[3] = {cf.half_w, cf.half_n, cf.half_p};
  S loc[3], q[3];
  for (int a = 0; a < 3; ++a) {
    loc[a] = S(0.0);
    for (int k = 0; k < 3; ++k) loc[a] += (x[k] - f.c[k]) * f.e[a][k];
    q[a] = fabs(loc[a]) - half[a];
  }
  S out2 = S(0.0);
  bool outside = false;
  for (int a = 0; a < 3; ++a) if (val(q[a]) > 0.0) { out2 += q[a] * q[a]; outside = true; }
  S phi;
  S nl[3];
  if (outside) {
    const S od = sqrt(out2);
    phi = od;
    for (int a = 0; a < 3; ++a) {
      const double sgn = val(loc[a]) >= 0.0 ? 1.0 : -1.0;
      nl[a] = val(q[a]) > 0.0 ? q[a] * sgn / od : S(0.0);
    }
  } else {
    int am = 0;
    for (int a = 1; a < 3; ++a) if (val(q[a]) > val(q[am])) am = a;
    phi = q[am];
    for (int a = 0; a < 3; ++a) nl[a] = S(0.0);
    nl[am] = S(val(loc[am]) >= 0.0 ? 1.0 : -1.0);
  }
  for (int k = 0; k < 3; ++k) {
    nrm[k] = S(0.0);
    for (int a = 0; a < 3; ++a) nrm[k] += nl[a] * f.e[a][k];
  }
  return phi;
}

// Coulomb frictional contact against a moving rigid surface (Algorithm 1, grid collision):
// relative velocity, separating -> unchanged, sticking inside the friction
// cone -> zero relative velocity, else slip with the tangential part reduced.
template <class S>
static void coulomb(const S vs[3], const S n[3], double mu_b, S v[3]) {
  S vr[3], vn = S(0.0);
  for (int k = 0; k < 3; ++k) { vr[k] = v[k] - vs[k]; vn += vr[k] * n[k]; }
  if (val(vn) >= 0.0) return;
  S vt[3], vt2 = S(0.0);
  for (int k = 0; k < 3; ++k) { vt[k] = vr[k] - vn * n[k]; vt2 += vt[k] * vt[k]; }
  const double vtn = std::sqrt(val(vt2));
  if (vtn <= -mu_b * val(vn)) {
    for (int k = 0; k < 3; ++k) v[k] = vs[k];
  } else {
    const S scale = 1.0 + mu_b * vn / sqrt(vt2);
    for (int k = 0; k < 3; ++k) v[k] = vs[k] + scale * vt[k];
  }
}

// Material constants: Lame constants from (E, nu) (Sec. III-A), alpha_f from
// the friction angle (text of Eq. DP), cohesion shift k_c (build reading).
template <class S>
static void material(const S& E, const S& nu, const S& phi_deg, double cohesion, S* mu, S* lam,
                     S* alpha, S* kc) {
  *mu = E / (2.0 * (1.0 + nu));
  *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const S phi = phi_deg * (kPi / 180.0);
  const S sp = sin(phi);
  *alpha = std::sqrt(2.0 / 3.0) * 2.0 * sp / (3.0 - sp);
  *kc = std::sqrt(2.0 / 3.0) * 6.0 * cohesion * cos(phi) / (3.0 - sp);
}

static double gradient_of(double, int) { return 0.0; }
template <int K> static double gradient_of(const Dual<K>& x, int k) { return x.d[k]; }

// ---------------------------------------------------------------------------
// Linear assignment for Eq. emd: the injective map from n rows to m >= n
// columns with the least total cost (the Hungarian method).  Rows are added
// one at a time; each addition runs a Dijkstra-like search over the columns on
// costs reduced by row and column potentials, and augments the matching along
// the cheapest path found, after which the potentials are updated so that the
// reduced costs stay non-negative.  O(n^2 m).  cost is n x m, row-major;
// returns the column of every row.
// ---------------------------------------------------------------------------
static void assign_min_cost(int n, int m, const std::vector<double>& cost, std::vector<int>* row_col) {
  const double kInf = std::numeric_limits<double>::infinity();
  std::vector<double> u(n + 1, 0.0), v(m + 1, 0.0), slack(m + 1);
  std::vector<int> match(m + 1, 0), from(m + 1, 0);   // match[j]: row of column j (1-based, 0 = free)
  std::vector<char> done(m + 1);
  for (int i = 1; i <= n; ++i) {
    match[0] = i;                                     // column 0 is the root of the search
    int j0 = 0;
    std::fill(slack.begin(), slack.end(), kInf);
    std::fill(done.begin(), done.end(), 0);
    do {
      done[j0] = 1;
      const int i0 = match[j0];
      double delta = kInf;
      int j1 = 0;
      for (int j = 1; j <= m; ++j) {
        if (done[j]) continue;
        const double red = cost[(size_t)(i0 - 1) * m + (j - 1)] - u[i0] - v[j];
        if (red < slack[j]) { slack[j] = red; from[j] = j0; }
        if (slack[j] < delta) { delta = slack[j]; j1 = j; }
      }
      for (int j = 0; j <= m; ++j) {
        if (done[j]) { u[match[j]] += delta; v[j] -= delta; }
        else slack[j] -= delta;
      }
      j0 = j1;
    } while (match[j0] != 0);
    while (j0) {                                      // augment along the path back to the root
      const int j1 = from[j0];
      match[j0] = match[j1];
      j0 = j1;
    }
  }
  row_col->assign(n, -1);
  for (int j = 1; j <= m; ++j) if (match[j]) (*row_col)[match[j] - 1] = j - 1;
}

// A value the reverse-mode tape must see as a variable.  A grid velocity set
// by a wall (zero) or by the blade during a phase with constant pose is a
// constant of the differentiated inputs; the reverse pass still holds an
// adjoint for it, which its treatments count.  On the tape such a value
// becomes a variable of its own with no parents; elsewhere it is unchanged.
template <class S> static S as_variable(const S& x) { return x; }
static RV as_variable(const RV& x) { return x.i >= 0 ? x : RV::input(x.v); }

// ---------------------------------------------------------------------------
// The simulator state and one sub-step (Algorithm 1).
// ---------------------------------------------------------------------------
template <class S>
struct Sim {
  const orc_config& c;
  int d, n, N, nodes;
  double dx, inv_dx, Vp, dt;
  S mu, lam, alpha, kc, mp;
  std::vector<S> x, v, C, F;          // N*3, N*3, N*9, N*9
  std::vector<S> gm, gmv, gv;         // nodes, nodes*3, nodes*3
  std::vector<Pose<S>> poses;
  const double* emd_target = nullptr;  // [emd_m][3] target surface points (Eq. emd)
  int emd_m = 0;
  int64_t stats[8];                    // clamps, case1, case2, case3, domain errors, EMD overflow

  Sim(const orc_config& cf, int N_) : c(cf), d(cf.dim), n(cf.n_grid), N(N_) {
    nodes = 1;
    for (int a = 0; a < d; ++a) nodes *= n;
    dx = 1.0 / n; inv_dx = double(n); dt = cf.dt;
    Vp = std::pow(dx, d) / cf.ppc;
    x.assign(N * 3, S(0.0)); v.assign(N * 3, S(0.0)); C.assign(N * 9, S(0.0)); F.assign(N * 9, S(0.0));
    gm.assign(nodes, S(0.0)); gmv.assign(nodes * 3, S(0.0)); gv.assign(nodes * 3, S(0.0));
    for (int k = 0; k < 8; ++k) stats[k] = 0;
  }

  // Material constants and particle mass m_p = rho V_p.
  void set_material(const S& E, const S& nu, const S& phi_deg, const S& rho) {
    material(E, nu, phi_deg, c.cohesion, &mu, &lam, &alpha, &kc);
    mp = rho * Vp;
  }

  int node_index(const int idx[3]) const {
    return d == 2 ? idx[0] * n + idx[1] : (idx[0] * n + idx[1]) * n + idx[2];
  }

  // Quadratic B-spline stencil of a particle: base node = floor(x/dx - 1/2)
  // per axis, fractional offset f in [1/2, 3/2), weights over 3 nodes.
  bool stencil(int p, int base[3], S fx[3], S w[3][3]) {
    for (int a = 0; a < d; ++a) {
      base[a] = (int)std::floor(val(x[p * 3 + a]) * inv_dx - 0.5);
      if (base[a] < 0 || base[a] + 2 >= n) { stats[4]++; return false; }
      fx[a] = x[p * 3 + a] * inv_dx - double(base[a]);
      w[a][0] = 0.5 * (1.5 - fx[a]) * (1.5 - fx[a]);
      w[a][1] = 0.75 - (fx[a] - 1.0) * (fx[a] - 1.0);
      w[a][2] = 0.5 * (fx[a] - 0.5) * (fx[a] - 0.5);
    }
    return true;
  }

  // F update, SVD, constitutive model, P2G.
  bool p2g() {
    std::fill(gm.begin(), gm.end(), S(0.0));
    std::fill(gmv.begin(), gmv.end(), S(0.0));
    const double Dinv = 4.0 * inv_dx * inv_dx;
    for (int p = 0; p < N; ++p) {
      S Ft[3][3], Fn[3][3], tau[3][3];
      for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        S acc = S(0.0);
        for (int k = 0; k < d; ++k) {
          const S ik = S(i == k ? 1.0 : 0.0) + dt * C[p * 9 + i * 3 + k];
          acc += ik * F[p * 9 + k * 3 + j];
        }
        Ft[i][j] = (i < d && j < d) ? acc : S(0.0);
      }
      int cs, ncl;
      constitutive(d, Ft, mu, lam, alpha, kc, Fn, tau, &cs, &ncl);
      stats[0] += ncl; stats[cs]++;
      for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) F[p * 9 + i * 3 + j] = Fn[i][j];
      // MLS-MPM affine momentum: A = -dt V_p (4/dx^2) sigma + m_p C.
      S A[3][3];
      for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j)
        A[i][j] = (-dt * Vp * Dinv) * tau[i][j] + mp * C[p * 9 + i * 3 + j];
      int base[3] = {0, 0, 0};
      S fx[3], w[3][3];
      if (!stencil(p, base, fx, w)) return false;
      const int o2 = d == 3 ? 3 : 1;
      for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int oz = 0; oz < o2; ++oz) {
        const int off[3] = {o0, o1, oz};
        S wt = S(1.0), r[3];
        int idx[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) r[a] = S(0.0);
        for (int a = 0; a < d; ++a) { wt = wt * w[a][off[a]]; r[a] = (double(off[a]) - fx[a]) * dx; idx[a] = base[a] + off[a]; }
        const int gi = node_index(idx);
        gm[gi] += wt * mp;
        for (int a = 0; a < d; ++a) {
          S ar = S(0.0);
          for (int b = 0; b < d; ++b) ar += A[a][b] * r[b];
          gmv[gi * 3 + a] += wt * (mp * v[p * 3 + a] + ar);
        }
      }
    }
    return true;
  }

  // Agent pose of this sub-step, gravity, collision (shovel, then
  // sticky container walls of `bound` node layers).
  void grid_update(int step) {
    const bool shovel = c.shovel && d == 3;
    Frame<S> fr;
    if (shovel) fr = shovel_frame(c, poses[step].tip, poses[step].psi);
    for (int gi = 0; gi < nodes; ++gi) {
      int idx[3] = {0, 0, 0};
      if (d == 2) { idx[0] = gi / n; idx[1] = gi % n; }
      else { idx[0] = gi / (n * n); idx[1] = (gi / n) % n; idx[2] = gi % n; }
      S vv[3] = {S(0.0), S(0.0), S(0.0)};
      if (val(gm[gi]) > 0.0) {
        for (int a = 0; a < d; ++a) vv[a] = gmv[gi * 3 + a] / gm[gi];
        vv[1] += dt * c.gravity;
        if (shovel) {
          S xi[3], nr[3];
          for (int a = 0; a < 3; ++a) xi[a] = S(idx[a] * dx);
          const S phi = box_sdf(c, fr, xi, nr);
          if (val(phi) < c.skin) {
            const Pose<S>& P = poses[step];
            // Rigid velocity v_lin + omega x (x - tip), omega = (0, 0, -psi_dot).
            S vs[3];
            vs[0] = P.vel[0] + P.omega * (xi[1] - P.tip[1]);
            vs[1] = P.vel[1] - P.omega * (xi[0] - P.tip[0]);
            vs[2] = P.vel[2];
            coulomb(vs, nr, c.mu_b, vv);
          }
        }
        bool wall = false;
        for (int a = 0; a < d; ++a) if (idx[a] < c.bound || idx[a] >= n - c.bound) wall = true;
        if (wall) for (int a = 0; a < 3; ++a) vv[a] = S(0.0);
        for (int a = 0; a < d; ++a) vv[a] = as_variable(vv[a]);
      }
      for (int a = 0; a < 3; ++a) gv[gi * 3 + a] = vv[a];
    }
  }

  // Particle collision: the grid collision applied to a particle's velocity at its
  // position x_p (before advection): the shovel's Coulomb contact when x_p is
  // within the contact skin, then the sticky container (zero velocity) when
  // x_p lies in the wall layers (closer than bound cells to a face).
  void particle_collision(int p, int step, S vn[3]) {
    if (c.shovel && d == 3) {
      const Frame<S> fr = shovel_frame(c, poses[step].tip, poses[step].psi);
      S xp[3] = {x[p * 3 + 0], x[p * 3 + 1], x[p * 3 + 2]}, nr[3];
      const S phi = box_sdf(c, fr, xp, nr);
      if (val(phi) < c.skin) {
        const Pose<S>& P = poses[step];
        S vs[3];
        vs[0] = P.vel[0] + P.omega * (xp[1] - P.tip[1]);
        vs[1] = P.vel[1] - P.omega * (xp[0] - P.tip[0]);
        vs[2] = P.vel[2];
        coulomb(vs, nr, c.mu_b, vn);
      }
    }
    bool wall = false;
    for (int a = 0; a < d; ++a) {
      const double xa = val(x[p * 3 + a]);
      if (xa < c.bound * dx || xa >= (n - c.bound) * dx) wall = true;
    }
    if (wall) for (int a = 0; a < 3; ++a) vn[a] = S(0.0);
  }

  // G2P (APIC velocity and affine matrix), particle collision
  // (when enabled), advection.
  bool g2p(int step) {
    const double Dinv = 4.0 * inv_dx * inv_dx;
    for (int p = 0; p < N; ++p) {
      int base[3] = {0, 0, 0};
      S fx[3], w[3][3];
      if (!stencil(p, base, fx, w)) return false;
      S vn[3] = {S(0.0), S(0.0), S(0.0)}, Cn[3][3];
      for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Cn[i][j] = S(0.0);
      const int o2 = d == 3 ? 3 : 1;
      for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int oz = 0; oz < o2; ++oz) {
        const int off[3] = {o0, o1, oz};
        S wt = S(1.0), r[3];
        int idx[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) r[a] = S(0.0);
        for (int a = 0; a < d; ++a) { wt = wt * w[a][off[a]]; r[a] = (double(off[a]) - fx[a]) * dx; idx[a] = base[a] + off[a]; }
        const int gi = node_index(idx);
        for (int a = 0; a < d; ++a) {
          vn[a] += wt * gv[gi * 3 + a];
          for (int b = 0; b < d; ++b) Cn[a][b] += (Dinv * wt) * gv[gi * 3 + a] * r[b];
        }
      }
      if (c.particle_contact) particle_collision(p, step, vn);
      for (int a = 0; a < d; ++a) {
        v[p * 3 + a] = as_variable(vn[a]);
        x[p * 3 + a] += dt * vn[a];
        for (int b = 0; b < d; ++b) C[p * 9 + a * 3 + b] = Cn[a][b];
      }
    }
    return true;
  }

  bool substep(int step) {
    if (!p2g()) return false;
    grid_update(step);
    return g2p(step);
  }

  // ------------------------------------------------------------------------
  // Loss at the final state.
  // Height map (Sec. III-A, Eq. hm): every particle touches the pixel of its
  // own (x, z) and of the four points offset by +-r along x and z; a pixel
  // keeps the largest height y seen (initialised to 0; ties keep the lowest
  // particle index).  In 2D the map is a 1D profile over x with 3 points.
  // Loss = w_hm / n_pix * sum(((H - H_target)/dx)^2)
  //      + w_mass * ((M_in - m_target)/m_ref)^2, where M_in is the grid mass
  // (a P2G of particle masses at the final positions) of the nodes inside the
  // scoop slab on the push side of the final blade pose.
  // ------------------------------------------------------------------------
  // Owner of every height-map pixel: the particle with the largest height y
  // among those whose stencil points fall in the pixel, lowest index on ties;
  // -1 when no particle above y = 0 reaches it (the map starts at 0).
  std::vector<int> heightmap_owners() const {
    const int res = c.hm_res;
    const int npix = d == 3 ? res * res : res;
    std::vector<int> own(npix, -1);
    const double pix = c.hm_size / res;
    const double r = c.hm_offset;
    for (int p = 0; p < N; ++p) {
      const double y = val(x[p * 3 + 1]);
      const int npts = d == 3 ? 5 : 3;
      const double ox[5] = {0, r, -r, 0, 0}, oz[5] = {0, 0, 0, r, -r};
      for (int k = 0; k < npts; ++k) {
        const double px = val(x[p * 3 + 0]) + ox[k];
        const int ix = (int)std::floor((px - c.hm_origin[0]) / pix);
        int iz = 0;
        if (d == 3) {
          const double pz = val(x[p * 3 + 2]) + oz[k];
          iz = (int)std::floor((pz - c.hm_origin[1]) / pix);
          if (iz < 0 || iz >= res) continue;
        }
        if (ix < 0 || ix >= res) continue;
        int& o = own[d == 3 ? ix * res + iz : ix];
        if (y > (o < 0 ? 0.0 : val(x[o * 3 + 1]))) o = p;
      }
    }
    return own;
  }

  S loss(const double* target, int final_step, std::vector<S>* H_out) {
    const int res = c.hm_res;
    const int npix = d == 3 ? res * res : res;
    const std::vector<int> own = heightmap_owners();
    std::vector<S> H(npix, S(0.0));
    for (int i = 0; i < npix; ++i) if (own[i] >= 0) H[i] = x[own[i] * 3 + 1];
    S L = S(0.0);
    for (int i = 0; i < npix; ++i) {
      const S e = (H[i] - target[i]) * inv_dx;
      L += e * e;
    }
    L = L * (c.w_hm / npix);
    if (H_out) *H_out = H;
    if (c.shovel && d == 3 && c.w_mass != 0.0) {
      const Pose<S>& P = poses[final_step];
      const Frame<S> fr = shovel_frame(c, P.tip, P.psi);
      S Min = S(0.0);
      for (int p = 0; p < N; ++p) {
        int base[3];
        S fx[3], w[3][3];
        if (!stencil(p, base, fx, w)) continue;
        for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int o2 = 0; o2 < 3; ++o2) {
          const int idx[3] = {base[0] + o0, base[1] + o1, base[2] + o2};
          double q[3];
          for (int a = 0; a < 3; ++a) {
            q[a] = 0;
            for (int k = 0; k < 3; ++k) q[a] += (idx[k] * dx - val(fr.c[k])) * val(fr.e[a][k]);
          }
          const double sn = c.region_sign * q[1];
          const bool in = std::fabs(q[0]) <= c.half_w && std::fabs(q[2]) <= c.half_p &&
                          sn > c.half_n && sn <= c.half_n + c.region_depth;
          if (in) Min += w[0][o0] * w[1][o1] * w[2][o2] * mp;
        }
      }
      const S e = (Min - c.m_target) / c.m_ref;
      L += c.w_mass * e * e;
    }
    if (d == 3 && c.w_emd != 0.0) L += c.w_emd * emd();
    return L;
  }

  // Surface observation (Sec. III-A, "States and observations"): in each pixel
  // of the height-map window, the highest particle whose own (x, z) lies in it
  // (ties keep the lowest particle index); empty pixels give no point.
  std::vector<int> surface_particles() const {
    const int res = c.hm_res;
    const double pix = c.hm_size / res;
    std::vector<int> own(res * res, -1);
    for (int p = 0; p < N; ++p) {
      const int ix = (int)std::floor((val(x[p * 3 + 0]) - c.hm_origin[0]) / pix);
      const int iz = (int)std::floor((val(x[p * 3 + 2]) - c.hm_origin[1]) / pix);
      if (ix < 0 || ix >= res || iz < 0 || iz >= res) continue;
      int& o = own[ix * res + iz];
      if (o < 0 || val(x[p * 3 + 1]) > val(x[o * 3 + 1])) o = p;
    }
    std::vector<int> out;
    for (int o : own) if (o >= 0) out.push_back(o);
    return out;
  }

  // Eq. emd: the sum over the observed points of the distance to their
  // targets under the cheapest one-to-one assignment (it exists when there
  // are no more points than targets; otherwise stats[5] counts the failure
  // and the term is 0).  The assignment is a choice and carries no tangent.
  S emd() {
    const std::vector<int> obs = surface_particles();
    const int n = (int)obs.size(), m = emd_m;
    if (n == 0) return S(0.0);
    if (n > m || !emd_target) { stats[5]++; return S(0.0); }
    std::vector<double> cost((size_t)n * m);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < m; ++j) {
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a) { const double dd = val(x[obs[i] * 3 + a]) - emd_target[j * 3 + a]; s2 += dd * dd; }
        cost[(size_t)i * m + j] = std::sqrt(s2);
      }
    std::vector<int> phi;
    assign_min_cost(n, m, cost, &phi);
    S total = S(0.0);
    for (int i = 0; i < n; ++i) {
      S s2 = S(0.0);
      for (int a = 0; a < 3; ++a) { const S dd = x[obs[i] * 3 + a] - emd_target[phi[i] * 3 + a]; s2 += dd * dd; }
      if (val(s2) > 0.0) total += sqrt(s2);
    }
    return total;
  }
};

template <class S> static S param(const double* p, int k, bool dual);
template <> double param<double>(const double* p, int k, bool) { return p[k]; }
template <> Dual<9> param<Dual<9>>(const double* p, int k, bool) { return Dual<9>::var(p[k], k); }

static int validate(const orc_config* c, const double* p) {
  if (c->dim != 2 && c->dim != 3) return ORC_EINVAL;
  if (c->n_grid < 8 || c->dt <= 0 || c->ppc <= 0 || c->n_sub <= 0) return ORC_EINVAL;
  if (!(p[0] > 0) || !(p[1] > -1.0 && p[1] < 0.5) || !(p[2] > 0 && p[2] < 90) || !(p[3] > 0)) return ORC_EINVAL;
  return ORC_OK;
}

// Runs sub-steps [step0, step0 + n_steps) from a packed state and writes back
// the final state; optional loss and 9 gradients (the parameter order of p).
template <class S>
static int rollout(const orc_config* c, const double* p, int N, const double* state_in, int step0,
                   int n_steps, double* state_out, const double* target, double* loss_out,
                   double* grad_out, double* hm_out, int64_t* stats, double* grid_out, const double* emd_target,
                   int emd_m) {
  const bool dual = grad_out != nullptr;
  Sim<S> sim(*c, N);
  sim.emd_target = emd_target;
  sim.emd_m = emd_m;
  sim.set_material(param<S>(p, 0, dual), param<S>(p, 1, dual), param<S>(p, 2, dual), param<S>(p, 3, dual));
  const int total = step0 + n_steps;
  if (c->shovel && c->dim == 3) {
    const S sk[5] = {param<S>(p, 4, dual), param<S>(p, 5, dual), param<S>(p, 6, dual), param<S>(p, 7, dual),
                     param<S>(p, 8, dual)};
    pose_table(*c, sk, c->dt, std::max(total, 1), &sim.poses);
  }
  const int d = c->dim, sd = 2 * d + 2 * d * d;
  for (int q = 0; q < N; ++q) {
    const double* s = state_in + (size_t)q * sd;
    for (int a = 0; a < d; ++a) { sim.x[q * 3 + a] = S(s[a]); sim.v[q * 3 + a] = S(s[d + a]); }
    for (int a = 0; a < d; ++a) for (int b = 0; b < d; ++b) {
      sim.C[q * 9 + a * 3 + b] = S(s[2 * d + a * d + b]);
      sim.F[q * 9 + a * 3 + b] = S(s[2 * d + d * d + a * d + b]);
    }
  }
  int rc = ORC_OK;
  for (int st = step0; st < total; ++st) {
    if (grid_out && st == total - 1) {
      // Record the grid of the last step: P2G mass/momentum, then velocity.
      if (!sim.p2g()) { rc = ORC_EDOMAIN; break; }
      for (int gi = 0; gi < sim.nodes; ++gi) {
        grid_out[gi * 7 + 0] = val(sim.gm[gi]);
        for (int a = 0; a < 3; ++a) grid_out[gi * 7 + 1 + a] = val(sim.gmv[gi * 3 + a]);
      }
      sim.grid_update(st);
      for (int gi = 0; gi < sim.nodes; ++gi)
        for (int a = 0; a < 3; ++a) grid_out[gi * 7 + 4 + a] = val(sim.gv[gi * 3 + a]);
      if (!sim.g2p(st)) { rc = ORC_EDOMAIN; break; }
    } else if (!sim.substep(st)) { rc = ORC_EDOMAIN; break; }
  }
  if (stats) for (int k = 0; k < 8; ++k) stats[k] = sim.stats[k];
  if (rc != ORC_OK) return rc;
  if (state_out)
    for (int q = 0; q < N; ++q) {
      double* s = state_out + (size_t)q * sd;
      for (int a = 0; a < d; ++a) { s[a] = val(sim.x[q * 3 + a]); s[d + a] = val(sim.v[q * 3 + a]); }
      for (int a = 0; a < d; ++a) for (int b = 0; b < d; ++b) {
        s[2 * d + a * d + b] = val(sim.C[q * 9 + a * 3 + b]);
        s[2 * d + d * d + a * d + b] = val(sim.F[q * 9 + a * 3 + b]);
      }
    }
  if (target) {
    std::vector<S> H;
    const S L = sim.loss(target, total - 1, &H);
    if (loss_out) *loss_out = val(L);
    if (hm_out) for (size_t i = 0; i < H.size(); ++i) hm_out[i] = val(H[i]);
    if (grad_out) for (int k = 0; k < 9; ++k) grad_out[k] = gradient_of(L, k);
  }
  return ORC_OK;
}

// ---------------------------------------------------------------------------
// Reverse mode with the gradient treatments of Sec. III-E.  The rollout is
// recorded on a tape (every operation of Algorithm 1, the loss, the skill's
// pose table and the material constants), then swept backwards once.  The
// adjoint of each key variable is treated, one vector per variable, where it
// is complete: the grid velocities after the grid update of sub-step n once
// the G2P of n is swept, the grid momenta and masses of P2G n once the grid
// update of n is swept, and the particle positions, velocities and
// deformation gradients of the state entering sub-step n once all of
// sub-step n is swept.  The loss's own seed is not treated.
// Rules (Sec. III-E): clip every element to [-c, c]; scale: divide by
// 10^dd + delta when dd = round(log10 max|g|) - oom* > 0 (halves away from
// zero); normalise: divide by the 2-norm + delta.
// ---------------------------------------------------------------------------
enum { TREAT_NONE = 0, TREAT_CLIP = 1, TREAT_SCALE = 2, TREAT_NORM = 3 };

static void treat_values(std::vector<double>& g, int mode, double c, double oom, double delta) {
  if (mode == TREAT_CLIP) {
    for (double& x : g) x = std::min(std::max(x, -c), c);
  } else if (mode == TREAT_SCALE) {
    double amax = 0.0;
    for (double x : g) amax = std::max(amax, std::fabs(x));
    if (!(amax > 0.0) || std::isinf(amax)) return;
    const double l = std::log10(amax);
    const double r = std::copysign(std::floor(std::fabs(l) + 0.5), l);
    const double dd = r - oom;
    if (dd > 0) { const double f = std::pow(10.0, dd) + delta; for (double& x : g) x /= f; }
  } else if (mode == TREAT_NORM) {
    double s2 = 0.0;
    for (double x : g) s2 += x * x;
    const double den = std::sqrt(s2) + delta;
    if (den > 0) for (double& x : g) x /= den;
  }
}

static void vector_stats(const std::vector<double>& g, double out[3]) {
  if (g.empty()) { out[0] = out[1] = out[2] = 0.0; return; }
  double mx = g[0], mn = g[0], s2 = 0.0;
  for (double x : g) { mx = std::max(mx, x); mn = std::min(mn, x); s2 += x * x; }
  out[0] = mx; out[1] = mn; out[2] = std::sqrt(s2);
}

struct TapeMark {
  int64_t pos;                       // tape size when the variables were complete in the forward
  int step, var;                     // sub-step and variable (0 x, 1 v, 2 F, 3 grid v, 4 grid mv, 5 grid m)
  std::vector<int32_t> idx;          // tape nodes of the vector's elements (-1: a constant)
};

static int rollout_reverse(const orc_config* c, const double* p, int N, const double* state_in, int step0, int n_steps,
                           const double* target, int mode, double clip_c, double oom, double delta, double* loss_out,
                           double* grad_out, double* stats_out) {
  Tape tape;
  active_tape() = &tape;
  const int d = c->dim, sd = 2 * d + 2 * d * d;
  RV prm[9];
  for (int k = 0; k < 9; ++k) prm[k] = RV::input(p[k]);
  std::vector<TapeMark> marks;
  int rc = ORC_OK;
  {
    Sim<RV> sim(*c, N);
    sim.set_material(prm[0], prm[1], prm[2], prm[3]);
    const int total = step0 + n_steps;
    if (c->shovel && c->dim == 3) {
      const RV sk[5] = {prm[4], prm[5], prm[6], prm[7], prm[8]};
      pose_table(*c, sk, c->dt, std::max(total, 1), &sim.poses);
    }
    // the initial state is a set of variables too: its adjoint is the first
    // treated vector of the sweep's end, as in the reverse pass
    for (int q = 0; q < N; ++q) {
      const double* st = state_in + (size_t)q * sd;
      for (int a = 0; a < d; ++a) { sim.x[q * 3 + a] = RV::input(st[a]); sim.v[q * 3 + a] = RV::input(st[d + a]); }
      for (int a = 0; a < d; ++a) for (int b = 0; b < d; ++b) {
        sim.C[q * 9 + a * 3 + b] = RV::input(st[2 * d + a * d + b]);
        sim.F[q * 9 + a * 3 + b] = RV::input(st[2 * d + d * d + a * d + b]);
      }
    }
    auto mark = [&](int step, int var) {
      TapeMark m;
      m.pos = tape.size();
      m.step = step;
      m.var = var;
      if (var == 0 || var == 1) {
        const std::vector<RV>& src = var == 0 ? sim.x : sim.v;
        for (int q = 0; q < N; ++q) for (int a = 0; a < d; ++a) m.idx.push_back(src[q * 3 + a].i);
      } else if (var == 2) {
        for (int q = 0; q < N; ++q) for (int a = 0; a < d; ++a) for (int b = 0; b < d; ++b)
          m.idx.push_back(sim.F[q * 9 + a * 3 + b].i);
      } else if (var == 3 || var == 4) {
        const std::vector<RV>& src = var == 3 ? sim.gv : sim.gmv;
        for (int g = 0; g < sim.nodes; ++g) for (int a = 0; a < d; ++a) m.idx.push_back(src[g * 3 + a].i);
      } else {
        for (int g = 0; g < sim.nodes; ++g) m.idx.push_back(sim.gm[g].i);
      }
      marks.push_back(std::move(m));
    };
    for (int st = step0; st < total && rc == ORC_OK; ++st) {
      mark(st, 0); mark(st, 1); mark(st, 2);
      if (!sim.p2g()) { rc = ORC_EDOMAIN; break; }
      mark(st, 4); mark(st, 5);
      sim.grid_update(st);
      mark(st, 3);
      if (!sim.g2p(st)) rc = ORC_EDOMAIN;
    }
    if (rc == ORC_OK) {
      std::vector<RV> H;
      const RV L = sim.loss(target, total - 1, &H);
      if (loss_out) *loss_out = L.v;
      tape.adj.assign((size_t)tape.size(), 0.0);
      if (L.i >= 0) tape.adj[(size_t)L.i] = 1.0;
      // the sweep, treating each marked vector once every later node is swept
      int64_t i = tape.size() - 1;
      for (int mk = (int)marks.size() - 1; mk >= -1; --mk) {
        const int64_t stop = mk >= 0 ? marks[(size_t)mk].pos : 0;
        for (; i >= stop; --i) tape.back(i);
        if (mk < 0) break;
        TapeMark& m = marks[(size_t)mk];
        std::vector<double> g(m.idx.size());
        for (size_t k = 0; k < g.size(); ++k) g[k] = m.idx[k] >= 0 ? tape.adj[(size_t)m.idx[k]] : 0.0;
        double* so = stats_out ? stats_out + ((size_t)(m.step - step0) * 6 + m.var) * 6 : nullptr;
        if (so) vector_stats(g, so);
        treat_values(g, mode, clip_c, oom, delta);
        if (so) vector_stats(g, so + 3);
        for (size_t k = 0; k < g.size(); ++k) if (m.idx[k] >= 0) tape.adj[(size_t)m.idx[k]] = g[k];
      }
      for (int k = 0; k < 9; ++k) grad_out[k] = tape.adj[(size_t)prm[k].i];
    }
  }
  active_tape() = nullptr;
  return rc;
}

// ---------------------------------------------------------------------------
// Per-step diagnostics of a state (x, v, C, F per particle): the particle
// mass N m_p, the momentum sum m_p v_p, the kinetic energy sum m_p |v_p|^2 / 2,
// the return-map case (Eq. DP) and the clamped singular values of the next
// constitutive update on F_tmp = (I + dt C) F, and the CFL number
// max_p max_a |v_a| dt / dx.  Plain loops over the particles; the cases come
// from the same constitutive update the rollout runs.
// ---------------------------------------------------------------------------
static int diagnostics(const orc_config* c, const double* p, int N, const double* state_in, double* out) {
  Sim<double> sim(*c, N);
  sim.set_material(p[0], p[1], p[2], p[3]);
  const int d = c->dim, sd = 2 * d + 2 * d * d;
  for (int k = 0; k < 10; ++k) out[k] = 0.0;
  for (int q = 0; q < N; ++q) {
    const double* s = state_in + (size_t)q * sd;
    double Cm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, F[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int a = 0; a < d; ++a) for (int b = 0; b < d; ++b) {
      Cm[a][b] = s[2 * d + a * d + b];
      F[a][b] = s[2 * d + d * d + a * d + b];
    }
    out[0] += sim.mp;
    double vmax = 0.0;
    for (int a = 0; a < d; ++a) {
      const double va = s[d + a];
      out[1 + a] += sim.mp * va;
      out[4] += 0.5 * sim.mp * va * va;
      vmax = std::max(vmax, std::fabs(va));
    }
    out[9] = std::max(out[9], vmax * sim.dt * sim.inv_dx);
    double Ft[3][3], Fn[3][3], tau[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += ((i == k ? 1.0 : 0.0) + sim.dt * Cm[i][k]) * F[k][j];
      Ft[i][j] = (i < d && j < d) ? acc : 0.0;
    }
    int cs = 0, ncl = 0;
    constitutive(d, Ft, sim.mu, sim.lam, sim.alpha, sim.kc, Fn, tau, &cs, &ncl);
    out[4 + cs] += 1.0;
    out[8] += ncl;
  }
  out[10] = std::nan("");
  return ORC_OK;
}

}  // namespace orc

// ============================================================================
// C interface (ctypes, from oracle/__init__.py)
// ============================================================================
using namespace orc;

extern "C" {

int orc_rollout(const orc_config* c, const double* p, int N, const double* state_in, int step0, int n_steps,
                double* state_out, const double* target, double* loss_out, double* grad_out,
                double* hm_out, int64_t* stats, double* grid_out, const double* emd_target, int emd_m) {
  if (validate(c, p) != ORC_OK || N < 0 || n_steps < 0 || step0 < 0 || emd_m < 0) return ORC_EINVAL;
  if (grad_out)
    return rollout<Dual<9>>(c, p, N, state_in, step0, n_steps, state_out, target, loss_out, grad_out, hm_out, stats,
                            grid_out, emd_target, emd_m);
  return rollout<double>(c, p, N, state_in, step0, n_steps, state_out, target, loss_out, nullptr, hm_out, stats,
                         grid_out, emd_target, emd_m);
}

// Diagnostics of a state (11 doubles: mass, momentum[3], kinetic energy,
// return-map cases 1..3 and clamps of the next constitutive update, CFL
// number, and NaN for the grid mass, which needs the last sub-step's grid).
int orc_diagnostics(const orc_config* c, const double* p, int N, const double* state_in, double* out) {
  if (validate(c, p) != ORC_OK || N < 0 || !state_in || !out) return ORC_EINVAL;
  return diagnostics(c, p, N, state_in, out);
}

// Reverse-mode gradient of the loss with the gradient treatments of
// Sec. III-E (mode 0 none, 1 clip, 2 scale, 3 normalise): loss, the 9
// parameter gradients, and (optional) per sub-step and variable the max, min
// and 2-norm of each adjoint vector before and after its treatment,
// stats[n_steps][6][6].  No EMD term.
int orc_rollout_reverse(const orc_config* c, const double* p, int N, const double* state_in, int step0, int n_steps,
                        const double* target, int mode, double clip_c, double oom, double delta, double* loss_out,
                        double* grad_out, double* stats_out) {
  if (validate(c, p) != ORC_OK || N < 0 || n_steps < 1 || step0 < 0 || !target || !grad_out || mode < 0 || mode > 3 ||
      c->w_emd != 0.0)
    return ORC_EINVAL;
  return rollout_reverse(c, p, N, state_in, step0, n_steps, target, mode, clip_c, oom, delta, loss_out, grad_out,
                         stats_out);
}

// One treatment (Sec. III-E) of a caller's vector, in place.
void orc_treat(int mode, int n, double* g, double clip_c, double oom, double delta) {
  std::vector<double> v(g, g + n);
  treat_values(v, mode, clip_c, oom, delta);
  for (int k = 0; k < n; ++k) g[k] = v[(size_t)k];
}

// The assignment of Eq. emd on an n x m cost matrix (n <= m): row_col[n].
int orc_assign(int n, int m, const double* cost, int* row_col) {
  if (n < 0 || m < n) return ORC_EINVAL;
  std::vector<double> cm(cost, cost + (size_t)n * m);
  std::vector<int> rc;
  assign_min_cost(n, m, cm, &rc);
  for (int i = 0; i < n; ++i) row_col[i] = rc[i];
  return ORC_OK;
}

// Particles of the surface observation of a packed state (pixel order).
int orc_surface_particles(const orc_config* c, int N, const double* state, int* out) {
  Sim<double> sim(*c, N);
  const int d = c->dim, sd = 2 * d + 2 * d * d;
  for (int q = 0; q < N; ++q) for (int a = 0; a < d; ++a) sim.x[q * 3 + a] = state[(size_t)q * sd + a];
  const std::vector<int> o = sim.surface_particles();
  for (size_t i = 0; i < o.size(); ++i) out[i] = o[i];
  return (int)o.size();
}

// Height map of Eq. hm and its pixel owners (particle index, -1 for an empty
// pixel) for the positions of a packed state.
int orc_heightmap(const orc_config* c, int N, const double* state, double* hm, int* owner) {
  Sim<double> sim(*c, N);
  const int d = c->dim, sd = 2 * d + 2 * d * d;
  for (int q = 0; q < N; ++q) for (int a = 0; a < d; ++a) sim.x[q * 3 + a] = state[(size_t)q * sd + a];
  const std::vector<int> o = sim.heightmap_owners();
  for (size_t i = 0; i < o.size(); ++i) { owner[i] = o[i]; hm[i] = o[i] >= 0 ? sim.x[o[i] * 3 + 1] : 0.0; }
  return (int)o.size();
}

// Skill actions for the paper's theta; jac (optional) = d action / d theta,
// [T][6][5].  Returns the number of actions, or -1 if more than max_T.
int orc_skill_actions(const double* theta, double v_l, double v_w, double dta, double d4, int unrounded,
                      int max_T, int* T_out, double* actions, double* jac) {
  Dual<5> th[5];
  for (int k = 0; k < 5; ++k) th[k] = Dual<5>::var(theta[k], k);
  std::vector<std::array<Dual<5>, 6>> acts;
  skill_actions(th, v_l, v_w, dta, d4, unrounded != 0, T_out, &acts);
  if ((int)acts.size() > max_T) return -1;
  for (size_t t = 0; t < acts.size(); ++t)
    for (int i = 0; i < 6; ++i) {
      actions[t * 6 + i] = acts[t][i].v;
      if (jac) for (int k = 0; k < 5; ++k) jac[(t * 6 + i) * 5 + k] = acts[t][i].d[k];
    }
  return (int)acts.size();
}

// Pose table [n_steps][8] = (tip xyz, psi, vel xyz, omega); jac [n_steps][8][5]
// with respect to the physical skill parameters sk = (depth, angle_deg, push,
// displace, push_angle_deg).
int orc_pose_table(const orc_config* c, const double* sk, double dt, int n_steps, double* out, double* jac) {
  std::vector<Pose<Dual<5>>> P;
  Dual<5> skd[5];
  for (int k = 0; k < 5; ++k) skd[k] = Dual<5>::var(sk[k], k);
  pose_table(*c, skd, dt, n_steps, &P);
  for (int n = 0; n < n_steps; ++n) {
    const Dual<5> e[8] = {P[n].tip[0], P[n].tip[1], P[n].tip[2], P[n].psi, P[n].vel[0], P[n].vel[1], P[n].vel[2], P[n].omega};
    for (int i = 0; i < 8; ++i) {
      out[n * 8 + i] = e[i].v;
      if (jac) for (int k = 0; k < 5; ++k) jac[(n * 8 + i) * 5 + k] = e[i].d[k];
    }
  }
  return ORC_OK;
}

int orc_svd(int d, const double* F, double* U, double* S, double* V) {
  double Fm[3][3] = {}, Um[3][3], Vm[3][3];
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) Fm[i][j] = F[i * d + j];
  svd(d, Fm, Um, S, Vm);
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) { U[i * d + j] = Um[i][j]; V[i * d + j] = Vm[i][j]; }
  return ORC_OK;
}

void orc_material(double E, double nu, double phi_deg, double cohesion, double* out4) {
  material(E, nu, phi_deg, cohesion, &out4[0], &out4[1], &out4[2], &out4[3]);
}

// Return map on singular values; returns the case (1, 2, 3).
int orc_return_map(int d, const double* s, double mu, double lam, double alpha, double kc, double* g, double* h) {
  int cs;
  return_map(d, s, mu, lam, alpha, kc, g, h, &cs);
  return cs;
}

// delta_gamma of Eq. DP (with the cohesion shift), for derivative pins.
double orc_delta_gamma(int d, const double* s, double mu, double lam, double alpha, double kc) {
  double eps[3], tr = 0, eh2 = 0;
  for (int i = 0; i < d; ++i) { eps[i] = std::log(s[i]); tr += eps[i]; }
  for (int i = 0; i < d; ++i) { const double e = eps[i] - tr / d; eh2 += e * e; }
  return std::sqrt(eh2) + (d * lam + 2 * mu) / (2 * mu) * tr * alpha - kc / (2 * mu);
}

// Constitutive update of one F_tmp (d x d, row-major) with one optional
// tangent direction (dFt, and d(E, nu, phi_deg)).  Returns the DP case, or -1
// if a singular value was clamped.
int orc_constitutive(int d, const double* Ft, double E, double nu, double phi_deg, double cohesion,
                     const double* dFt, const double* dpar, double* Fn, double* tau, double* dFn, double* dtau) {
  Dual<1> Fm[3][3], Fo[3][3], To[3][3];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    Fm[i][j] = Dual<1>(i < d && j < d ? Ft[i * d + j] : 0.0);
    if (dFt && i < d && j < d) Fm[i][j].d[0] = dFt[i * d + j];
  }
  Dual<1> Ed(E), nd(nu), pd(phi_deg);
  if (dpar) { Ed.d[0] = dpar[0]; nd.d[0] = dpar[1]; pd.d[0] = dpar[2]; }
  Dual<1> mu, lam, al, kc;
  material(Ed, nd, pd, cohesion, &mu, &lam, &al, &kc);
  int cs, ncl;
  constitutive(d, Fm, mu, lam, al, kc, Fo, To, &cs, &ncl);
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) {
    Fn[i * d + j] = Fo[i][j].v; tau[i * d + j] = To[i][j].v;
    if (dFn) dFn[i * d + j] = Fo[i][j].d[0];
    if (dtau) dtau[i * d + j] = To[i][j].d[0];
  }
  return ncl ? -1 : cs;
}

double orc_box_sdf(const orc_config* c, const double* tip, double psi, const double* x, double* n) {
  const Frame<double> f = shovel_frame(*c, tip, psi);
  return box_sdf(*c, f, x, n);
}

void orc_coulomb(const double* vs, const double* n, double mu_b, double* v) { coulomb(vs, n, mu_b, v); }

// Cell keys and the stable sort permutation.  base = floor(x n_grid - 1/2) per
// axis; tiles of `tile`^d cells; key = inst * n^d + tile_id * tile^d + cell in
// tile, tile_id and cell-in-tile lexicographic with the last axis fastest.
int orc_bin(int N, int d, int n_grid, int tile, const double* x, const int32_t* inst, uint32_t* keys,
            uint32_t* perm) {
  if (n_grid % tile) return ORC_EINVAL;
  const int nt = n_grid / tile;
  uint32_t cells = 1, tcells = 1;
  for (int a = 0; a < d; ++a) { cells *= n_grid; tcells *= tile; }
  for (int p = 0; p < N; ++p) {
    uint32_t t = 0, c = 0;
    for (int a = 0; a < d; ++a) {
      const int b = (int)std::floor(x[(size_t)p * d + a] * n_grid - 0.5);
      if (b < 0 || b + 2 >= n_grid) return ORC_EDOMAIN;
      t = t * nt + b / tile;
      c = c * tile + b % tile;
    }
    keys[p] = (inst ? (uint32_t)inst[p] : 0u) * cells + t * tcells + c;
  }
  std::vector<uint32_t> idx(N);
  std::iota(idx.begin(), idx.end(), 0u);
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return keys[a] < keys[b]; });
  for (int j = 0; j < N; ++j) perm[j] = idx[j];
  return ORC_OK;
}

}  // extern "C"
