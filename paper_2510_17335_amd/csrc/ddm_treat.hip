// Gradient treatments inside the reverse pass (Sec. III-E) and the statistics
// that show how the adjoints grow backwards in time (Appendix D, figure of the
// gradient scales of the key MLS-MPM variables).
//
// The adjoint of each key variable is one vector per instance: the particle
// positions, velocities and deformation gradients, the grid velocities after
// the grid update, and the grid momenta and masses that P2G produces.  The
// three treatments act on one such vector at a time:
//   clipping                element-wise into [-clip, clip];
//   order-of-magnitude      divide by 10^d + delta with d the rounded base-10
//     scaling               logarithm of the largest magnitude minus oom, when
//                           d > 0;
//   normalisation           divide by (2-norm + delta).
// The statistics of a vector are its largest and smallest element and its
// 2-norm, reduced per (instance, variable) into 64-bit accumulator words with
// global atomics: order-preserving keys of the maximum and of the maximum of
// the negated elements, and an FP64 sum of squares.  A NaN anywhere in a
// vector shows in its maximum (the keys order NaN above +inf).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddm_kernels.hpp"

namespace ddm {
namespace {

constexpr int kAccWords = 3;     // max key, max key of the negated values, sum of squares

__device__ __forceinline__ int64_t acc_index(int inst, int var, int phase) {
  return (((int64_t)inst * kTreatVars + var) * 2 + phase) * kAccWords;
}

// Total order of doubles as unsigned integers: negative values reversed, the
// sign bit set on the others.  0 is below every key a value can take.
__device__ __forceinline__ unsigned long long order_key(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)u);
}

// max that keeps a NaN of either side
__device__ __forceinline__ double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }

struct Stat {
  double mx, nmx, ss;   // max, max of the negated values, sum of squares
  __device__ Stat() : mx(-__builtin_inf()), nmx(-__builtin_inf()), ss(0.0) {}
  __device__ __forceinline__ void add(double v) {
    mx = nan_max(mx, v);
    nmx = nan_max(nmx, -v);
    ss += v * v;
  }
};

// Reduction over aligned groups of W lanes of a wave; the group's first lane
// adds the result to the accumulator words.
template <int W>
__device__ __forceinline__ void group_flush(Stat s, bool any, unsigned long long* a) {
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    s.mx = nan_max(s.mx, __shfl_xor(s.mx, o, 64));
    s.nmx = nan_max(s.nmx, __shfl_xor(s.nmx, o, 64));
    s.ss += __shfl_xor(s.ss, o, 64);
  }
  if (any && (threadIdx.x & (W - 1)) == 0) {
    atomicMax(a + 0, order_key(s.mx));
    atomicMax(a + 1, order_key(s.nmx));
    atomicAdd(reinterpret_cast<double*>(a + 2), s.ss);
  }
}

// Statistics of one accumulator: max, min and 2-norm of the vector, all zero
// for a vector without elements.
__device__ __forceinline__ void acc_stats(const unsigned long long* a, double& mx, double& mn, double& nrm) {
  if (a[0] == 0ull) { mx = mn = nrm = 0.0; return; }
  mx = key_value(a[0]);
  mn = -key_value(a[1]);
  nrm = sqrt(__longlong_as_double((long long)a[2]));
}

// C round(): halves away from zero.
__device__ __forceinline__ double round_half_away(double x) { return x < 0.0 ? -floor(-x + 0.5) : floor(x + 0.5); }

// Multiplier of a vector under scaling or normalisation (1 for clipping, whose
// action is element-wise, and for vectors the treatment leaves alone).
__device__ __forceinline__ double treat_factor(const Treat& t, const unsigned long long* a) {
  double mx, mn, nrm;
  acc_stats(a, mx, mn, nrm);
  if (t.mode == kTreatScale) {
    const double amax = nan_max(mx, -mn);
    if (!(amax > 0.0) || amax == __builtin_inf()) return 1.0;
    const double d = round_half_away(log10(amax)) - t.oom;
    return d > 0.0 ? 1.0 / (pow(10.0, d) + t.delta) : 1.0;
  }
  if (t.mode == kTreatNorm) {
    const double den = nrm + t.delta;
    return den > 0.0 && den == den ? 1.0 / den : 1.0;
  }
  return 1.0;
}

template <typename T>
__device__ __forceinline__ T treat_value(const Treat& t, T v, T f) {
  if (t.mode == kTreatClip) {
    const T c = T(t.clip);
    return v > c ? c : (v < -c ? -c : v);   // comparisons keep a NaN
  }
  return v * f;
}

// Particle variables: x rows [0, D), v rows [D, 2D), G = F - I rows
// [2D + D^2, 2D + 2D^2) of the adjoint state (the adjoint of G is that of F).
// Flat index r over the 2D + D^2 treated rows: state row r for r < 2D, else
// r + D^2 (the C rows are skipped).
template <int D> __device__ __forceinline__ int flat_row(int r) { return r < 2 * D ? r : r + D * D; }
template <int D> __device__ __forceinline__ int flat_var(int r) { return r < D ? 0 : (r < 2 * D ? 1 : 2); }

// One pass over the particle adjoints: statistics before the treatment
// (kPre), the treatment (kApply, with the factor reduced by an earlier kPre
// pass for scaling and normalisation), statistics after it (kPost).
constexpr int kPre = 1, kApply = 2, kPost = 4;

// Workgroup reduction of the 3 + 3 particle statistics, then one atomic per
// accumulator word; called by every thread of the workgroup.
__device__ void block_flush(Stat (&pre)[3], Stat (&post)[3], int what, unsigned long long* acc, int inst) {
  __shared__ double red[6][kBlock / 64][3];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    Stat s = q < 3 ? pre[q] : post[q - 3];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      s.mx = nan_max(s.mx, __shfl_xor(s.mx, o, 64));
      s.nmx = nan_max(s.nmx, __shfl_xor(s.nmx, o, 64));
      s.ss += __shfl_xor(s.ss, o, 64);
    }
    if (lane == 0) { red[q][wid][0] = s.mx; red[q][wid][1] = s.nmx; red[q][wid][2] = s.ss; }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    if ((what & (q < 3 ? kPre : kPost)) != 0) {
      Stat s;
      for (int w = 0; w < kBlock / 64; ++w) {
        s.mx = nan_max(s.mx, red[q][w][0]);
        s.nmx = nan_max(s.nmx, red[q][w][1]);
        s.ss += red[q][w][2];
      }
      unsigned long long* a = acc + acc_index(inst, q % 3, q < 3 ? 0 : 1);
      atomicMax(a + 0, order_key(s.mx));
      atomicMax(a + 1, order_key(s.nmx));
      atomicAdd(reinterpret_cast<double*>(a + 2), s.ss);
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 3; ++v) { pre[v] = Stat(); post[v] = Stat(); }
}

// A workgroup takes a contiguous range of particle blocks.  Instances own
// contiguous blocks, so the sums stay in registers and are flushed only when
// the instance changes.  All treated rows of a slot are loaded before any is
// stored, so their loads are in flight together.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_treat_particles(KCfg c, Bufs b, int nblk, T* __restrict__ adj, Treat t,
                                                            unsigned long long* acc, int what) {
  constexpr int NR = 2 * D + D * D;
  const int per = (nblk + gridDim.x - 1) / gridDim.x;
  const int b0 = blockIdx.x * per, b1 = min(nblk, b0 + per);
  Stat pre[3], post[3];
  T f[3] = {T(1), T(1), T(1)};
  int cur = -1;
  const bool stats = (what & (kPre | kPost)) != 0;
  for (int blk = b0; blk < b1; ++blk) {
    const int inst = b.blk_inst[blk];      // uniform over the workgroup
    if (inst != cur) {
      if (cur >= 0 && stats) block_flush(pre, post, what, acc, cur);
      cur = inst;
      if (what & kApply) {
#pragma unroll
        for (int v = 0; v < 3; ++v) f[v] = T(treat_factor(t, acc + acc_index(inst, v, 0)));
      }
    }
    const InstDev& I = b.inst[inst];
    const int64_t p = (int64_t)blk * kBlock + threadIdx.x;
    if (p - I.off < I.n) {                 // padding slots hold no particle
      T val[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) val[r] = adj[(int64_t)flat_row<D>(r) * c.ntot + p];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int v = flat_var<D>(r);
        if (what & kPre) pre[v].add((double)val[r]);
        if (what & kApply) val[r] = treat_value<T>(t, val[r], f[v]);
        if (what & kPost) post[v].add((double)val[r]);
      }
      if (what & kApply) {
#pragma unroll
        for (int r = 0; r < NR; ++r) adj[(int64_t)flat_row<D>(r) * c.ntot + p] = val[r];
      }
    }
  }
  if (cur >= 0 && stats) block_flush(pre, post, what, acc, cur);
}

// The same over the nodes of the listed active blocks of one grid buffer
// (every other node holds a zero adjoint): values 0 .. D-1 of a node form
// variable `var`, value 3 forms variable var + 1 when WM is set.  A
// group of 4^D lanes takes the nodes of one listed block per iteration and a
// contiguous share of the list; the list holds the blocks of an instance
// mostly together, so groups flush rarely.
template <typename T, int D, bool WM>
__global__ void __launch_bounds__(kBlock) k_treat_grid(KCfg c, Bufs b, const uint32_t* __restrict__ list,
                                                       const uint32_t* __restrict__ count, T* __restrict__ g, int var,
                                                       Treat t, unsigned long long* acc, int what) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t n = *count;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / NPB);
  const int64_t grp = (int64_t)blockIdx.x * (kBlock / NPB) + threadIdx.x / NPB;
  const int k = threadIdx.x % NPB;
  const int64_t per = (n + groups - 1) / groups;
  const int64_t e0 = grp * per, e1 = min(n, e0 + per);
  Stat pre[2], post[2];
  T f[2] = {T(1), T(1)};
  int cur = -1;
  constexpr int nv = WM ? 2 : 1;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < nv; ++q) {
      if (what & kPre) group_flush<NPB>(pre[q], true, acc + acc_index(cur, var + q, 0));
      if (what & kPost) group_flush<NPB>(post[q], true, acc + acc_index(cur, var + q, 1));
      pre[q] = Stat();
      post[q] = Stat();
    }
  };
  // four listed blocks per round: their list entries and node values are
  // loaded before any is processed
  constexpr int U = 4;
  for (int64_t e = e0; e < e1; e += U) {
    T val[U][4];
    T* nd[U];
    int ins[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ins[u] = -1;
      nd[u] = nullptr;
      if (e + u < e1) {
        int idx[3];
        int64_t node;
        active_node<D>(c, list[e + u], k, ins[u], idx, node);    // ins[u] is uniform over the group
        nd[u] = g + (b.inst[ins[u]].goff + node) * kNodeVals;
#pragma unroll
        for (int a = 0; a < 4; ++a) val[u][a] = nd[u][a];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ins[u] < 0) break;
      if (ins[u] != cur) {
        if (cur >= 0) flush();
        cur = ins[u];
        if (what & kApply) {
#pragma unroll
          for (int q = 0; q < nv; ++q) f[q] = T(treat_factor(t, acc + acc_index(cur, var + q, 0)));
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a >= D && a < 3) continue;
        const int q = a == 3 ? 1 : 0;
        if (q == 1 && !WM) continue;
        if (what & kPre) pre[q].add((double)val[u][a]);
        if (what & kApply) val[u][a] = treat_value<T>(t, val[u][a], f[q]);
        if (what & kPost) post[q].add((double)val[u][a]);
      }
      if (what & kApply) {
#pragma unroll
        for (int a = 0; a < 4; ++a) nd[u][a] = val[u][a];
      }
    }
  }
  if (cur >= 0 && (what & (kPre | kPost))) flush();
}

// out[inst][var][6] = max, min, 2-norm before the treatment, then after it
// (the values before it again when post == 0).
__global__ void k_treat_record(int n_inst, const unsigned long long* __restrict__ acc, int post, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst * kTreatVars) return;
  const int inst = i / kTreatVars, var = i % kTreatVars;
  double* o = out + (int64_t)i * 6;
  acc_stats(acc + acc_index(inst, var, 0), o[0], o[1], o[2]);
  acc_stats(acc + acc_index(inst, var, post ? 1 : 0), o[3], o[4], o[5]);
}

// Workgroups of the grid pass: about 8 listed blocks per group when every
// block is listed, at most 512.
unsigned grid_groups(const KCfg& c) {
  const int tshift = c.dim == 3 ? 6 : 4;
  const int64_t blocks = (c.nodes >> tshift) * c.n_inst;
  const int64_t per_wg = (int64_t)(kBlock >> tshift) * 8;
  const int64_t nb = (blocks + per_wg - 1) / per_wg;
  return (unsigned)(nb < 512 ? nb : 512);
}

}  // namespace

size_t treat_acc_words(int n_inst) { return (size_t)n_inst * kTreatVars * 2 * kAccWords; }

#define DDM_DISPATCH(PREC, DIM, KERNEL_CALL)                                  \
  do {                                                                        \
    if ((PREC) == 0) {                                                        \
      if ((DIM) == 3) { using T = float; constexpr int D = 3; KERNEL_CALL; }  \
      else { using T = float; constexpr int D = 2; KERNEL_CALL; }             \
    } else {                                                                  \
      if ((DIM) == 3) { using T = double; constexpr int D = 3; KERNEL_CALL; } \
      else { using T = double; constexpr int D = 2; KERNEL_CALL; }            \
    }                                                                         \
  } while (0)

namespace {

// Passes of one treatment: statistics before it for scaling and normalisation
// (their factor needs the whole vector), then one pass that treats and takes
// the remaining statistics.  Clipping and a bare record take one pass.
template <class Launch>
void treat_passes(const Treat& t, bool record, Launch launch) {
  const bool factor = t.mode == kTreatScale || t.mode == kTreatNorm;
  if (t.mode == kTreatNone) {
    if (record) launch(kPre);
    return;
  }
  if (factor) launch(kPre);
  launch(kApply | (record ? kPost : 0) | (!factor && record ? kPre : 0));
}

unsigned particle_groups(int nblk) { return (unsigned)(nblk < 2048 ? nblk : 2048); }

}  // namespace

void launch_treat_particles(int prec, const KCfg& c, const Bufs& b, int nblk, void* adj, const Treat& t, bool record,
                            unsigned long long* acc, hipStream_t s) {
  treat_passes(t, record, [&](int what) {
    DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_particles<T, D>), dim3(particle_groups(nblk)), dim3(kBlock),
                                                 0, s, c, b, nblk, (T*)adj, t, acc, what));
  });
}

void launch_treat_grid(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count, void* g,
                       int var, bool with_mass, const Treat& t, bool record, unsigned long long* acc, hipStream_t s) {
  treat_passes(t, record, [&](int what) {
    if (with_mass)
      DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_grid<T, D, true>), dim3(grid_groups(c)), dim3(kBlock), 0, s,
                                                   c, b, list, count, (T*)g, var, t, acc, what));
    else
      DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_grid<T, D, false>), dim3(grid_groups(c)), dim3(kBlock), 0,
                                                   s, c, b, list, count, (T*)g, var, t, acc, what));
  });
}

#undef DDM_DISPATCH

void launch_treat_record(int n_inst, const unsigned long long* acc, bool post, double* out, hipStream_t s) {
  const int n = n_inst * kTreatVars;
  hipLaunchKernelGGL(k_treat_record, dim3((n + 255) / 256), dim3(256), 0, s, n_inst, acc, post ? 1 : 0, out);
}

}  // namespace ddm
