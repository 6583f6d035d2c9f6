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
template <int D> __device__ __forceinline__ int var_row0(int v) { return v == 0 ? 0 : (v == 1 ? D : 2 * D + D * D); }
template <int D> __device__ __forceinline__ int var_rows(int v) { return v == 2 ? D * D : D; }

// One thread per padded slot, one workgroup per particle block (a block
// belongs to one instance, so a whole wave reduces into one accumulator).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_treat_stats_particles(KCfg c, Bufs b, const T* __restrict__ adj,
                                                                  unsigned long long* acc, int phase) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool live = p - I.off < I.n;
  const bool any = __any(live);
  if (!any) return;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    Stat s;
    if (live)
      for (int r = 0; r < var_rows<D>(v); ++r) s.add((double)adj[(int64_t)(var_row0<D>(v) + r) * c.ntot + p]);
    group_flush<64>(s, true, acc + acc_index(inst, v, phase));
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_treat_apply_particles(KCfg c, Bufs b, T* __restrict__ adj, Treat t,
                                                                  const unsigned long long* __restrict__ acc) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p - I.off >= I.n) return;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const T f = T(treat_factor(t, acc + acc_index(inst, v, 0)));
    for (int r = 0; r < var_rows<D>(v); ++r) {
      T& e = adj[(int64_t)(var_row0<D>(v) + r) * c.ntot + p];
      e = treat_value<T>(t, e, f);
    }
  }
}

// Grid vectors over the nodes of the listed active blocks (every other node
// holds a zero adjoint): values 0 .. D-1 of a node form variable `var`, value
// 3 forms variable var + 1 when with_mass is set.  Groups of 4^D lanes take
// the nodes of one block, hence of one instance.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_treat_stats_grid(KCfg c, Bufs b, const uint32_t* __restrict__ list,
                                                             const uint32_t* __restrict__ count,
                                                             const T* __restrict__ g, int var, int with_mass,
                                                             unsigned long long* acc, int phase) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = (int64_t)(*count) * NPB;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < items; base += (int64_t)gridDim.x * kBlock) {
    const int64_t it = base + threadIdx.x;
    const bool live = it < items;    // whole groups of NPB lanes, as items is a multiple of NPB
    Stat sv, sm;
    int inst = 0;
    if (live) {
      int idx[3];
      int64_t node;
      active_node<D>(c, list[it / NPB], (int)(it % NPB), inst, idx, node);
      const T* e = g + (b.inst[inst].goff + node) * kNodeVals;
#pragma unroll
      for (int a = 0; a < D; ++a) sv.add((double)e[a]);
      if (with_mass) sm.add((double)e[3]);
    }
    group_flush<NPB>(sv, live, acc + acc_index(inst, var, phase));
    if (with_mass) group_flush<NPB>(sm, live, acc + acc_index(inst, var + 1, phase));
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_treat_apply_grid(KCfg c, Bufs b, const uint32_t* __restrict__ list,
                                                             const uint32_t* __restrict__ count, T* __restrict__ g,
                                                             int var, int with_mass, Treat t,
                                                             const unsigned long long* __restrict__ acc) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = (int64_t)(*count) * NPB;
  for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < items; it += (int64_t)gridDim.x * kBlock) {
    int inst, idx[3];
    int64_t node;
    active_node<D>(c, list[it / NPB], (int)(it % NPB), inst, idx, node);
    T* e = g + (b.inst[inst].goff + node) * kNodeVals;
    const T f = T(treat_factor(t, acc + acc_index(inst, var, 0)));
#pragma unroll
    for (int a = 0; a < D; ++a) e[a] = treat_value<T>(t, e[a], f);
    if (with_mass) e[3] = treat_value<T>(t, e[3], T(treat_factor(t, acc + acc_index(inst, var + 1, 0))));
  }
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

unsigned grid_blocks(const KCfg& c) {
  const int tshift = c.dim == 3 ? 6 : 4;
  const int64_t items = ((c.nodes >> tshift) * c.n_inst) << tshift;
  const int64_t nb = (items + kBlock - 1) / kBlock;
  return (unsigned)(nb < 4096 ? nb : 4096);
}

}  // namespace

size_t treat_acc_words(int n_inst) { return (size_t)n_inst * kTreatVars * 2 * kAccWords; }

#define DDM_DISPATCH(PREC, DIM, KERNEL_CALL)                          \
  do {                                                                \
    if ((PREC) == 0) {                                                \
      if ((DIM) == 3) { using T = float; constexpr int D = 3; KERNEL_CALL; }  \
      else { using T = float; constexpr int D = 2; KERNEL_CALL; }             \
    } else {                                                          \
      if ((DIM) == 3) { using T = double; constexpr int D = 3; KERNEL_CALL; } \
      else { using T = double; constexpr int D = 2; KERNEL_CALL; }            \
    }                                                                 \
  } while (0)

void launch_treat_stats_particles(int prec, const KCfg& c, const Bufs& b, int nblk, const void* adj,
                                  unsigned long long* acc, int phase, hipStream_t s) {
  DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_stats_particles<T, D>), dim3(nblk), dim3(kBlock), 0, s, c, b,
                                               (const T*)adj, acc, phase));
}

void launch_treat_apply_particles(int prec, const KCfg& c, const Bufs& b, int nblk, void* adj, const Treat& t,
                                  const unsigned long long* acc, hipStream_t s) {
  DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_apply_particles<T, D>), dim3(nblk), dim3(kBlock), 0, s, c, b,
                                               (T*)adj, t, acc));
}

void launch_treat_stats_grid(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count,
                             const void* g, int var, bool with_mass, unsigned long long* acc, int phase, hipStream_t s) {
  DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_stats_grid<T, D>), dim3(grid_blocks(c)), dim3(kBlock), 0, s,
                                               c, b, list, count, (const T*)g, var, with_mass ? 1 : 0, acc, phase));
}

void launch_treat_apply_grid(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count,
                             void* g, int var, bool with_mass, const Treat& t, const unsigned long long* acc,
                             hipStream_t s) {
  DDM_DISPATCH(prec, c.dim, hipLaunchKernelGGL((k_treat_apply_grid<T, D>), dim3(grid_blocks(c)), dim3(kBlock), 0, s,
                                               c, b, list, count, (T*)g, var, with_mass ? 1 : 0, t, acc));
}

#undef DDM_DISPATCH

void launch_treat_record(int n_inst, const unsigned long long* acc, bool post, double* out, hipStream_t s) {
  const int n = n_inst * kTreatVars;
  hipLaunchKernelGGL(k_treat_record, dim3((n + 255) / 256), dim3(256), 0, s, n_inst, acc, post ? 1 : 0, out);
}

}  // namespace ddm
