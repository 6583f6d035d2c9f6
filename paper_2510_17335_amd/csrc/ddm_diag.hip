// Per-step diagnostics of a context's current state: particle mass,
// momentum and kinetic energy, the return-map case (Eq. DP) that each
// particle's next constitutive update takes and the singular values it would
// clamp, the CFL number, and the mass on the grid of the last sub-step's P2G.
// They read the state and grid and write nothing else, so they can run
// between any two calls.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddm_device.hpp"
#include "ddm_kernels.hpp"
#include "ddm_state.hpp"

namespace ddm {

namespace {

// Output row of one instance (the order of DDM_N_DIAG).
constexpr int kDiagSums = 9;         // mass, momentum[3], energy, cases[3], clamps: summed
constexpr int kDiagCfl = 9;          // maximum
constexpr int kDiagGridMass = 10;
constexpr int kDiagVals = 11;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One block of particles (one instance per block): sums reduced over the
// block, then added to the instance's row with one atomic per value; the CFL
// maximum through the bit pattern of a non-negative double, whose integer
// order is its numeric order.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_diag_particles(KCfg c, Bufs b, const void* state, double* out) {
  __shared__ double red[kBlock / 64][kDiagSums + 1];
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc[kDiagSums + 1];
#pragma unroll
  for (int k = 0; k <= kDiagSums; ++k) acc[k] = 0.0;
  if (p - I.off < I.n) {
    const P<T, D> st = pv<T, D>(state, c.ntot);
    const double mp = I.mp;
    double vmax = 0.0;
    acc[0] = mp;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double va = (double)st.v(a, p);
      acc[1 + a] = mp * va;
      acc[4] += 0.5 * mp * va * va;
      vmax = fmax(vmax, fabs(va));
    }
    acc[kDiagSums] = vmax * I.dt * c.inv_dx;
    // the next constitutive update: F_tmp = (I + dt C)(I + G), as P2G forms it
    const T dt = T(I.dt);
    T Cm[3][3], Gm[3][3], Ft[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) { Cm[a][bb] = T(0); Gm[a][bb] = T(0); Ft[a][bb] = T(0); }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) { Cm[a][bb] = st.C(a, bb, p); Gm[a][bb] = st.G(a, bb, p); }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        T s = Cm[a][bb];
#pragma unroll
        for (int k = 0; k < D; ++k) s += Cm[a][k] * Gm[k][bb];
        Ft[a][bb] = Gm[a][bb] + dt * s;
      }
    Constit<T, D> cs;
    constit_forward<T, D>(Ft, T(I.mu), T(I.lam), T(I.alpha), T(I.kc), cs);
    acc[5] = cs.dp.cs == 1 ? 1.0 : 0.0;
    acc[6] = cs.dp.cs == 2 ? 1.0 : 0.0;
    acc[7] = cs.dp.cs == 3 ? 1.0 : 0.0;
    acc[8] = (double)cs.nclamp;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagSums; ++k) {
    const double s = wave_sum_d(acc[k]);
    if (lane == 0) red[wid][k] = s;
  }
  const double m = wave_max_d(acc[kDiagSums]);
  if (lane == 0) red[wid][kDiagSums] = m;
  __syncthreads();
  double* row = out + (int64_t)inst * kDiagVals;
  if (threadIdx.x < kDiagSums) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    if (s != 0.0) atomicAdd(row + threadIdx.x, s);
  } else if (threadIdx.x == kDiagSums) {
    double mx = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) mx = fmax(mx, red[w][kDiagSums]);
    atomicMax(reinterpret_cast<unsigned long long*>(row + kDiagCfl), (unsigned long long)__double_as_longlong(mx));
  }
}

// Nodal masses of the last sub-step over its active blocks, per instance; a
// lane adds its own node when the lanes of its wave do not share one instance.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_diag_grid(KCfg c, Bufs b, const T* __restrict__ pre, ActiveSet act,
                                                      double* out) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = pre ? (int64_t)(*act.count) * NPB : 0;
  if (!pre) {
    // no grid since the last init, set_state or backward
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < c.n_inst) out[(int64_t)i * kDiagVals + kDiagGridMass] = __longlong_as_double(0x7FF8000000000000ll);
    return;
  }
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < items; base += (int64_t)gridDim.x * kBlock) {
    const int64_t it = base + threadIdx.x;
    int inst = -1;
    double m = 0.0;
    if (it < items) {
      int idx[3];
      int64_t node;
      active_node<D>(c, act.list[it / NPB], (int)(it % NPB), inst, idx, node);
      m = (double)pre[(b.inst[inst].goff + node) * kNodeVals + 3];
    }
    const int first = __shfl(inst, 0, 64);
    if (__all(inst == first || inst < 0)) {
      const double s = wave_sum_d(m);
      if ((threadIdx.x & 63) == 0 && first >= 0 && s != 0.0) atomicAdd(out + (int64_t)first * kDiagVals + kDiagGridMass, s);
    } else if (inst >= 0 && m != 0.0) {
      atomicAdd(out + (int64_t)inst * kDiagVals + kDiagGridMass, m);
    }
  }
}

}  // namespace

void launch_diagnostics(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const void* grid_pre,
                        const ActiveSet& act, double* out, hipStream_t s) {
  launch_fill_zero(out, (int64_t)c.n_inst * kDiagVals, 8, s);
  const int64_t npb = c.dim == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t total_blocks = c.nodes / npb * c.n_inst;
  const unsigned ng = grid_pre ? (unsigned)std::min<int64_t>(4096, (total_blocks * npb + kBlock - 1) / kBlock)
                               : (unsigned)((c.n_inst + kBlock - 1) / kBlock);
#define DDM_DIAG(T, DD)                                                                                  \
  hipLaunchKernelGGL((k_diag_particles<T, DD>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, out);     \
  hipLaunchKernelGGL((k_diag_grid<T, DD>), dim3(ng), dim3(kBlock), 0, s, c, b, (const T*)grid_pre, act, out)
  if (prec == 0) {
    if (c.dim == 3) { DDM_DIAG(float, 3); } else { DDM_DIAG(float, 2); }
  } else {
    if (c.dim == 3) { DDM_DIAG(double, 3); } else { DDM_DIAG(double, 2); }
  }
#undef DDM_DIAG
}

}  // namespace ddm
