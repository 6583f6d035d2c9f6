// Earth mover's distance of Eq. emd between the surface observation of the
// final state and a target point cloud, per instance, and its adjoint.
//
// Observation (Sec. III-A, "States and observations"): in each pixel of the
// height-map window the highest particle whose own (x, z) lies in it, ties to
// the lowest particle id; empty pixels give no point.  Points are taken in
// pixel order.
//
// Assignment: the injective map phi from the n observed points to the m >= n
// targets with the least sum of distances, by the Hungarian method with
// shortest augmenting paths (the oracle's algorithm), started from the row
// reduction: every point's potential is its distance to the nearest target and
// points take their nearest targets where free.  Each remaining point searches
// the targets on costs reduced by row and column potentials, one target per
// step, until it reaches a free target, then augments along the path and
// updates the potentials.  The result is a least-sum assignment, the oracle's
// one whenever the least sum is attained by a single assignment.  One workgroup per
// instance: a step updates the slack of every target in parallel (each thread
// keeps its targets' slack, potentials and positions in registers) and takes
// the least one with a workgroup reduction (ties to the lowest target, as the
// oracle).  A point's search finishes one target per step, so it ends within
// m + 1 steps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddm_kernels.hpp"
#include "ddm_state.hpp"

namespace ddm {
namespace {

constexpr int kEmdThreads = 1024;
constexpr int kEmdCols = kEmdMaxPoints / kEmdThreads;   // targets per thread
constexpr unsigned long long kNoOwner = ~0ull;

__device__ __forceinline__ unsigned long long dkey(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dval(unsigned long long k) {
  const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)u);
}

// Pixel of a particle's own (x, z), or -1 outside the window; the same
// arithmetic as the height map's first stencil point.
__device__ __forceinline__ int own_pixel(const KCfg& c, double x, double z) {
  const double fx = floor((x - c.hm_ox) / c.hm_pix), fz = floor((z - c.hm_oz) / c.hm_pix);
  if (!(fx >= 0.0 && fx < (double)c.hm_res && fz >= 0.0 && fz < (double)c.hm_res)) return -1;
  return (int)fx * c.hm_res + (int)fz;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_emd_max(KCfg c, Bufs b, const void* state, unsigned long long* top) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p - I.off >= I.n) return;
  const P<T, 3> st = pv<T, 3>(state, c.ntot);
  const int px = own_pixel(c, Pos<T>::real(st.xr(0, p)), Pos<T>::real(st.xr(2, p)));
  if (px < 0) return;
  atomicMax(&top[(int64_t)inst * c.hm_res * c.hm_res + px], dkey(Pos<T>::real(st.xr(1, p))));
}

// owner word = (particle id << 32) | slot, the lowest id among the highest
template <typename T>
__global__ void __launch_bounds__(kBlock) k_emd_owner(KCfg c, Bufs b, const void* state, const uint32_t* pid,
                                                      const unsigned long long* top, unsigned long long* own) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p - I.off >= I.n) return;
  const P<T, 3> st = pv<T, 3>(state, c.ntot);
  const int px = own_pixel(c, Pos<T>::real(st.xr(0, p)), Pos<T>::real(st.xr(2, p)));
  if (px < 0) return;
  const int64_t q = (int64_t)inst * c.hm_res * c.hm_res + px;
  if (top[q] == dkey(Pos<T>::real(st.xr(1, p))))
    atomicMin(&own[q], ((unsigned long long)pid[p] << 32) | (unsigned long long)(p - I.off));
}

__device__ __forceinline__ double dist3(const double* a, const double* b) {
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

// Least (value, index) over the workgroup, ties to the lower index.  The
// caller puts a barrier between this call and the next write to s_v / s_i.
__device__ __forceinline__ void block_argmin(double& val, int& idx, double* s_v, int* s_i) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double ov = __shfl_xor(val, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov < val || (ov == val && oi < idx)) { val = ov; idx = oi; }
  }
  if (lane == 0) { s_v[wid] = val; s_i[wid] = idx; }
  __syncthreads();
  val = s_v[0];
  idx = s_i[0];
  for (int w = 1; w < kEmdThreads / 64; ++w)
    if (s_v[w] < val || (s_v[w] == val && s_i[w] < idx)) { val = s_v[w]; idx = s_i[w]; }
}

template <typename T>
__global__ void __launch_bounds__(kEmdThreads) k_emd_assign(KCfg c, Bufs b, const void* state, EmdBufs E, int m) {
  const int inst = blockIdx.x;
  const int npix = c.hm_res * c.hm_res;
  const int64_t base = (int64_t)inst * npix;
  const InstDev& I = b.inst[inst];
  const P<T, 3> st = pv<T, 3>(state, c.ntot);
  double* obs = E.obs + base * 3;
  int* obs_slot = E.obs_slot + base;
  const double* tgt = E.target + base * 3;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kEmdThreads / 64;
  __shared__ int s_cnt[kEmdThreads / 64 + 1];
  __shared__ int s_n;
  __shared__ double s_v[kEmdThreads / 64];
  __shared__ int s_i[kEmdThreads / 64];
  __shared__ double s_u[kEmdMaxPoints + 1];    // row potentials, rows 1..n
  __shared__ short s_match[kEmdMaxPoints + 1]; // row of each target, 0 = free; target 0 is the search root
  __shared__ short s_from[kEmdMaxPoints + 1];  // previous target on the search tree
  __shared__ short s_near[kEmdMaxPoints + 1];  // nearest target of each point, 0 once matched at the start

  // 1. compaction of the observed pixels, in pixel order
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  for (int c0 = 0; c0 < npix; c0 += kEmdThreads) {
    const int i = c0 + threadIdx.x;
    const bool has = i < npix && E.own[base + i] != kNoOwner;
    const unsigned long long bal = __ballot(has);
    if (lane == 0) s_cnt[wid] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = s_n;
      for (int w = 0; w < nw; ++w) { const int t = s_cnt[w]; s_cnt[w] = acc; acc += t; }
      s_cnt[nw] = acc;
    }
    __syncthreads();
    if (has) {
      const int k = s_cnt[wid] + __popcll(bal & ((1ull << lane) - 1ull));
      const int slot = (int)(E.own[base + i] & 0xFFFFFFFFull);
      const int64_t p = I.off + slot;
      obs[k * 3 + 0] = Pos<T>::real(st.xr(0, p));
      obs[k * 3 + 1] = Pos<T>::real(st.xr(1, p));
      obs[k * 3 + 2] = Pos<T>::real(st.xr(2, p));
      obs_slot[k] = slot;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_n = s_cnt[nw];
    __syncthreads();
  }
  const int n = s_n;
  if (n == 0 || n > m) {
    if (threadIdx.x == 0) {
      E.n_obs[inst] = 0;
      E.emd[inst] = 0.0;
      if (n > m) atomicOr(&b.err->flags, 8u);
    }
    return;
  }

  // 2. shortest augmenting paths, one point (row) at a time.  Each thread owns
  // the targets j = tid + 1 + k * kEmdThreads (k < kEmdCols): their slack,
  // potential, search mark and position stay in its registers; the row
  // potentials, the matching and the search tree are in LDS.
  double tj[kEmdCols][3], vj[kEmdCols], sl[kEmdCols];
  bool dn[kEmdCols];
#pragma unroll
  for (int k = 0; k < kEmdCols; ++k) {
    const int j = threadIdx.x + 1 + k * kEmdThreads;
    vj[k] = 0.0;
    for (int a = 0; a < 3; ++a) tj[k][a] = j <= m ? tgt[(j - 1) * 3 + a] : 0.0;
  }
  for (int j = threadIdx.x; j <= m; j += kEmdThreads) s_match[j] = 0;
  // start: u_i = the distance to the nearest target (a wave per point, ties to
  // the lowest target), which keeps every reduced cost non-negative; a point
  // whose nearest target is still free takes it (a tight pair), in point order
  for (int i = wid + 1; i <= n; i += nw) {
    double best = __builtin_inf();
    int bj = 0x7FFFFFFF;
    for (int j = lane + 1; j <= m; j += 64) {
      const double d = dist3(obs + (i - 1) * 3, tgt + (j - 1) * 3);
      if (d < best) { best = d; bj = j; }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oj = __shfl_xor(bj, o, 64);
      if (ov < best || (ov == best && oj < bj)) { best = ov; bj = oj; }
    }
    if (lane == 0) { s_u[i] = best; s_near[i] = (short)bj; }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i <= n; ++i) {
      const int j = s_near[i];
      if (s_match[j] == 0) { s_match[j] = (short)i; s_near[i] = 0; }   // s_near 0: matched
    }
  }
  __syncthreads();
  for (int row = 1; row <= n; ++row) {
    if (s_near[row] == 0) continue;        // matched at the start (uniform over the group)
#pragma unroll
    for (int k = 0; k < kEmdCols; ++k) { sl[k] = __builtin_inf(); dn[k] = false; }
    if (threadIdx.x == 0) s_match[0] = (short)row;
    __syncthreads();
    int j0 = 0;
    for (int step = 0; step <= m; ++step) {
      const int i0 = s_match[j0];
      const double ui = s_u[i0];
      const double xi[3] = {obs[(i0 - 1) * 3 + 0], obs[(i0 - 1) * 3 + 1], obs[(i0 - 1) * 3 + 2]};
      double best = __builtin_inf();
      int bj = 0x7FFFFFFF;
#pragma unroll
      for (int k = 0; k < kEmdCols; ++k) {
        const int j = threadIdx.x + 1 + k * kEmdThreads;
        if (j > m || dn[k]) continue;
        const double red = dist3(xi, tj[k]) - ui - vj[k];
        if (red < sl[k]) { sl[k] = red; s_from[j] = (short)j0; }
        if (sl[k] < best) { best = sl[k]; bj = j; }
      }
      block_argmin(best, bj, s_v, s_i);
      if (bj > m) break;                  // no finite slack: non-finite positions (uniform over the group)
      const double delta = best;
      if (threadIdx.x == 0) s_u[s_match[0]] += delta;   // the root column 0
#pragma unroll
      for (int k = 0; k < kEmdCols; ++k) {
        const int j = threadIdx.x + 1 + k * kEmdThreads;
        if (j > m) continue;
        if (dn[k]) { s_u[s_match[j]] += delta; vj[k] -= delta; }
        else sl[k] -= delta;
      }
      // the reached target joins the search tree
#pragma unroll
      for (int k = 0; k < kEmdCols; ++k)
        if (threadIdx.x + 1 + k * kEmdThreads == bj) dn[k] = true;
      __syncthreads();
      j0 = bj;
      if (s_match[j0] == 0) break;        // a free target: the path is complete
    }
    // every thread takes the outcome before thread 0 rewrites the matching
    const bool failed = j0 > m || s_match[j0] != 0;   // the search ended without a free target
    __syncthreads();
    if (failed) {
      if (threadIdx.x == 0) { atomicOr(&b.err->flags, 8u); E.n_obs[inst] = 0; E.emd[inst] = 0.0; }
      return;
    }
    // augment along the path back to the root
    if (threadIdx.x == 0) {
      while (j0) { const int j1 = s_from[j0]; s_match[j0] = s_match[j1]; j0 = j1; }
    }
    __syncthreads();
  }

  // 3. the assignment and the distance under it
  for (int j = threadIdx.x + 1; j <= m; j += kEmdThreads)
    if (s_match[j]) E.assign[base + s_match[j] - 1] = j - 1;
  __syncthreads();
  double sum = 0.0;
  for (int i = threadIdx.x; i < n; i += kEmdThreads) sum += dist3(obs + i * 3, tgt + E.assign[base + i] * 3);
  for (int o = 1; o < 64; o <<= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) s_v[wid] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += s_v[w];
    E.emd[inst] = s;
    E.n_obs[inst] = n;
  }
}

// loss[inst] += w_emd * EMD
__global__ void k_emd_add(int n_inst, double w, const double* emd, double* loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_inst) loss[i] += w * emd[i];
}

// Adjoint: d EMD / d x_p = (x_p - t_phi) / |x_p - t_phi| for the owner of
// each observed point (the assignment and the owner choice carry none); a
// particle owns at most one pixel of the observation.
template <typename T>
__global__ void k_emd_seed(KCfg c, Bufs b, EmdBufs E, double w, void* adj) {
  const int inst = blockIdx.x;
  const int npix = c.hm_res * c.hm_res;
  const int64_t base = (int64_t)inst * npix;
  const InstDev& I = b.inst[inst];
  const Adj<T, 3> ad = av<T, 3>(adj, c.ntot);
  const int n = E.n_obs[inst];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double* xo = E.obs + (base + i) * 3;
    const double* t = E.target + (base + E.assign[base + i]) * 3;
    const double d = dist3(xo, t);
    if (!(d > 0.0)) continue;
    const int64_t p = I.off + E.obs_slot[base + i];
    for (int a = 0; a < 3; ++a) ad.x(a, p) += T(w * (xo[a] - t[a]) / d);
  }
}

}  // namespace

void launch_emd(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                const EmdBufs& E, int m, double w_emd, double* loss, hipStream_t s) {
  const int64_t words = (int64_t)c.n_inst * c.hm_res * c.hm_res;
  launch_fill_zero(E.top, words, 8, s);
  launch_fill_u32(E.own, words * 2, 0xFFFFFFFFu, s);
  if (prec == 0) {
    hipLaunchKernelGGL((k_emd_max<float>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, E.top);
    hipLaunchKernelGGL((k_emd_owner<float>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, E.top, E.own);
    hipLaunchKernelGGL((k_emd_assign<float>), dim3(c.n_inst), dim3(kEmdThreads), 0, s, c, b, state, E, m);
  } else {
    hipLaunchKernelGGL((k_emd_max<double>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, E.top);
    hipLaunchKernelGGL((k_emd_owner<double>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, E.top, E.own);
    hipLaunchKernelGGL((k_emd_assign<double>), dim3(c.n_inst), dim3(kEmdThreads), 0, s, c, b, state, E, m);
  }
  hipLaunchKernelGGL(k_emd_add, dim3((c.n_inst + 255) / 256), dim3(256), 0, s, c.n_inst, w_emd, E.emd, loss);
}

void launch_emd_seed(int prec, const KCfg& c, const Bufs& b, const EmdBufs& E, double w_emd, void* adj,
                     hipStream_t s) {
  if (prec == 0) hipLaunchKernelGGL((k_emd_seed<float>), dim3(c.n_inst), dim3(kBlock), 0, s, c, b, E, w_emd, adj);
  else hipLaunchKernelGGL((k_emd_seed<double>), dim3(c.n_inst), dim3(kBlock), 0, s, c, b, E, w_emd, adj);
}

}  // namespace ddm
