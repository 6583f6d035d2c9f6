// Earth mover's distance of Eq. emd between the surface observation of the
// final state and a target point cloud, per instance, and its adjoint.
//
// Observation (Sec. III-A, "States and observations"): in each pixel of the
// height-map window the highest particle whose own (x, z) lies in it, ties to
// the lowest particle id; empty pixels give no point.  Points are taken in
// pixel order.
//
// Assignment: the injective map phi from the n observed points to the m >= n
// targets with the least sum of distances, by the auction algorithm with
// epsilon scaling (Bertsekas).  The problem is made square with m - n dummy
// bidders that value every target at zero (they take the targets no point
// needs, so the square optimum is the injective one), which keeps epsilon
// scaling valid.  In each round every unassigned bidder bids for its best
// target (largest value - price) by raising that target's price by the gap to
// its second-best value plus epsilon; each target goes to its highest bidder
// (ties to the lowest bidder index) and its former owner becomes unassigned.
// When every bidder is assigned, epsilon shrinks and the round loop restarts
// with the prices kept.  The final assignment is within m * epsilon_min of the
// least sum.  One workgroup per instance runs the whole
// auction; a bound on the number of rounds makes every wave exit, and hitting
// it sets device error flag 16 (flag 8: more points than targets).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddm_kernels.hpp"
#include "ddm_state.hpp"

namespace ddm {
namespace {

constexpr int kEmdThreads = 1024;
constexpr int64_t kEmdMaxRounds = 200000;    // about a second of rounds
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

// Best and second-best value over one wave, with the index of the best.
__device__ __forceinline__ void wave_top2(double& b1, int& j1, double& b2) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double ob1 = __shfl_xor(b1, o, 64), ob2 = __shfl_xor(b2, o, 64);
    const int oj = __shfl_xor(j1, o, 64);
    const bool take = ob1 > b1 || (ob1 == b1 && oj < j1);
    const double lo = take ? b1 : ob1;
    b2 = fmax(lo, fmax(b2, ob2));
    if (take) { b1 = ob1; j1 = oj; }
  }
}

__device__ __forceinline__ double dist3(const double* a, const double* b) {
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

template <typename T>
__global__ void __launch_bounds__(kEmdThreads) k_emd_auction(KCfg c, Bufs b, const void* state, EmdBufs E, int m,
                                                             double eps_rel) {
  const int inst = blockIdx.x;
  const int npix = c.hm_res * c.hm_res;
  const int64_t base = (int64_t)inst * npix;
  const InstDev& I = b.inst[inst];
  const P<T, 3> st = pv<T, 3>(state, c.ntot);
  double* obs = E.obs + base * 3;
  int* obs_slot = E.obs_slot + base;
  const double* tgt = E.target + base * 3;
  double* price = E.price + base;
  int* owner = E.obj_owner + base;
  int* assign = E.assign + base;
  unsigned long long* bmax = E.bid_max + base;
  int* bwin = E.bid_win + base;
  double* bval = E.bid_val + base;
  int* bobj = E.bid_obj + base;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kEmdThreads / 64;
  __shared__ int s_cnt[kEmdThreads / 64 + 1];
  __shared__ int s_n, s_unassigned, s_flag;
  __shared__ double s_red[kEmdThreads / 64];
  __shared__ double s_lo[kEmdThreads / 64][3], s_hi[kEmdThreads / 64][3];

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
      E.n_obs[inst] = n > m ? 0 : n;
      E.emd[inst] = 0.0;
      if (n > m) atomicOr(&b.err->flags, 8u);
    }
    return;
  }

  // 2. epsilon schedule from the extent of the two point sets
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = threadIdx.x; i < n + m; i += kEmdThreads) {
    const double* q = i < n ? obs + i * 3 : tgt + (i - n) * 3;
    for (int a = 0; a < 3; ++a) { lo[a] = fmin(lo[a], q[a]); hi[a] = fmax(hi[a], q[a]); }
  }
  for (int a = 0; a < 3; ++a) {
    double l = lo[a], h = hi[a];
    for (int o = 1; o < 64; o <<= 1) { l = fmin(l, __shfl_xor(l, o, 64)); h = fmax(h, __shfl_xor(h, o, 64)); }
    if (lane == 0) { s_lo[wid][a] = l; s_hi[wid][a] = h; }
  }
  __syncthreads();
  double C = 0.0;
  for (int a = 0; a < 3; ++a) {
    double l = 1e300, h = -1e300;
    for (int w = 0; w < nw; ++w) { l = fmin(l, s_lo[w][a]); h = fmax(h, s_hi[w][a]); }
    C += (h - l) * (h - l);               // n + m >= 2 points, so h >= l
  }
  C = sqrt(C) + 1e-300;                   // the largest distance is at most the diagonal
  const double eps_min = C * eps_rel;
  double eps = C * 0.25;

  for (int j = threadIdx.x; j < m; j += kEmdThreads) { price[j] = 0.0; bmax[j] = 0ull; bwin[j] = 0x7FFFFFFF; }
  if (threadIdx.x == 0) s_flag = 0;
  __syncthreads();
  int64_t rounds = 0;
  for (;;) {
    // a phase: every point starts unassigned, prices are kept
    for (int j = threadIdx.x; j < m; j += kEmdThreads) owner[j] = -1;
    for (int i = threadIdx.x; i < m; i += kEmdThreads) assign[i] = -1;
    __syncthreads();
    for (;;) {
      if (threadIdx.x == 0) s_unassigned = 0;
      __syncthreads();
      // bids: a wave per unassigned bidder (points i < n, dummies above),
      // lanes over the targets
      int mine = 0;
      for (int i = wid; i < m; i += nw) {
        if (assign[i] >= 0) continue;      // uniform over the wave
        ++mine;
        const double* xi = obs + (i < n ? i : 0) * 3;
        double b1 = -1e300, b2 = -1e300;
        int j1 = 0x7FFFFFFF;
        for (int j = lane; j < m; j += 64) {
          const double v = (i < n ? -dist3(xi, tgt + j * 3) : 0.0) - price[j];
          if (v > b1) { b2 = b1; b1 = v; j1 = j; }
          else if (v > b2) b2 = v;
        }
        wave_top2(b1, j1, b2);
        const double gap = b2 > -1e299 ? b1 - b2 : C;
        const double bid = price[j1] + gap + eps;
        if (lane == 0) {
          bval[i] = bid;
          bobj[i] = j1;
          atomicMax(&bmax[j1], dkey(bid));
        }
      }
      if (lane == 0 && mine) atomicAdd(&s_unassigned, mine);
      __syncthreads();
      if (s_unassigned == 0) break;
      // the highest bid for a target wins, ties to the lowest point index
      for (int i = threadIdx.x; i < m; i += kEmdThreads)
        if (assign[i] < 0 && dkey(bval[i]) == bmax[bobj[i]]) atomicMin(&bwin[bobj[i]], i);
      __syncthreads();
      for (int j = threadIdx.x; j < m; j += kEmdThreads) {
        const int w = bwin[j];
        if (w == 0x7FFFFFFF) continue;
        const int old = owner[j];
        if (old >= 0) assign[old] = -1;
        owner[j] = w;
        assign[w] = j;
        price[j] = dval(bmax[j]);
        bmax[j] = 0ull;
        bwin[j] = 0x7FFFFFFF;
      }
      __syncthreads();
      if (++rounds > kEmdMaxRounds) {
        if (threadIdx.x == 0) s_flag = 1;
        break;
      }
    }
    __syncthreads();
    if (s_flag || eps <= eps_min) break;
    eps = fmax(eps * 0.2, eps_min);
  }
  if (s_flag) {
    if (threadIdx.x == 0) { atomicOr(&b.err->flags, 16u); E.n_obs[inst] = 0; E.emd[inst] = 0.0; }
    return;
  }
  // 3. the distance under the assignment
  double sum = 0.0;
  for (int i = threadIdx.x; i < n; i += kEmdThreads) sum += dist3(obs + i * 3, tgt + assign[i] * 3);
  for (int o = 1; o < 64; o <<= 1) sum += __shfl_xor(sum, o, 64);
  __syncthreads();
  if (lane == 0) s_red[wid] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += s_red[w];
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
    hipLaunchKernelGGL((k_emd_auction<float>), dim3(c.n_inst), dim3(kEmdThreads), 0, s, c, b, state, E, m, 1e-10);
  } else {
    hipLaunchKernelGGL((k_emd_max<double>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, E.top);
    hipLaunchKernelGGL((k_emd_owner<double>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, E.top, E.own);
    hipLaunchKernelGGL((k_emd_auction<double>), dim3(c.n_inst), dim3(kEmdThreads), 0, s, c, b, state, E, m, 1e-10);
  }
  hipLaunchKernelGGL(k_emd_add, dim3((c.n_inst + 255) / 256), dim3(256), 0, s, c.n_inst, w_emd, E.emd, loss);
}

void launch_emd_seed(int prec, const KCfg& c, const Bufs& b, const EmdBufs& E, double w_emd, void* adj,
                     hipStream_t s) {
  if (prec == 0) hipLaunchKernelGGL((k_emd_seed<float>), dim3(c.n_inst), dim3(kBlock), 0, s, c, b, E, w_emd, adj);
  else hipLaunchKernelGGL((k_emd_seed<double>), dim3(c.n_inst), dim3(kBlock), 0, s, c, b, E, w_emd, adj);
}

}  // namespace ddm
