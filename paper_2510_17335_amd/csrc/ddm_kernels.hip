// HIP kernels of the MLS-MPM sub-step (Algorithm 1 of the paper), the loss
// (Eq. hm plus the scoop-mass term) and the adjoint of each sub-step
// (Eq. po/pa), for gfx950 wave64.
//
// Layout: particle state in structure-of-arrays, component-major with stride
// ntot: x[D], v[D], C[D*D], G[D*D] with G = F - I (row-major matrices).  In
// FP32 the positions are unsigned 32-bit fixed point (x = value * 2^-32), in
// FP64 doubles.  Instances occupy
// consecutive ranges padded to kBlock slots, so every 256-thread block belongs
// to one instance (blk_inst).  Grid: per instance n^D nodes, x-major, each
// node a 4-vector (mv0, mv1, mv2, m) before the grid update and (v0, v1, v2, m)
// after it.
#include <hip/hip_runtime.h>

#include <cstring>

#include "ddm_device.hpp"
#include "ddm_kernels.hpp"
#include "ddm_state.hpp"

namespace ddm {

__device__ __forceinline__ void flag_error(DevErr* e, unsigned int bit, int inst) {
  const unsigned int old = atomicOr(&e->flags, bit);
  if (old == 0) atomicExch(&e->first_inst, (unsigned int)inst);
}

// Tiles of a tile kernel.  Without a queue, workgroup b takes tiles b, b +
// gridDim.x, ... (one each when the grid has a workgroup per tile).  With one
// (a persistent launch of fewer workgroups), thread 0 claims the next tile
// from the queue's counter, so a workgroup that finishes early takes the next
// tile without a new dispatch and the load balances itself; the workgroup
// that finishes last resets the counters for the next launch.  Every call
// is reached by the whole workgroup; the loop body ends with a barrier, so the
// shared slot is read by all threads before thread 0 overwrites it.
// The claimed index is read back as a wave-uniform value, so that the tile's
// record and origin stay in scalar registers.
__device__ __forceinline__ uint32_t next_tile(const TileList& tl, uint32_t t, uint32_t* slot) {
  if (!tl.queue) return t + gridDim.x;
  if (threadIdx.x == 0) *slot = atomicAdd(tl.queue, 1u);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*slot);
}
__device__ __forceinline__ uint32_t first_tile(const TileList& tl, uint32_t* slot) {
  if (!tl.queue) return blockIdx.x;
  if (threadIdx.x == 0) *slot = atomicAdd(tl.queue, 1u);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*slot);
}
__device__ __forceinline__ void finish_tiles(const TileList& tl) {
  if (!tl.queue || threadIdx.x != 0) return;
  __threadfence();
  if (atomicAdd(tl.queue + 1, 1u) == gridDim.x - 1) {
    tl.queue[0] = 0u;
    tl.queue[1] = 0u;
    __threadfence();
  }
}

// Stencil of one particle: base node, fractional offset, weights and their
// derivatives per axis.  Returns false (and flags) when a node would fall
// outside [0, n).
template <typename T, int D> struct Stencil {
  int base[3];
  T w[3][3], dw[3][3], f[3];
};

template <typename T, int D>
__device__ __forceinline__ bool make_stencil(const P<T, D>& st, int64_t p, const KCfg& c, Stencil<T, D>& S) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (!Pos<T>::cell(st.xr(a, p), c, S.base[a], S.f[a])) return false;
    bspline(S.f[a], S.w[a], S.dw[a]);
  }
  return true;
}

template <int D>
__device__ __forceinline__ int64_t node_of(const int base[3], int o0, int o1, int o2, int n) {
  return D == 2 ? (int64_t)(base[0] + o0) * n + (base[1] + o1)
                : ((int64_t)(base[0] + o0) * n + (base[1] + o1)) * n + (base[2] + o2);
}

template <typename T> __device__ __forceinline__ T ld(const void* p, int64_t i) { return static_cast<const T*>(p)[i]; }

// Row of entry (a, b) of a symmetric D x D matrix stored as its upper triangle.
template <int D> __device__ __forceinline__ int sym_row(int a, int b) {
  const int i = a < b ? a : b, j = a < b ? b : a;
  return D == 3 ? (i == 0 ? j : (i == 1 ? 2 + j : 5)) : i + j;
}

// One grid node record (4 values) in one vector load: 16 B for float, two
// 16 B loads for double (node records are 4-element aligned).
template <typename T> struct Node4 { T v[4]; };
__device__ __forceinline__ Node4<float> ld_node(const float* p) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  return Node4<float>{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Node4<double> ld_node(const double* p) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  return Node4<double>{{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void st_node(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void st_node(double* p, double a, double b, double c, double d) {
  reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
  reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
}

// Wave64 + block reduction of one double, added atomically to *dst by one lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// With part (the deterministic mode's partials) the workgroup's sums go to
// part[blockIdx.x][k] instead, zeros included, for launch_det_finish.
template <int N>
__device__ __forceinline__ void block_accumulate(double (&v)[N], double* dst, double* part = nullptr) {
  __shared__ double red[kBlock / 64][N];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    if (part) part[(int64_t)blockIdx.x * kDetVals + threadIdx.x] = s;
    else if (s != 0.0) atomicAdd(&dst[threadIdx.x], s);
  }
}

// Fixed-order sum of one instance's partials (one workgroup per instance):
// thread t sums a contiguous run of blocks, the runs are combined by the wave
// butterfly and then wave by wave; the partials read are zeroed.
__global__ void __launch_bounds__(kBlock) k_det_finish(KCfg c, Bufs b, int grid_blocks, int nvals, double* dst,
                                                       int64_t stride) {
  __shared__ double red[kBlock / 64][kDetVals];
  const int inst = blockIdx.x;
  int64_t b0, b1;
  if (grid_blocks) {
    const int64_t per = (int64_t)1 << (c.dim * (c.nlog2 - 2));
    b0 = inst * per;
    b1 = b0 + per;
  } else {
    const InstDev& I = b.inst[inst];
    b0 = I.off / kBlock;
    b1 = b0 + (I.n + kBlock - 1) / kBlock;
  }
  const int64_t chunk = (b1 - b0 + kBlock - 1) / kBlock;
  const int64_t lo = b0 + threadIdx.x * chunk, hi = min(b1, lo + chunk);
  double acc[kDetVals];
#pragma unroll
  for (int k = 0; k < kDetVals; ++k) acc[k] = 0.0;
  for (int64_t q = lo; q < hi; ++q) {
    double* row = b.dpart + q * kDetVals;
#pragma unroll
    for (int k = 0; k < kDetVals; ++k) {
      if (k < nvals) { acc[k] += row[k]; row[k] = 0.0; }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDetVals; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < nvals) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
    dst[(int64_t)inst * stride + threadIdx.x] += v;
  }
}

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------
// Fills with a 32-bit pattern (a kernel rather than a memset node, so that the
// sequence stays correct when it is captured into a graph and replayed).
__global__ void k_fill(uint32_t* p, int64_t words, uint32_t value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

void launch_fill_u32(void* p, int64_t words, uint32_t value, hipStream_t s) {
  if (words <= 0) return;
  int64_t blocks = (words + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(kBlock), 0, s, static_cast<uint32_t*>(p), words, value);
}

void launch_fill_zero(void* p, int64_t count, int elem_bytes, hipStream_t s) {
  launch_fill_u32(p, count * elem_bytes / 4, 0u, s);
}

// XO: write the position rows and the ids only (the other rows are not there).
template <typename T, int D, bool XO>
__global__ void k_init_state(KCfg c, Bufs b, const T* __restrict__ x0, void* state, uint32_t* pid) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t local = p - I.off;
  P<T, D> st = pv<T, D>(state, c.ntot);
  // x0 is the instance-concatenated, unpadded [n_total][D] array.
  int64_t src = 0;
  for (int k = 0; k < inst; ++k) src += b.inst[k].n;
  const bool live = local < I.n;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    st.xr(a, p) = Pos<T>::from_real(live ? (double)x0[(src + local) * D + a] : 0.5);
    if (XO) continue;
    st.v(a, p) = T(0);
#pragma unroll
    for (int bb = 0; bb < D; ++bb) { st.C(a, bb, p) = T(0); st.G(a, bb, p) = T(0); }
  }
  pid[p] = live ? (uint32_t)local : 0xFFFFFFFFu;
}

void launch_init_state(int prec, const KCfg& c, const Bufs& b, int nblk, const void* x0, void* state,
                       uint32_t* pid, hipStream_t s, bool positions_only) {
#define DDM_INIT(T, DD, XO) \
  hipLaunchKernelGGL((k_init_state<T, DD, XO>), dim3(nblk), dim3(kBlock), 0, s, c, b, (const T*)x0, state, pid)
  if (prec == 0) {
    if (c.dim == 3) { if (positions_only) DDM_INIT(float, 3, true); else DDM_INIT(float, 3, false); }
    else { if (positions_only) DDM_INIT(float, 2, true); else DDM_INIT(float, 2, false); }
  } else {
    if (c.dim == 3) { if (positions_only) DDM_INIT(double, 3, true); else DDM_INIT(double, 3, false); }
    else { if (positions_only) DDM_INIT(double, 2, true); else DDM_INIT(double, 2, false); }
  }
#undef DDM_INIT
}

// Copies a small host blob (passed by value as the kernel argument) to device memory.
struct Blob { uint32_t w[kBlobWords]; };
__global__ void k_put_blob(uint32_t* dst, Blob b, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = b.w[i];
}

void launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  Blob b;
  memset(&b, 0, sizeof(b));
  memcpy(b.w, src, bytes);
  hipLaunchKernelGGL(k_put_blob, dim3(1), dim3(64), 0, s, static_cast<uint32_t*>(dst), b, (int)((bytes + 3) / 4));
}

// ---------------------------------------------------------------------------
// P2G (Algorithm 1, deformation update to scatter): F_tmp = (I + dt C) F, i.e. G_tmp = G + dt C (I + G),
// SVD, return map, stress,
// then the quadratic B-spline scatter of mass and MLS-MPM momentum
// mv_i += w (m v + A (x_i - x_p)), A = -dt V_p (4/dx^2) tau + m C.
// ---------------------------------------------------------------------------
// Tile geometry: global tile id -> instance and the window origin (tile
// corner minus one cell, so particles that drifted by up to one cell since
// the last binning still fall inside the kWin^D node window).
template <int D>
__device__ __forceinline__ void tile_origin(const KCfg& c, uint32_t gt, int& inst, int org[3]) {
  const int nt = c.n / kTile;
  const uint32_t per = D == 3 ? (uint32_t)(nt * nt * nt) : (uint32_t)(nt * nt);
  inst = (int)(gt / per);
  uint32_t t = gt - (uint32_t)inst * per;
  org[2] = 0;
  for (int a = D - 1; a >= 0; --a) { org[a] = (int)(t % nt) * kTile - 1; t /= nt; }
}

// LDS window: component-major (one plane of `stride` entries per scattered
// value), x stride padded from kWin^2 to kWin^2 + 2 nodes.  Entries are
// double in every precision: on gfx950 an LDS float atomic add takes about
// 195 cycles per wave instruction per CU against about 10 for a double one
// (measured), and the sums gain precision.  The padding sets which lanes of
// a scatter instruction (same stencil node, different runs and planes) land
// on the same banks: with 2, P2G took 520 us per launch on the 64-instance
// batch against 525 with 4, and the G2P adjoint 499 against 500.5 (6 grows
// the G2P adjoint past 40 KB of LDS, three workgroups per CU, 588 us).
template <int D> struct Win {
  static constexpr int nodes = D == 3 ? kWin * kWin * kWin : kWin * kWin;
  static constexpr int xs = D == 3 ? kWin * kWin + 2 : kWin;
  static constexpr int stride = kWin * xs;
  static __device__ __forceinline__ int idx(int i, int j, int k) { return D == 3 ? i * xs + j * kWin + k : i * xs + j; }
  static __device__ __forceinline__ void coords(int n, int l[3]) {
    if (D == 3) { l[0] = n / (kWin * kWin); l[1] = (n / kWin) % kWin; l[2] = n % kWin; }
    else { l[0] = n / kWin; l[1] = n % kWin; l[2] = 0; }
  }
};

// Per-particle constitutive update and P2G contributions; emit(node offsets,
// weight, values) receives the D+1 scattered values of each stencil node.
template <typename T, int D>
__device__ __forceinline__ bool p2g_particle(const KCfg& c, const Bufs& b, const InstDev& I, int inst,
                                             const P<T, D>& si, const P<T, D>& so, int64_t p, Stencil<T, D>& S,
                                             T (&A)[3][3], T (&vel)[3], T* tau_out) {
  const T dt = T(I.dt), mp = T(I.mp);
  T Cm[3][3], Gm[3][3], Ft[3][3];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) { Cm[a][bb] = si.C(a, bb, p); Gm[a][bb] = si.G(a, bb, p); }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) {
      T acc = Cm[a][bb];
#pragma unroll
      for (int k = 0; k < D; ++k) acc += Cm[a][k] * Gm[k][bb];
      Ft[a][bb] = Gm[a][bb] + dt * acc;
    }
  T Fn[3][3], tau[3][3];
  const int nclamp = constit_step<T, D>(Ft, T(I.mu), T(I.lam), T(I.alpha), T(I.kc), Fn, tau);
  if (nclamp) { flag_error(b.err, 4u, inst); atomicAdd(&b.err->clamps, (unsigned long long)nclamp); }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) so.G(a, bb, p) = Fn[a][bb];
  if (tau_out) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = a; bb < D; ++bb) tau_out[(int64_t)sym_row<D>(a, bb) * c.ntot + p] = tau[a][bb];
  }
  const T k_str = -dt * T(I.Vp) * T(4.0 * c.inv_dx * c.inv_dx);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) A[a][bb] = k_str * tau[a][bb] + mp * Cm[a][bb];
#pragma unroll
  for (int a = 0; a < D; ++a) vel[a] = mp * si.v(a, p);
  if (!make_stencil<T, D>(si, p, c, S)) { flag_error(b.err, 2u, inst); return false; }
  return true;
}

// ---------------------------------------------------------------------------
// Run-based window scatter of one round of up to kBlock sorted particles.
// Phase 1 (the caller): thread t handles slot t of the round and leaves in
// LDS the particle's q (D values), B (D x D) and fractional position f, and
// wbase[t] = the window index of its stencil base (-1: nothing to scatter).
// Phase 2 (here): consecutive slots with the same base form a run (sorted
// particles of one cell); work items are (run, stencil row), a row being the
// 3 nodes along the last axis; each item sums its run's contributions in
// registers and adds them to the double LDS window once.  An LDS float atomic
// is slow on gfx950 (about 195 cycles per wave instruction, double about 10)
// and every atomic instruction costs the same whether 1 or 64 lanes are
// active, so the gain comes from issuing about 1/ppc as many atomics.
// ---------------------------------------------------------------------------
template <typename T> struct alignas(16) RunLDS {
  // group g of slot t (w_a^k: weight of offset k on axis a; w_a^1 = 1 - w_a^0 - w_a^2):
  //   0: q0 q1 q2 w_0^0   1: B00 B01 B02 w_0^2   2: B10 B11 B12 w_1^0
  //   3: B20 B21 B22 w_1^2   and w4: w_2^0 w_2^2
  // (kept small: the G2P adjoint fits 4 workgroups per CU at 40 KB of LDS)
  T rec[4][kBlock][4];
  T w4[kBlock][2];
  short wbase[kBlock];
  int wcount[kBlock / 64];
  unsigned short start[kBlock + 1];
};

template <typename T> __device__ __forceinline__ void st4(T* p, T a, T b, T c, T d) { p[0] = a; p[1] = b; p[2] = c; p[3] = d; }
template <> __device__ __forceinline__ void st4<float>(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
template <typename T> __device__ __forceinline__ void ld4(const T* p, T (&o)[4]) { o[0] = p[0]; o[1] = p[1]; o[2] = p[2]; o[3] = p[3]; }
template <> __device__ __forceinline__ void ld4<float>(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}

// Phase-1 record of slot t: q, B and the stencil weights w[axis][offset].
template <typename T, int D>
__device__ __forceinline__ void put_record(RunLDS<T>& L, int t, const T (&q)[3], const T (&B)[3][3], const T (&w)[3][3]) {
  st4<T>(L.rec[0][t], q[0], q[1], D == 3 ? q[2] : T(0), w[0][0]);
  st4<T>(L.rec[1][t], B[0][0], B[0][1], D == 3 ? B[0][2] : T(0), w[0][2]);
  st4<T>(L.rec[2][t], B[1][0], B[1][1], D == 3 ? B[1][2] : T(0), w[1][0]);
  if (D == 3) {
    st4<T>(L.rec[3][t], B[2][0], B[2][1], B[2][2], w[1][2]);
    L.w4[t][0] = w[2][0];
    L.w4[t][1] = w[2][2];
  } else {
    st4<T>(L.rec[3][t], T(0), T(0), T(0), w[1][2]);
  }
}

// Phase 2 for a round of rc slots whose records and wbase are in L (the
// caller synchronised after writing them).  NV = D + 1 scatters momentum and
// mass (mass per particle m); NV = D scatters a D-vector.  Work items cover
// NN = 3 or 9 nodes of a run's stencil: NN = 9 takes a plane (fixed offset o0
// in 3D, the whole stencil in 2D), NN = 3 a row along the last axis (fewer
// registers, more items, but each item reads the run's records again).  Both
// scatter kernels use planes: P2G ran 568 us per launch with rows and 516 with
// planes on the 64-instance workload.  Ends synchronised.
// NCOL = 1: every item adds to the window at once (LDS atomics in arbitrary
// order).  NCOL = 3^D (the deterministic mode, with particles binned before
// the sub-step so that a cell's particles form one run): pass k takes the runs
// whose base cell lies in residue class k (window coordinates modulo 3 per
// axis), whose 3^D stencils are disjoint, so that every node receives at most
// one addition per pass and the passes fix the order.
template <int D>
__device__ __forceinline__ int base_class(int wbase) {
  const int i = wbase / Win<D>::xs, r = wbase - i * Win<D>::xs;
  if (D == 2) return (i % 3) * 3 + r % 3;
  return ((i % 3) * 3 + (r / kWin) % 3) * 3 + (r % kWin) % 3;
}

template <typename T, int D, int NV, int NN, int NCOL>
__device__ void run_scatter_round(RunLDS<T>& L, int rc, double* win, T m) {
  constexpr int WS = Win<D>::stride;
  constexpr int NJ = NN / 3;                                  // rows per item
  constexpr int ITEMS = (D == 3 ? 9 : 3) / NJ;                // items per run
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const bool flag = t < rc && L.wbase[t] >= 0 && (t == 0 || L.wbase[t] != L.wbase[t - 1]);
  const unsigned long long bal = __ballot(flag);
  if (lane == 0) L.wcount[wid] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) { off += w < wid ? L.wcount[w] : 0; tot += L.wcount[w]; }
  if (flag) L.start[off + __popcll(bal & ((1ull << lane) - 1ull))] = (unsigned short)t;
  if (t == 0) L.start[tot] = (unsigned short)rc;
  __syncthreads();
  for (int col = 0; col < NCOL; ++col) {
  for (int it = t; it < tot * ITEMS; it += kBlock) {
    const int r = it / ITEMS, sub = it - r * ITEMS;
    // the item's first row: 3D (o0, j0), 2D j0; rows j0 .. j0 + NJ - 1 along the middle axis
    const int o0 = D == 3 ? (NJ == 3 ? sub : sub / 3) : 0;
    const int j0 = NJ == 3 ? 0 : (D == 3 ? sub % 3 : sub);
    const int s0 = L.start[r], s1 = L.start[r + 1];
    const int base = L.wbase[s0];
    if (NCOL > 1 && base_class<D>(base) != col) continue;
    // acc[row j][node k][value]: 3D node (o0, j0 + j, k), 2D node (j0 + j, k)
    T acc[NJ][3][4];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[j][k][a] = T(0);
    for (int sl = s0; sl < s1; ++sl) {
      if (L.wbase[sl] != base) continue;            // a particle without a window record
      T g0[4], g1[4], g2[4], g3[4], g4[4] = {T(0), T(0), T(0), T(0)};
      ld4<T>(L.rec[0][sl], g0);
      ld4<T>(L.rec[1][sl], g1);
      ld4<T>(L.rec[2][sl], g2);
      ld4<T>(L.rec[3][sl], g3);
      if (D == 3) { g4[0] = L.w4[sl][0]; g4[1] = L.w4[sl][1]; }
      // per-axis weights
      const T wa[3] = {g0[3], T(1) - g0[3] - g1[3], g1[3]};
      const T wb[3] = {g2[3], T(1) - g2[3] - g3[3], g3[3]};
      const T wc[3] = {g4[0], T(1) - g4[0] - g4[1], g4[1]};
      // B columns (B row a is group a + 1)
      const T bc0[3] = {g1[0], g2[0], D == 3 ? g3[0] : T(0)};
      const T bc1[3] = {g1[1], g2[1], D == 3 ? g3[1] : T(0)};
      const T bc2[3] = {g1[2], g2[2], D == 3 ? g3[2] : T(0)};
      // 3D: inner axes 1 (j) and 2 (k) at fixed o0; 2D: axes 0 (j) and 1 (k)
      const T wo = D == 3 ? (o0 == 0 ? wa[0] : (o0 == 1 ? wa[1] : wa[2])) : T(1);
      const T(&wj)[3] = D == 3 ? wb : wa;
      const T(&wk)[3] = D == 3 ? wc : wb;
      const T(&bj)[3] = D == 3 ? bc1 : bc0;
      const T(&bk)[3] = D == 3 ? bc2 : bc1;
      T tj[3];
#pragma unroll
      for (int a = 0; a < D; ++a) tj[a] = g0[a] + (D == 3 ? T(o0) * bc0[a] : T(0)) + (NJ == 3 ? T(0) : T(j0) * bj[a]);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int jj = NJ == 3 ? j : j0;
        const T w1 = wo * (jj == 0 ? wj[0] : (jj == 1 ? wj[1] : wj[2]));
        T tk[3];
#pragma unroll
        for (int a = 0; a < D; ++a) tk[a] = tj[a];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T w = w1 * wk[k];
#pragma unroll
          for (int a = 0; a < D; ++a) { acc[j][k][a] += w * tk[a]; tk[a] += bk[a]; }
          if (NV == D + 1) acc[j][k][3] += w;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) tj[a] += bj[a];
      }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int jj = NJ == 3 ? j : j0;
        const int wi = base + (D == 3 ? Win<D>::idx(o0, jj, k) : Win<D>::idx(jj, k, 0));
#pragma unroll
        for (int a = 0; a < D; ++a) atomicAdd(win + a * WS + wi, (double)acc[j][k][a]);
        if (NV == D + 1) atomicAdd(win + 3 * WS + wi, (double)(acc[j][k][3] * m));
      }
  }
  if (NCOL > 1) __syncthreads();
  }
  __syncthreads();
}

// Adds the node blocks of a particle's stencil (nodes base .. base + 2 per
// axis) to the active set, each block once.
template <int D>
__device__ void mark_stencil_blocks(const KCfg& c, int inst, const int base[3], const ActiveSet& act) {
  const int nt = c.n / kTile;
  const uint32_t per = D == 3 ? (uint32_t)(nt * nt * nt) : (uint32_t)(nt * nt);
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) { lo[a] = base[a] / kTile; hi[a] = (base[a] + 2) / kTile; }
  for (int b0 = lo[0]; b0 <= hi[0]; ++b0)
    for (int b1 = lo[1]; b1 <= hi[1]; ++b1)
      for (int b2 = lo[2]; b2 <= hi[2]; ++b2) {
        const uint32_t gb = (uint32_t)inst * per +
                            (D == 3 ? (uint32_t)((b0 * nt + b1) * nt + b2) : (uint32_t)(b0 * nt + b1));
        if (atomicOr(&act.mask[gb], 1u) == 0u) act.list[atomicAdd(act.count, 1u)] = gb;
      }
}

// Quadratic B-spline scatter of one particle: node o = (o0, o1, o2) receives
// w_o (q + B o) (D values) and w_o m, w_o the product of the per-axis weights
// wt[axis][o_axis]; q + B o is advanced incrementally along the last axis.
template <typename T, int D, typename Emit>
__device__ __forceinline__ void scatter_stencil(const T (&wt)[3][3], const T (&q)[3], const T (&B)[3][3], T m,
                                                Emit&& emit) {
#pragma unroll
  for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
    for (int o1 = 0; o1 < 3; ++o1) {
      const T wxy = wt[0][o0] * wt[1][o1];
      T t[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int a = 0; a < D; ++a) t[a] = q[a] + T(o0) * B[a][0] + T(o1) * B[a][1];
#pragma unroll
      for (int o2 = 0; o2 < (D == 3 ? 3 : 1); ++o2) {
        const T w = D == 3 ? wxy * wt[2][o2] : wxy;
        T v[4] = {T(0), T(0), T(0), w * m};
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = w * t[a];
        emit(o0, o1, o2, v);
        if (D == 3) {
#pragma unroll
          for (int a = 0; a < D; ++a) t[a] += B[a][2];
        }
      }
    }
}

// P2G over occupied tiles: one workgroup per tile (grid-stride over the tile
// list), contributions accumulated with LDS atomics in a kWin^D window that is
// then stored whole to the tile's staging record (no global atomics); the
// grid update sums the windows covering each node.  Particles outside the
// window (drifted more than one cell since binning) add to the outlier grid
// with global atomics and put their node blocks in the active set.
template <typename T, int D, bool DET>
__global__ void __launch_bounds__(kBlock) k_p2g(KCfg c, Bufs b, TileList tl, const void* st_in, void* st_out,
                                                T* __restrict__ stg, T* __restrict__ gout, ActiveSet act,
                                                T* __restrict__ tau_out) {
  __shared__ double win[Win<D>::stride * kNodeVals];
  __shared__ RunLDS<T> rl;
  const uint32_t ntiles = *tl.count;
  const P<T, D> si = pv<T, D>(st_in, c.ntot), so = pv<T, D>(st_out, c.ntot);
  __shared__ uint32_t tile_slot;
  for (uint32_t t = first_tile(tl, &tile_slot); t < ntiles; t = next_tile(tl, t, &tile_slot)) {
    const TileRec tr = tl.list[t];
    int inst, org[3];
    tile_origin<D>(c, tr.tile, inst, org);
    const InstDev& I = b.inst[inst];
    T* g = gout + I.goff * kNodeVals;
    const T mpt = T(I.mp);
    for (int i = threadIdx.x; i < Win<D>::stride * kNodeVals; i += kBlock) win[i] = 0.0;
    const int cnt = (int)(tr.end - tr.start);
    for (int r0 = 0; r0 < cnt; r0 += kBlock) {
      const int rc = min(kBlock, cnt - r0);
      int wb = -1;
      if (threadIdx.x < rc) {
        const int64_t p = (int64_t)tr.start + r0 + threadIdx.x;
        Stencil<T, D> S;
        T A[3][3], vel[3];
        if (p2g_particle<T, D>(c, b, I, inst, si, so, p, S, A, vel, tau_out)) {
          // node o receives w_o (q + B o) and w_o m_p with q = m_p v - A f dx and
          // B = A dx (the MLS-MPM momentum m_p v + A (x_i - x_p), x_i - x_p = (o - f) dx)
          T q[3] = {T(0), T(0), T(0)}, B[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
          const T tdx = T(c.dx);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            T af = T(0);
#pragma unroll
            for (int bb = 0; bb < D; ++bb) { B[a][bb] = A[a][bb] * tdx; af += B[a][bb] * S.f[bb]; }
            q[a] = vel[a] - af;
          }
          int loc[3] = {0, 0, 0};
          bool inwin = true;
#pragma unroll
          for (int a = 0; a < D; ++a) { loc[a] = S.base[a] - org[a]; inwin &= loc[a] >= 0 && loc[a] <= kWin - 3; }
          if (inwin) {
            wb = Win<D>::idx(loc[0], loc[1], loc[2]);
            put_record<T, D>(rl, threadIdx.x, q, B, S.w);
          } else {
            mark_stencil_blocks<D>(c, inst, S.base, act);
            scatter_stencil<T, D>(S.w, q, B, mpt, [&](int o0, int o1, int o2, const T (&v)[4]) {
              T* dst = g + node_of<D>(S.base, o0, o1, o2, c.n) * kNodeVals;
#pragma unroll
              for (int a = 0; a < D; ++a) atomicAdd(dst + a, v[a]);
              atomicAdd(dst + 3, v[3]);
            });
          }
        }
      }
      rl.wbase[threadIdx.x] = wb;
      __syncthreads();
      run_scatter_round<T, D, D + 1, 9, DET ? (D == 3 ? 27 : 9) : 1>(rl, rc, win, mpt);
    }
    __syncthreads();
    // the whole window, zeros included, to the tile's staging record
    T* rec = stg + (int64_t)t * (kNodeVals * Win<D>::nodes);
    for (int i = threadIdx.x; i < Win<D>::nodes; i += kBlock) {
      int l[3];
      Win<D>::coords(i, l);
      const int wi = Win<D>::idx(l[0], l[1], l[2]);
      st_node(rec + (int64_t)i * kNodeVals, (T)win[wi], (T)win[Win<D>::stride + wi], (T)win[2 * Win<D>::stride + wi],
              (T)win[3 * Win<D>::stride + wi]);
    }
    __syncthreads();
  }
  finish_tiles(tl);
}

void launch_det_finish(const KCfg& c, const Bufs& b, bool grid_blocks, int nvals, double* dst, int64_t stride,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_det_finish, dim3(c.n_inst), dim3(kBlock), 0, s, c, b, grid_blocks ? 1 : 0, nvals, dst, stride);
}

void launch_p2g(int prec, const KCfg& c, const Bufs& b, const TileList& tl, int nwg, const void* st_in, void* st_out,
                const Staging& stg, void* gout, const ActiveSet& act, void* tau_out, hipStream_t s) {
#define DDM_P2G(T, DD)                                                                                             \
  if (c.det)                                                                                                       \
    hipLaunchKernelGGL((k_p2g<T, DD, true>), dim3(nwg), dim3(kBlock), 0, s, c, b, tl, st_in, st_out, (T*)stg.win,  \
                       (T*)gout, act, (T*)tau_out);                                                                \
  else                                                                                                             \
    hipLaunchKernelGGL((k_p2g<T, DD, false>), dim3(nwg), dim3(kBlock), 0, s, c, b, tl, st_in, st_out, (T*)stg.win, \
                       (T*)gout, act, (T*)tau_out)
  if (prec == 0) {
    if (c.dim == 3) { DDM_P2G(float, 3); } else { DDM_P2G(float, 2); }
  } else {
    if (c.dim == 3) { DDM_P2G(double, 3); } else { DDM_P2G(double, 2); }
  }
#undef DDM_P2G
}

// Blade pose of one sub-step (tip, angle, velocities) from the pose table.
template <typename T>
__device__ __forceinline__ Blade<T> load_blade(const void* poses, int inst, int max_steps, int step) {
  const T* q = static_cast<const T*>(poses) + ((int64_t)inst * max_steps + step) * kPoseVals;
  Blade<T> bl;
  bl.tip[0] = q[0]; bl.tip[1] = q[1]; bl.tip[2] = q[2]; bl.psi = q[3];
  bl.vel[0] = q[4]; bl.vel[1] = q[5]; bl.vel[2] = q[6]; bl.omega = q[7];
  bl.sp = q[8];           // sin and cos of the angle, evaluated once per sub-step on the host
  bl.cp = q[9];
  return bl;
}

template <typename T>
__device__ __forceinline__ void blade_velocity(const Blade<T>& bl, const T xi[3], T vs[3]) {
  // v_lin + omega x (x - tip), omega = (0, 0, -psi_dot)
  vs[0] = bl.vel[0] + bl.omega * (xi[1] - bl.tip[1]);
  vs[1] = bl.vel[1] - bl.omega * (xi[0] - bl.tip[0]);
  vs[2] = bl.vel[2];
}

// ---------------------------------------------------------------------------
// Grid update (Algorithm 1, agent move to grid collision): v = mv/m + dt g, shovel contact at the
// pose of this sub-step, then sticky walls.  Nodes without mass get v = 0.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void node_coords(int64_t node, int n, int idx[3]) {
  if (D == 2) { idx[0] = (int)(node / n); idx[1] = (int)(node % n); idx[2] = 0; }
  else { idx[0] = (int)(node / ((int64_t)n * n)); idx[1] = (int)((node / n) % n); idx[2] = (int)(node % n); }
}

// Sum of the staged windows covering a node: per axis the tiles (x + 1) / 4 - 1
// and (x + 1) / 4, whose windows start at 4t - 1.
template <typename T, int D>
__device__ __forceinline__ void gather_windows(const KCfg& c, int inst, const int idx[3], const T* __restrict__ stg,
                                               const uint32_t* __restrict__ tslot, T acc[4]) {
  const int nt = c.n / kTile;
  const uint32_t per = D == 3 ? (uint32_t)(nt * nt * nt) : (uint32_t)(nt * nt);
  int tt[3][2], ll[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int t1 = a < D ? (idx[a] + 1) >> 2 : 0;
    tt[a][0] = t1 - 1; tt[a][1] = t1;
    ll[a][0] = a < D ? idx[a] - kTile * (t1 - 1) + 1 : 0;
    ll[a][1] = a < D ? idx[a] - kTile * t1 + 1 : 0;
  }
#pragma unroll
  for (int j0 = 0; j0 < 2; ++j0)
#pragma unroll
    for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
      for (int j2 = 0; j2 < (D == 3 ? 2 : 1); ++j2) {
        const int q0 = tt[0][j0], q1 = tt[1][j1], q2 = D == 3 ? tt[2][j2] : 0;
        if (q0 < 0 || q0 >= nt || q1 < 0 || q1 >= nt || (D == 3 && (q2 < 0 || q2 >= nt))) continue;
        const uint32_t gt = (uint32_t)inst * per + (D == 3 ? (uint32_t)((q0 * nt + q1) * nt + q2) : (uint32_t)(q0 * nt + q1));
        const uint32_t r = tslot[gt];
        if (r == kNoSlot) continue;
        const int wn = D == 3 ? (ll[0][j0] * kWin + ll[1][j1]) * kWin + ll[2][j2] : ll[0][j0] * kWin + ll[1][j1];
        const Node4<T> v = ld_node(stg + ((int64_t)r * Win<D>::nodes + wn) * kNodeVals);
#pragma unroll
        for (int a = 0; a < kNodeVals; ++a) acc[a] += v.v[a];
      }
}

// Velocity of one node from its momentum and mass (acc = mv, m): v = mv/m + dt g,
// the shovel contact at the pose of sub-step `step`, the sticky walls; zero
// without mass.
template <typename T, int D>
__device__ __forceinline__ void node_velocity(const KCfg& c, const Bufs& b, int inst, int step, const int idx[3],
                                              const T (&acc)[4], T (&v)[3]) {
  const T m = acc[3];
  v[0] = v[1] = v[2] = T(0);
  if (m > T(0)) {
    const T dt = T(b.inst[inst].dt);
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = acc[a] / m;
    v[1] += dt * T(c.gravity);
    if (D == 3 && c.shovel) {
      const Blade<T> bl = load_blade<T>(b.poses, inst, c.max_steps, step);
      const T xi[3] = {T(idx[0]) * T(c.dx), T(idx[1]) * T(c.dx), T(idx[2]) * T(c.dx)};
      const T half[3] = {T(c.half[0]), T(c.half[1]), T(c.half[2])};
      SDF<T> f;
      sdf_eval<T>(bl, half, xi, f);
      if (f.phi < T(c.skin)) {
        T vs[3];
        blade_velocity<T>(bl, xi, vs);
        coulomb_forward<T>(vs, f.n, T(c.mu_b), v);
      }
    }
    bool wall = false;
#pragma unroll
    for (int a = 0; a < D; ++a) wall |= (idx[a] < c.bound) || (idx[a] >= c.n - c.bound);
    if (wall) v[0] = v[1] = v[2] = T(0);
  }
}

// pre_cap < 0: grid_pre is the dense grid (node gid at gid); pre_cap >= 0:
// grid_pre is a record of pre_cap node entries in the order of the active list
// (item it at it), and more items than that set error bit 4.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_grid_update(KCfg c, Bufs b, int step, const T* __restrict__ stg,
                                                        const uint32_t* __restrict__ tslot, T* __restrict__ gout,
                                                        ActiveSet act, T* __restrict__ pre, int64_t pre_cap,
                                                        T* __restrict__ post, uint32_t* __restrict__ list_out,
                                                        uint32_t* __restrict__ count_out) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const uint32_t nact = *act.count;
  if (count_out && blockIdx.x == 0 && threadIdx.x == 0) *count_out = nact;
  const int64_t items = (int64_t)nact * NPB;
  if (pre_cap >= 0 && items > pre_cap && blockIdx.x == 0 && threadIdx.x == 0) flag_error(b.err, 16u, 0);
  for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < items; it += (int64_t)gridDim.x * kBlock) {
    const uint32_t gb = act.list[it / NPB];
    const int k = (int)(it % NPB);
    if (list_out && k == 0) list_out[it / NPB] = gb;
    int inst, idx[3];
    int64_t node;
    active_node<D>(c, gb, k, inst, idx, node);
    const int64_t gid = b.inst[inst].goff + node;
    T acc[4] = {T(0), T(0), T(0), T(0)};
    gather_windows<T, D>(c, inst, idx, stg, tslot, acc);
    {
      // particles that left their windows: read and clear
      T* go = gout + gid * kNodeVals;
      const Node4<T> o = ld_node(go);
      if (o.v[3] != T(0) || o.v[0] != T(0) || o.v[1] != T(0) || o.v[2] != T(0)) {
#pragma unroll
        for (int a = 0; a < kNodeVals; ++a) { acc[a] += o.v[a]; go[a] = T(0); }
      }
    }
    T v[3];
    node_velocity<T, D>(c, b, inst, step, idx, acc, v);
    if (pre_cap < 0) st_node(pre + gid * kNodeVals, acc[0], acc[1], acc[2], acc[3]);
    else if (it < pre_cap) st_node(pre + it * kNodeVals, acc[0], acc[1], acc[2], acc[3]);
    post[gid * kNodeVals + 0] = v[0];
    post[gid * kNodeVals + 1] = v[1];
    post[gid * kNodeVals + 2] = v[2];
    post[gid * kNodeVals + 3] = acc[3];
  }
}

// The post-update grid of a sub-step again from the record of its pre-update
// grid (pre_cap entries in the order of the active list), over the sub-step's
// listed active blocks: the same arithmetic on the same values as
// k_grid_update, so the velocities are the ones G2P used.  The reverse pass
// keeps only the pre-update grids and rebuilds these.  pre_dense (may be
// NULL) also receives the pre-update values at their grid positions.
// Entries beyond the record's capacity (flagged when recorded) read as empty.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_grid_post_from_pre(KCfg c, Bufs b, int step,
                                                               const uint32_t* __restrict__ list,
                                                               const uint32_t* __restrict__ count,
                                                               const T* __restrict__ pre, int64_t pre_cap,
                                                               T* __restrict__ post, T* __restrict__ pre_dense) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = (int64_t)(*count) * NPB;
  for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < items; it += (int64_t)gridDim.x * kBlock) {
    int inst, idx[3];
    int64_t node;
    active_node<D>(c, list[it / NPB], (int)(it % NPB), inst, idx, node);
    const int64_t gid = b.inst[inst].goff + node;
    Node4<T> q = {{T(0), T(0), T(0), T(0)}};
    if (it < pre_cap) q = ld_node(pre + it * kNodeVals);
    const T acc[4] = {q.v[0], q.v[1], q.v[2], q.v[3]};
    T v[3];
    node_velocity<T, D>(c, b, inst, step, idx, acc, v);
    st_node(post + gid * kNodeVals, v[0], v[1], v[2], acc[3]);
    if (pre_dense) st_node(pre_dense + gid * kNodeVals, acc[0], acc[1], acc[2], acc[3]);
  }
}

static unsigned active_grid(const KCfg& c) {
  const int tshift = c.dim == 3 ? 6 : 4;
  const int64_t total_tiles = (c.nodes >> tshift) * c.n_inst;
  const int64_t items = total_tiles << tshift;
  const int64_t nb = (items + kBlock - 1) / kBlock;
  return (unsigned)(nb < 4096 ? nb : 4096);
}

void launch_grid_post_from_pre(int prec, const KCfg& c, const Bufs& b, int step, const uint32_t* list,
                               const uint32_t* count, const void* pre, int64_t pre_cap, void* post, void* pre_dense,
                               hipStream_t s) {
  const unsigned nb = active_grid(c);
#define DDM_GP(T, DD)                                                                                       \
  hipLaunchKernelGGL((k_grid_post_from_pre<T, DD>), dim3(nb), dim3(kBlock), 0, s, c, b, step, list, count, \
                     (const T*)pre, pre_cap, (T*)post, (T*)pre_dense)
  if (prec == 0) {
    if (c.dim == 3) DDM_GP(float, 3); else DDM_GP(float, 2);
  } else {
    if (c.dim == 3) DDM_GP(double, 3); else DDM_GP(double, 2);
  }
#undef DDM_GP
}

void launch_grid_update(int prec, const KCfg& c, const Bufs& b, int step, const Staging& stg, void* gout,
                        const ActiveSet& act, void* pre, int64_t pre_cap, void* post, uint32_t* list_out,
                        uint32_t* count_out, hipStream_t s) {
  const unsigned nb = active_grid(c);
#define DDM_GU(T, DD)                                                                                              \
  hipLaunchKernelGGL((k_grid_update<T, DD>), dim3(nb), dim3(kBlock), 0, s, c, b, step, (const T*)stg.win, stg.tslot, \
                     (T*)gout, act, (T*)pre, pre_cap, (T*)post, list_out, count_out)
  if (prec == 0) {
    if (c.dim == 3) DDM_GU(float, 3); else DDM_GU(float, 2);
  } else {
    if (c.dim == 3) DDM_GU(double, 3); else DDM_GU(double, 2);
  }
#undef DDM_GU
}

// ---------------------------------------------------------------------------
// Particle-level collision (Algorithm 1, after the gather): the grid's collision rule
// applied to a particle's velocity at its position before advection.  A
// particle in the wall layers (closer than bound cells to a face; the test is
// exact on the fixed-point position) stops; otherwise, within the contact skin
// of the blade, the blade's Coulomb contact acts on it.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ bool in_wall_layers(const KCfg& c, const P<T, D>& st, int64_t p, double xr[3]) {
  bool wall = false;
  xr[0] = xr[1] = xr[2] = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xr[a] = Pos<T>::real(st.xr(a, p));
    wall |= xr[a] < c.bound * c.dx || xr[a] >= (c.n - c.bound) * c.dx;
  }
  return wall;
}

template <typename T, int D>
__device__ __forceinline__ void particle_collision(const KCfg& c, const Bufs& b, int inst, int step,
                                                   const P<T, D>& st, int64_t p, T v[3]) {
  double xr[3];
  if (in_wall_layers<T, D>(c, st, p, xr)) {
    v[0] = v[1] = v[2] = T(0);
    return;
  }
  if (D == 3 && c.shovel) {
    const Blade<T> bl = load_blade<T>(b.poses, inst, c.max_steps, step);
    const T xp[3] = {T(xr[0]), T(xr[1]), T(xr[2])};
    const T half[3] = {T(c.half[0]), T(c.half[1]), T(c.half[2])};
    SDF<T> f;
    sdf_eval<T>(bl, half, xp, f);
    if (f.phi < T(c.skin)) {
      T vs[3];
      blade_velocity<T>(bl, xp, vs);
      coulomb_forward<T>(vs, f.n, T(c.mu_b), v);
    }
  }
}

// G2P of one particle (Algorithm 1, gather to advection) without writing it:
// v_p = sum w v_i and C_p = (4/dx^2) sum w v_i r^T from the grid velocities g
// of its instance, the particle-level collision when PC, and the advanced
// position.  Returns false when the advance leaves the fixed-point range or
// the result is not finite (the caller flags it).  Computing everything
// before the stores lets the compiler keep the kernel at 89 registers.
template <typename T, int D, bool PC>
__device__ __forceinline__ bool g2p_compute(const KCfg& c, const Bufs& b, int inst, int step, const P<T, D>& si,
                                            int64_t p, const Stencil<T, D>& S, const T* __restrict__ g, T (&vn)[3],
                                            T (&Cn)[3][3], typename Pos<T>::X (&xn)[3]) {
  const T dx = T(c.dx), Dk = T(4.0 * c.inv_dx * c.inv_dx);
  // v_p = sum w_o v_o, C_p = (4/dx^2) sum w_o v_o r_o^T with r_o = (o - f) dx:
  // sums along the last axis first, then per row
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vn[a] = T(0);
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) Cn[a][bb] = T(0);
  }
  T rr[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) rr[a][k] = a < D ? (T(k) - S.f[a]) * dx : T(0);
#pragma unroll
  for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
    for (int o1 = 0; o1 < (D == 3 ? 3 : 1); ++o1) {
      const T wxy = S.w[0][o0] * (D == 3 ? S.w[1][o1] : T(1));
      T u[3] = {T(0), T(0), T(0)}, ul[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int ol = 0; ol < 3; ++ol) {
        const T wl = S.w[D - 1][ol], wr = wl * rr[D - 1][ol];
        const Node4<T> nd = ld_node(g + (D == 3 ? node_of<D>(S.base, o0, o1, ol, c.n) : node_of<D>(S.base, o0, ol, 0, c.n)) * kNodeVals);
#pragma unroll
        for (int a = 0; a < D; ++a) { u[a] += wl * nd.v[a]; ul[a] += wr * nd.v[a]; }
      }
      const T r0 = Dk * wxy * rr[0][o0], r1 = D == 3 ? Dk * wxy * rr[1][o1] : T(0), wl2 = Dk * wxy;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        vn[a] += wxy * u[a];
        Cn[a][0] += r0 * u[a];
        if (D == 3) Cn[a][1] += r1 * u[a];
        Cn[a][D - 1] += wl2 * ul[a];
      }
    }
  if (PC) particle_collision<T, D>(c, b, inst, step, si, p, vn);
  const T dt = T(b.inst[inst].dt);
  T chk = T(0);
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    bool oka;
    xn[a] = Pos<T>::advance(si.xr(a, p), dt * vn[a], oka);
    ok &= oka;
    chk += vn[a];
#pragma unroll
    for (int bb = 0; bb < D; ++bb) chk += Cn[a][bb];
  }
  return isfinite(chk) && ok;
}

// ---------------------------------------------------------------------------
// G2P (Algorithm 1, gather to advection): v_p = sum w v_i, C_p = (4/dx^2) sum w v_i r^T,
// the particle-level collision when enabled, x_p += dt v_p.
// ---------------------------------------------------------------------------
// PC: with the particle-level collision (a separate instance, so that the
// plain kernel keeps its register budget).
// In FP32 without the particle-level collision the kernel fits 80 registers
// with no spills: 6 waves per SIMD, more gathers in flight.
template <typename T, int D, bool PC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PC || sizeof(T) == 8 ? 1 : 6)))
k_g2p(KCfg c, Bufs b, int step, const void* st_in, void* st_out, const T* __restrict__ post) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const P<T, D> si = pv<T, D>(st_in, c.ntot), so = pv<T, D>(st_out, c.ntot);
  if (p - I.off >= I.n) {
    // padding slots keep a harmless position so they never trip a check
#pragma unroll
    for (int a = 0; a < D; ++a) so.xr(a, p) = Pos<T>::from_real(0.5);
    return;
  }
  Stencil<T, D> S;
  if (!make_stencil<T, D>(si, p, c, S)) { flag_error(b.err, 2u, inst); return; }
  T vn[3], Cn[3][3];
  typename Pos<T>::X xn[3];
  const bool ok = g2p_compute<T, D, PC>(c, b, inst, step, si, p, S, post + I.goff * kNodeVals, vn, Cn, xn);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    so.xr(a, p) = xn[a];
    so.v(a, p) = vn[a];
#pragma unroll
    for (int bb = 0; bb < D; ++bb) so.C(a, bb, p) = Cn[a][bb];
  }
  if (!ok) flag_error(b.err, 1u, inst);
}

void launch_g2p(int prec, const KCfg& c, const Bufs& b, int nblk, int step, const void* st_in, void* st_out,
                const void* post, hipStream_t s) {
#define DDM_G2P(T, DD, PC) \
  hipLaunchKernelGGL((k_g2p<T, DD, PC>), dim3(nblk), dim3(kBlock), 0, s, c, b, step, st_in, st_out, (const T*)post)
  const bool pc = c.pcontact != 0;
  if (prec == 0) {
    if (c.dim == 3) { if (pc) DDM_G2P(float, 3, true); else DDM_G2P(float, 3, false); }
    else { if (pc) DDM_G2P(float, 2, true); else DDM_G2P(float, 2, false); }
  } else {
    if (c.dim == 3) { if (pc) DDM_G2P(double, 3, true); else DDM_G2P(double, 3, false); }
    else { if (pc) DDM_G2P(double, 2, true); else DDM_G2P(double, 2, false); }
  }
#undef DDM_G2P
}

// The FP32 elementary functions of the constitutive update, one value per
// thread, for accuracy tests: fn 0 log1p, 1 expm1.
__global__ void k_eval_math(int fn, const float* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  y[i] = fn == 0 ? flog1p(x[i]) : fexpm1(x[i]);
}

void launch_eval_math(int fn, const float* x, float* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_eval_math, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, fn, x, y, n);
}

// State export in the initial particle order: column off_i + pid of the
// output takes the slot holding particle pid of instance i; padding columns
// are zero.
__global__ void k_export_state(KCfg c, Bufs b, int rows, int elem_bytes, const void* in, void* out, const uint32_t* pid) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const InstDev& I = b.inst[b.blk_inst[blockIdx.x]];
  const bool live = p - I.off < I.n;
  const int64_t dst = live ? I.off + pid[p] : p;
  for (int r = 0; r < rows; ++r) {
    if (elem_bytes == 4) {
      const uint32_t v = live ? static_cast<const uint32_t*>(in)[(int64_t)r * c.ntot + p] : 0u;
      static_cast<uint32_t*>(out)[(int64_t)r * c.ntot + dst] = v;
    } else {
      const uint64_t v = live ? static_cast<const uint64_t*>(in)[(int64_t)r * c.ntot + p] : 0ull;
      static_cast<uint64_t*>(out)[(int64_t)r * c.ntot + dst] = v;
    }
  }
}

void launch_export_state(const KCfg& c, const Bufs& b, int nblk, int rows, int elem_bytes, const void* in, void* out,
                         const uint32_t* pid, hipStream_t s) {
  hipLaunchKernelGGL(k_export_state, dim3(nblk), dim3(kBlock), 0, s, c, b, rows, elem_bytes, in, out, pid);
}

__global__ void k_reset_pid(Bufs b, uint32_t* pid) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const InstDev& I = b.inst[b.blk_inst[blockIdx.x]];
  pid[p] = p - I.off < I.n ? (uint32_t)(p - I.off) : 0xFFFFFFFFu;
}

void launch_reset_pid(const Bufs& b, int nblk, uint32_t* pid, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_pid, dim3(nblk), dim3(kBlock), 0, s, b, pid);
}

// Dense export; nodes outside the active blocks of the last sub-step hold no
// mass and are exported as zeros.
template <typename T, int D>
__global__ void k_grid_export(KCfg c, const T* pre, const T* post, const uint32_t* mask, T* out) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= c.nodes * c.n_inst) return;
  const int inst = (int)(g / c.nodes);
  int idx[3];
  node_coords<D>(g - (int64_t)inst * c.nodes, c.n, idx);
  const int nt = c.n / kTile;
  const int64_t lb = D == 3 ? ((int64_t)(idx[0] / kTile) * nt + idx[1] / kTile) * nt + idx[2] / kTile
                            : (int64_t)(idx[0] / kTile) * nt + idx[1] / kTile;
  const bool act = mask[(c.nodes >> (D == 3 ? 6 : 4)) * inst + lb] != 0u;
  out[g * 8 + 0] = act ? pre[g * 4 + 3] : T(0);
  for (int a = 0; a < 3; ++a) {
    out[g * 8 + 1 + a] = act ? pre[g * 4 + a] : T(0);
    out[g * 8 + 4 + a] = act ? post[g * 4 + a] : T(0);
  }
  out[g * 8 + 7] = act ? T(1) : T(0);
}

void launch_grid_export(int prec, const KCfg& c, const void* pre, const void* post, const uint32_t* mask, void* out,
                        hipStream_t s) {
  const int64_t total = c.nodes * c.n_inst;
  const unsigned nb = (unsigned)((total + kBlock - 1) / kBlock);
#define DDM_GX(T, DD) \
  hipLaunchKernelGGL((k_grid_export<T, DD>), dim3(nb), dim3(kBlock), 0, s, c, (const T*)pre, (const T*)post, mask, (T*)out)
  if (prec == 0) {
    if (c.dim == 3) DDM_GX(float, 3); else DDM_GX(float, 2);
  } else {
    if (c.dim == 3) DDM_GX(double, 3); else DDM_GX(double, 2);
  }
#undef DDM_GX
}

// ---------------------------------------------------------------------------
// Loss.  Height map (Eq. hm): every particle touches the pixel of its own
// (x, z) and of the four points offset by +-r_p along x and z (2D: a profile
// over x, three points); a pixel keeps the largest height, ties to the lowest
// particle id.  Squared distance to the target, plus the scoop-mass term on a
// P2G of particle masses at the final positions inside the scoop slab.
// ---------------------------------------------------------------------------
// Pixel arithmetic in double on the exact stored position.
template <int D>
__device__ __forceinline__ int hm_pixels(const KCfg& c, double x, double z, int pix[5]) {
  const double pw = c.hm_pix, r = c.hm_off;
  const double ox[5] = {0.0, r, -r, 0.0, 0.0}, oz[5] = {0.0, 0.0, 0.0, r, -r};
  const int npts = D == 3 ? 5 : 3;
  int cnt = 0;
  for (int k = 0; k < npts; ++k) {
    const double px = x + ox[k];
    const double fx = floor((px - c.hm_ox) / pw);
    int iz = 0;
    if (D == 3) {
      const double pz = z + oz[k];
      const double fz = floor((pz - c.hm_oz) / pw);
      if (!(fz >= 0.0 && fz < (double)c.hm_res)) { pix[k] = -1; continue; }
      iz = (int)fz;
    }
    if (!(fx >= 0.0 && fx < (double)c.hm_res)) { pix[k] = -1; continue; }
    pix[k] = D == 3 ? (int)fx * c.hm_res + iz : (int)fx;
    ++cnt;
  }
  for (int k = npts; k < 5; ++k) pix[k] = -1;
  return cnt;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_hm_max(KCfg c, Bufs b, const void* state, unsigned long long* hm) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p - I.off >= I.n) return;
  const P<T, D> st = pv<T, D>(state, c.ntot);
  const double y = Pos<T>::real(st.xr(1, p));
  if (!(y > 0.0)) return;
  int pix[5];
  hm_pixels<D>(c, Pos<T>::real(st.xr(0, p)), D == 3 ? Pos<T>::real(st.xr(2, p)) : 0.0, pix);
  const int npix = D == 3 ? c.hm_res * c.hm_res : c.hm_res;
  const unsigned long long yb = Pos<T>::key(st.xr(1, p));
  for (int k = 0; k < 5; ++k)
    if (pix[k] >= 0) atomicMax(&hm[(int64_t)inst * npix + pix[k]], yb);
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_hm_owner(KCfg c, Bufs b, const void* state, const uint32_t* pid,
                                                     const unsigned long long* hm, unsigned int* owner) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p - I.off >= I.n) return;
  const P<T, D> st = pv<T, D>(state, c.ntot);
  const double y = Pos<T>::real(st.xr(1, p));
  if (!(y > 0.0)) return;
  int pix[5];
  hm_pixels<D>(c, Pos<T>::real(st.xr(0, p)), D == 3 ? Pos<T>::real(st.xr(2, p)) : 0.0, pix);
  const int npix = D == 3 ? c.hm_res * c.hm_res : c.hm_res;
  const unsigned long long yb = Pos<T>::key(st.xr(1, p));
  for (int k = 0; k < 5; ++k)
    if (pix[k] >= 0 && hm[(int64_t)inst * npix + pix[k]] == yb) atomicMin(&owner[(int64_t)inst * npix + pix[k]], pid[p]);
}

// Scoop region: nodes inside the slab in front of the final blade pose.
template <typename T>
__device__ __forceinline__ bool in_region(const KCfg& c, const Blade<T>& bl, const T xi[3]) {
  T e[3][3];
  blade_axes(bl, e);
  T q[3];
  const T hp = T(c.half[2]);
  for (int a = 0; a < 3; ++a) {
    q[a] = T(0);
    for (int k = 0; k < 3; ++k) q[a] += (xi[k] - (bl.tip[k] - hp * e[2][k])) * e[a][k];
  }
  const T sn = T(c.region_sign) * q[1];
  return dabs(q[0]) <= T(c.half[0]) && dabs(q[2]) <= hp && sn > T(c.half[1]) && sn <= T(c.half[1]) + T(c.region_depth);
}

template <typename T>
__device__ __forceinline__ Blade<T> final_blade(const KCfg& c, const Bufs& b, int inst, int final_step) {
  if (final_step >= 0) return load_blade<T>(b.poses, inst, c.max_steps, final_step);
  Blade<T> bl;
  for (int k = 0; k < 3; ++k) { bl.tip[k] = T(b.inst[inst].tip0[k]); bl.vel[k] = T(0); }
  bl.psi = T(0); bl.omega = T(0); bl.sp = T(0); bl.cp = T(1);
  return bl;
}

// Per particle: sum over stencil nodes inside the region of w (and grad w).
template <typename T, int D>
__device__ __forceinline__ T region_weights(const KCfg& c, const Blade<T>& bl, const Stencil<T, D>& S, T gw[3]) {
  T acc = T(0);
  gw[0] = gw[1] = gw[2] = T(0);
  const T dx = T(c.dx), inv_dx = T(c.inv_dx);
  for (int o0 = 0; o0 < 3; ++o0)
    for (int o1 = 0; o1 < 3; ++o1)
      for (int o2 = 0; o2 < 3; ++o2) {
        const int off[3] = {o0, o1, o2};
        const T xi[3] = {T(S.base[0] + o0) * dx, T(S.base[1] + o1) * dx, T(S.base[2] + o2) * dx};
        if (!in_region<T>(c, bl, xi)) continue;
        const T w0 = S.w[0][o0], w1 = S.w[1][o1], w2 = S.w[2][o2];
        acc += w0 * w1 * w2;
        gw[0] += S.dw[0][o0] * inv_dx * w1 * w2;
        gw[1] += w0 * S.dw[1][o1] * inv_dx * w2;
        gw[2] += w0 * w1 * S.dw[2][o2] * inv_dx;
        (void)off;
      }
  return acc;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_region_mass(KCfg c, Bufs b, const void* state, int final_step, double* region) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v[1] = {0.0};
  if (p - I.off < I.n) {
    const P<T, D> st = pv<T, D>(state, c.ntot);
    Stencil<T, D> S;
    if (make_stencil<T, D>(st, p, c, S)) {
      const Blade<T> bl = final_blade<T>(c, b, inst, final_step);
      T gw[3];
      v[0] = (double)(region_weights<T, D>(c, bl, S, gw) * T(I.mp));
    }
  }
  block_accumulate<1>(v, region + inst, b.dpart);
}

template <typename T, int D>
__global__ void k_loss_final(KCfg c, const unsigned long long* hm, const unsigned int* owner, LossBufs L) {
  const int inst = blockIdx.x;
  const int npix = D == 3 ? c.hm_res * c.hm_res : c.hm_res;
  double acc = 0.0;
  const double inv_dx = c.inv_dx;
  for (int i = threadIdx.x; i < npix; i += blockDim.x) {
    const int64_t k = (int64_t)inst * npix + i;
    const double h = Pos<T>::unkey(hm[k]);
    L.hm_val[k] = h;
    const double e = (h - L.target[k]) * inv_dx;
    acc += e * e;
    L.dldh[k] = owner[k] != 0xFFFFFFFFu ? 2.0 * c.w_hm / npix * (h - L.target[k]) * inv_dx * inv_dx : 0.0;
  }
  __shared__ double red[kBlock / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) s += red[w];
    double loss = c.w_hm / npix * s;
    double dldm = 0.0;
    if (D == 3 && c.shovel && c.w_mass != 0.0) {
      const double e = (L.region[inst] - c.m_target) / c.m_ref;
      loss += c.w_mass * e * e;
      dldm = 2.0 * c.w_mass * e / c.m_ref;
    }
    L.loss[inst] = loss;
    L.dldm[inst] = dldm;
  }
}

void launch_loss(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                 int final_step, const LossBufs& L, hipStream_t s) {
  const int npix = c.dim == 3 ? c.hm_res * c.hm_res : c.hm_res;
  launch_fill_zero(L.hm_bits, (int64_t)c.n_inst * npix, 8, s);
  launch_fill_u32(L.owner, (int64_t)c.n_inst * npix, 0xFFFFFFFFu, s);
  launch_fill_zero(L.region, c.n_inst, 8, s);
#define DDM_LOSS(T, DD)                                                                                      \
  hipLaunchKernelGGL((k_hm_max<T, DD>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, L.hm_bits);            \
  hipLaunchKernelGGL((k_hm_owner<T, DD>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, L.hm_bits, L.owner); \
  if (DD == 3 && c.shovel && c.w_mass != 0.0) {                                                              \
    hipLaunchKernelGGL((k_region_mass<T, 3>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, final_step, L.region); \
    if (b.dpart) launch_det_finish(c, b, false, 1, L.region, 1, s);                                           \
  }                                                                                                          \
  hipLaunchKernelGGL((k_loss_final<T, DD>), dim3(c.n_inst), dim3(kBlock), 0, s, c, L.hm_bits, L.owner, L);
  if (prec == 0) {
    if (c.dim == 3) { DDM_LOSS(float, 3) } else { DDM_LOSS(float, 2) }
  } else {
    if (c.dim == 3) { DDM_LOSS(double, 3) } else { DDM_LOSS(double, 2) }
  }
#undef DDM_LOSS
}

// Seed of the reverse pass: adjoint of the final state from the loss.
// Height: dL/dy_p sums dL/dH over the pixels p owns (each pixel once).
// Scoop mass: dL/dx_p = dL/dM m_p sum_{i in R} grad w, dL/dm_p -> rho.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_loss_seed(KCfg c, Bufs b, const void* state, const uint32_t* pid,
                                                      int final_step, LossBufs L, void* adj, double* pacc) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const P<T, D> st = pv<T, D>(state, c.ntot);
  const Adj<T, D> ad = av<T, D>(adj, c.ntot);
  double racc[1] = {0.0};
  T xb[3] = {T(0), T(0), T(0)};
  if (p - I.off < I.n) {
    const double y = Pos<T>::real(st.xr(1, p));
    if (y > 0.0) {
      int pix[5];
      hm_pixels<D>(c, Pos<T>::real(st.xr(0, p)), D == 3 ? Pos<T>::real(st.xr(2, p)) : 0.0, pix);
      const int npix = D == 3 ? c.hm_res * c.hm_res : c.hm_res;
      double yb = 0.0;
      for (int k = 0; k < 5; ++k) {
        if (pix[k] < 0) continue;
        bool dup = false;
        for (int j = 0; j < k; ++j) dup |= pix[j] == pix[k];
        const int64_t q = (int64_t)inst * npix + pix[k];
        if (!dup && L.owner[q] == pid[p]) yb += L.dldh[q];
      }
      xb[1] = T(yb);
    }
    if (D == 3 && c.shovel && c.w_mass != 0.0) {
      Stencil<T, D> S;
      if (make_stencil<T, D>(st, p, c, S)) {
        const Blade<T> bl = final_blade<T>(c, b, inst, final_step);
        T gw[3];
        const T wsum = region_weights<T, D>(c, bl, S, gw);
        const T dm = T(L.dldm[inst]);
        for (int a = 0; a < 3; ++a) xb[a] += dm * T(I.mp) * gw[a];
        racc[0] = (double)dm * (double)wsum * I.Vp;
      }
    }
  }
  for (int a = 0; a < D; ++a) {
    ad.x(a, p) = xb[a];
    ad.v(a, p) = T(0);
    for (int bb = 0; bb < D; ++bb) { ad.C(a, bb, p) = T(0); ad.G(a, bb, p) = T(0); }
  }
  block_accumulate<1>(racc, pacc + (int64_t)inst * 8 + 4, b.dpart);
}

void launch_loss_seed(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                      int final_step, const LossBufs& L, void* adj, double* pacc, hipStream_t s) {
  if (prec == 0) {
    if (c.dim == 3) hipLaunchKernelGGL((k_loss_seed<float, 3>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, final_step, L, adj, pacc);
    else hipLaunchKernelGGL((k_loss_seed<float, 2>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, final_step, L, adj, pacc);
  } else {
    if (c.dim == 3) hipLaunchKernelGGL((k_loss_seed<double, 3>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, final_step, L, adj, pacc);
    else hipLaunchKernelGGL((k_loss_seed<double, 2>), dim3(nblk), dim3(kBlock), 0, s, c, b, state, pid, final_step, L, adj, pacc);
  }
  if (b.dpart) launch_det_finish(c, b, false, 1, pacc + 4, 8, s);
}

// ---------------------------------------------------------------------------
// Adjoint of G2P + advection.  With vb = v'bar + dt x'bar:
//   xbar = x'bar + sum_i [grad w (v_i . vb + (4/dx^2) v_i^T C'bar r) - (4/dx^2) w C'bar^T v_i]
//   v_i bar += w (vb + (4/dx^2) C'bar r)            (scattered to the grid)
// ---------------------------------------------------------------------------
template <typename T, int D, bool DET>
__global__ void __launch_bounds__(kBlock) k_g2p_adj(KCfg c, Bufs b, TileList tl, const void* stv,
                                                    const T* __restrict__ post, const void* adj_next, void* adj_cur,
                                                    T* __restrict__ gvb, T* __restrict__ stg) {
  __shared__ double win[Win<D>::stride * D];
  __shared__ RunLDS<T> rl;
  __shared__ alignas(16) T gwin[Win<D>::nodes][kNodeVals];     // grid velocities of the tile's window
  const uint32_t ntiles = *tl.count;
  const P<T, D> st = pv<T, D>(stv, c.ntot);
  const Adj<T, D> an = av<T, D>(adj_next, c.ntot), ac = av<T, D>(adj_cur, c.ntot);
  const T dx = T(c.dx), inv_dx = T(c.inv_dx), Dk = T(4.0 * c.inv_dx * c.inv_dx);
  constexpr int WS = Win<D>::stride;
  // a plain grid-stride loop: the work queue's loop form costs this kernel ten
  // registers and a wave per SIMD
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileRec tr = tl.list[t];
    int inst, org[3];
    tile_origin<D>(c, tr.tile, inst, org);
    const InstDev& I = b.inst[inst];
    const T dt = T(I.dt);
    const T* g = post + I.goff * kNodeVals;
    T* gbv = gvb + I.goff * kNodeVals;
    for (int i = threadIdx.x; i < WS * D; i += kBlock) win[i] = 0.0;
    // stage the window's grid velocities (nodes outside the grid are never read)
    for (int i = threadIdx.x; i < Win<D>::nodes; i += kBlock) {
      int l[3];
      Win<D>::coords(i, l);
      const int gi[3] = {org[0] + l[0], org[1] + l[1], D == 3 ? org[2] + l[2] : 0};
      bool ok = true;
#pragma unroll
      for (int a = 0; a < D; ++a) ok &= gi[a] >= 0 && gi[a] < c.n;
      Node4<T> v = {{T(0), T(0), T(0), T(0)}};
      if (ok) v = ld_node(g + node_of<D>(gi, 0, 0, 0, c.n) * kNodeVals);
      st_node(gwin[i], v.v[0], v.v[1], v.v[2], v.v[3]);
    }
    __syncthreads();
    const int cnt = (int)(tr.end - tr.start);
    for (int r0 = 0; r0 < cnt; r0 += kBlock) {
    const int rc = min(kBlock, cnt - r0);
    int wb = -1;
    do {
      if (threadIdx.x >= rc) break;
      const int64_t p = (int64_t)tr.start + r0 + threadIdx.x;
      Stencil<T, D> S;
      if (!make_stencil<T, D>(st, p, c, S)) break;
      T xb[3], vb[3], Cb[3][3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        xb[a] = an.x(a, p);
        vb[a] = an.v(a, p) + dt * xb[a];
#pragma unroll
        for (int bb = 0; bb < D; ++bb) Cb[a][bb] = an.C(a, bb, p);
      }
      int loc[3] = {0, 0, 0};
      bool inwin = true;
#pragma unroll
      for (int a = 0; a < D; ++a) { loc[a] = S.base[a] - org[a]; inwin &= loc[a] >= 0 && loc[a] <= kWin - 3; }
      // With t_o = vb + Dk C'bar r_o = q + B o (q = vb - B f, B = Dk dx C'bar):
      //   node o receives w_o t_o;
      //   xbar += sum_o grad w_o (v_o . t_o) - Dk C'bar^T sum_o w_o v_o,
      // the first sum factored by axis (weights are products of per-axis terms).
      T q[3] = {T(0), T(0), T(0)}, B[3][3], dwi[3][3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T bf = T(0);
#pragma unroll
        for (int bb = 0; bb < D; ++bb) { B[a][bb] = Dk * dx * Cb[a][bb]; bf += B[a][bb] * S.f[bb]; }
        q[a] = vb[a] - bf;
#pragma unroll
        for (int k = 0; k < 3; ++k) dwi[a][k] = S.dw[a][k] * inv_dx;
      }
      T xg[3] = {T(0), T(0), T(0)}, vw[3] = {T(0), T(0), T(0)};
      auto body = [&](auto&& emit, auto&& load) {
        // Offsets 0 and 1 stay loops: unrolling all 27 nodes hoists their
        // loads and costs occupancy.
#pragma unroll 1
        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll 1
          for (int o1 = 0; o1 < 3; ++o1) {
            const T w0 = sel3(S.w[0], o0), w1 = sel3(S.w[1], o1);
            const T wxy = w0 * w1;
            const T a0 = sel3(dwi[0], o0) * w1, a1 = w0 * sel3(dwi[1], o1);
            T t[3] = {T(0), T(0), T(0)}, u[3] = {T(0), T(0), T(0)}, sw = T(0), sd = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) t[a] = q[a] + T(o0) * B[a][0] + T(o1) * B[a][1];
#pragma unroll
            for (int o2 = 0; o2 < (D == 3 ? 3 : 1); ++o2) {
              const T w2 = D == 3 ? S.w[2][o2] : T(1);
              const T w = wxy * w2;
              const int64_t nd = node_of<D>(S.base, o0, o1, o2, c.n) * kNodeVals;
              const Node4<T> gv = load(o0, o1, o2, nd);
              T sdot = T(0);
#pragma unroll
              for (int a = 0; a < D; ++a) { sdot += gv.v[a] * t[a]; u[a] += w2 * gv.v[a]; }
              sw += w2 * sdot;
              if (D == 3) sd += dwi[2][o2] * sdot;
              emit(o0, o1, o2, nd, w, t);
              if (D == 3) {
#pragma unroll
                for (int a = 0; a < D; ++a) t[a] += B[a][2];
              }
            }
            xg[0] += a0 * sw;
            xg[1] += a1 * sw;
            if (D == 3) xg[2] += wxy * sd;
#pragma unroll
            for (int a = 0; a < D; ++a) vw[a] += wxy * u[a];
          }
      };
      if (inwin) {
        // the scatter of w_o t_o happens in the run phase
        const int wn0 = D == 3 ? (loc[0] * kWin + loc[1]) * kWin + loc[2] : loc[0] * kWin + loc[1];
        body([&](int, int, int, int64_t, T, const T (&)[3]) {},
             [&](int o0, int o1, int o2, int64_t) {
               return ld_node(gwin[wn0 + (D == 3 ? (o0 * kWin + o1) * kWin + o2 : o0 * kWin + o1)]);
             });
        wb = Win<D>::idx(loc[0], loc[1], loc[2]);
        put_record<T, D>(rl, threadIdx.x, q, B, S.w);
      } else {
        body([&](int, int, int, int64_t nd, T w, const T (&t)[3]) {
#pragma unroll
               for (int a = 0; a < D; ++a) atomicAdd(gbv + nd + a, w * t[a]);
             },
             [&](int, int, int, int64_t nd) { return ld_node(g + nd); });
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T ctv = T(0);
#pragma unroll
        for (int bb = 0; bb < D; ++bb) ctv += Cb[bb][a] * vw[bb];
        xb[a] += xg[a] - Dk * ctv;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) ac.x(a, p) = xb[a];
    } while (false);
    rl.wbase[threadIdx.x] = wb;
    __syncthreads();
    run_scatter_round<T, D, D, 9, DET ? (D == 3 ? 27 : 9) : 1>(rl, rc, win, T(0));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Win<D>::nodes; i += kBlock) {
      int l[3];
      Win<D>::coords(i, l);
      const int wi = Win<D>::idx(l[0], l[1], l[2]);
      if (DET) {
        // the whole window, zeros included, to the tile's record (the layout of P2G's staging)
        st_node(stg + ((int64_t)t * Win<D>::nodes + i) * kNodeVals, (T)win[wi], (T)win[WS + wi],
                D == 3 ? (T)win[2 * WS + wi] : T(0), T(0));
        continue;
      }
      bool any = false;
#pragma unroll
      for (int a = 0; a < D; ++a) any |= win[a * WS + wi] != 0.0;
      if (!any) continue;
      const int gbase[3] = {org[0] + l[0], org[1] + l[1], D == 3 ? org[2] + l[2] : 0};
      T* dst = gbv + node_of<D>(gbase, 0, 0, 0, c.n) * kNodeVals;
#pragma unroll
      for (int a = 0; a < D; ++a) atomicAdd(dst + a, (T)win[a * WS + wi]);
    }
    __syncthreads();
  }
}

// The staged windows of the G2P adjoint (deterministic mode) added to the
// v-bar grid node by node, each node's covering windows in a fixed order.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_windows(KCfg c, Bufs b, const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ count, const T* __restrict__ stg,
                                                        const uint32_t* __restrict__ tslot, T* __restrict__ gvb) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = (int64_t)(*count) * NPB;
  for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < items; it += (int64_t)gridDim.x * kBlock) {
    int inst, idx[3];
    int64_t node;
    active_node<D>(c, list[it / NPB], (int)(it % NPB), inst, idx, node);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    gather_windows<T, D>(c, inst, idx, stg, tslot, acc);
    T* dst = gvb + (b.inst[inst].goff + node) * kNodeVals;
#pragma unroll
    for (int a = 0; a < D; ++a) dst[a] += acc[a];
  }
}

void launch_g2p_adj(int prec, const KCfg& c, const Bufs& b, const TileList& tl, int nwg, const void* st,
                    const void* post, const void* adj_next, void* adj_cur, void* gvb, void* stg, hipStream_t s) {
#define DDM_G2PADJ(T, DD)                                                                                         \
  if (stg)                                                                                                          \
    hipLaunchKernelGGL((k_g2p_adj<T, DD, true>), dim3(nwg), dim3(kBlock), 0, s, c, b, tl, st, (const T*)post,      \
                       adj_next, adj_cur, (T*)gvb, (T*)stg);                                                        \
  else                                                                                                              \
    hipLaunchKernelGGL((k_g2p_adj<T, DD, false>), dim3(nwg), dim3(kBlock), 0, s, c, b, tl, st, (const T*)post,     \
                       adj_next, adj_cur, (T*)gvb, (T*)nullptr)
  if (prec == 0) {
    if (c.dim == 3) { DDM_G2PADJ(float, 3); } else { DDM_G2PADJ(float, 2); }
  } else {
    if (c.dim == 3) { DDM_G2PADJ(double, 3); } else { DDM_G2PADJ(double, 2); }
  }
#undef DDM_G2PADJ
}

void launch_adj_windows(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count,
                        const void* stg, const uint32_t* tslot, void* gvb, hipStream_t s) {
  const unsigned nb = active_grid(c);
#define DDM_AW(T, DD)                                                                                            \
  hipLaunchKernelGGL((k_adj_windows<T, DD>), dim3(nb), dim3(kBlock), 0, s, c, b, list, count, (const T*)stg, tslot, \
                     (T*)gvb)
  if (prec == 0) {
    if (c.dim == 3) DDM_AW(float, 3); else DDM_AW(float, 2);
  } else {
    if (c.dim == 3) DDM_AW(double, 3); else DDM_AW(double, 2);
  }
#undef DDM_AW
}

// ---------------------------------------------------------------------------
// Adjoint of the particle-level collision.  With vb = v'bar + dt x'bar the
// adjoint of the collided velocity: a particle in the wall layers passes no
// adjoint to the G2P velocity; one in contact with the blade gets ub from the
// Coulomb adjoint at the G2P velocity u (re-gathered from the grid), and,
// since the contact sees x_p only through x_p - tip, the position adjoint
// minus the tip adjoint of the normal and of the blade velocity.  The x and v
// rows of adj_next are rewritten so that the G2P adjoint reads
// v bar + dt x bar = ub and x bar with the contact term included.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pcontact_adj(KCfg c, Bufs b, int step, const void* stv,
                                                         const T* __restrict__ post, void* adj_next,
                                                         double* pose_bar) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double pb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool any = false;
  if (p - I.off < I.n) {
    const P<T, D> st = pv<T, D>(stv, c.ntot);
    const Adj<T, D> an = av<T, D>(adj_next, c.ntot);
    const T dt = T(I.dt);
    double xr[3];
    if (in_wall_layers<T, D>(c, st, p, xr)) {
#pragma unroll
      for (int a = 0; a < D; ++a) an.v(a, p) = -dt * an.x(a, p);
    } else if (D == 3 && c.shovel) {
      const Blade<T> bl = load_blade<T>(b.poses, inst, c.max_steps, step);
      const T xp[3] = {T(xr[0]), T(xr[1]), T(xr[2])};
      const T half[3] = {T(c.half[0]), T(c.half[1]), T(c.half[2])};
      SDF<T> f;
      sdf_eval<T>(bl, half, xp, f);
      Stencil<T, D> S;
      if (f.phi < T(c.skin) && make_stencil<T, D>(st, p, c, S)) {
        const T* g = post + I.goff * kNodeVals;
        T u[3] = {T(0), T(0), T(0)};
#pragma unroll 1
        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll 1
          for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
              const T w = sel3(S.w[0], o0) * sel3(S.w[1], o1) * S.w[2][o2];
              const Node4<T> nd = ld_node(g + node_of<D>(S.base, o0, o1, o2, c.n) * kNodeVals);
#pragma unroll
              for (int a = 0; a < 3; ++a) u[a] += w * nd.v[a];
            }
        T vb[3], vs[3], ub[3], vsb[3], nb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) vb[a] = an.v(a, p) + dt * an.x(a, p);
        blade_velocity<T>(bl, xp, vs);
        coulomb_backward<T>(vs, f.n, T(c.mu_b), u, vb, ub, vsb, nb);
        // v_s = v_lin + (omega (y - tip_y), -omega (x - tip_x), 0)
        T tipb[3] = {T(0), T(0), T(0)}, psib = T(0);
        const T omb = vsb[0] * (xp[1] - bl.tip[1]) - vsb[1] * (xp[0] - bl.tip[0]);
        tipb[1] -= bl.omega * vsb[0];
        tipb[0] += bl.omega * vsb[1];
        sdf_normal_backward<T>(bl, half, xp, f, nb, tipb, psib);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T xb = an.x(a, p) - tipb[a];
          an.x(a, p) = xb;
          an.v(a, p) = ub[a] - dt * xb;
        }
        pb[0] = tipb[0]; pb[1] = tipb[1]; pb[2] = tipb[2]; pb[3] = psib;
        pb[4] = vsb[0]; pb[5] = vsb[1]; pb[6] = vsb[2]; pb[7] = omb;
        any = true;
      }
    }
  }
  // a 256-slot block belongs to one instance
  if (D == 3 && c.shovel && b.dpart) {
    block_accumulate<8>(pb, nullptr, b.dpart);
  } else if (D == 3 && c.shovel && __any(any)) {
    double* dst = pose_bar + ((int64_t)inst * c.max_steps + step) * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double sum = wave_sum(pb[k]);
      if ((threadIdx.x & 63) == 0 && sum != 0.0) atomicAdd(dst + k, sum);
    }
  }
}

void launch_pcontact_adj(int prec, const KCfg& c, const Bufs& b, int nblk, int step, const void* st,
                         const void* post, void* adj_next, double* pose_bar, hipStream_t s) {
  if (prec == 0) {
    if (c.dim == 3) hipLaunchKernelGGL((k_pcontact_adj<float, 3>), dim3(nblk), dim3(kBlock), 0, s, c, b, step, st, (const float*)post, adj_next, pose_bar);
    else hipLaunchKernelGGL((k_pcontact_adj<float, 2>), dim3(nblk), dim3(kBlock), 0, s, c, b, step, st, (const float*)post, adj_next, pose_bar);
  } else {
    if (c.dim == 3) hipLaunchKernelGGL((k_pcontact_adj<double, 3>), dim3(nblk), dim3(kBlock), 0, s, c, b, step, st, (const double*)post, adj_next, pose_bar);
    else hipLaunchKernelGGL((k_pcontact_adj<double, 2>), dim3(nblk), dim3(kBlock), 0, s, c, b, step, st, (const double*)post, adj_next, pose_bar);
  }
  if (b.dpart && c.dim == 3 && c.shovel)
    launch_det_finish(c, b, false, 8, pose_bar + (int64_t)step * 8, (int64_t)c.max_steps * 8, s);
}

// ---------------------------------------------------------------------------
// Adjoint of the grid update: walls cut the gradient, contact is replayed with
// the same branch, u = mv/m + dt g gives mv bar = u bar / m and
// m bar = -u bar . (mv/m) / m.  Pose adjoints (tip, psi, v_lin, omega) of the
// sub-step are reduced over the contact nodes.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_grid_adj(KCfg c, Bufs b, int step, const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ count, const T* __restrict__ pre,
                                                     int64_t pre_cap, T* __restrict__ gvb, T* __restrict__ gb,
                                                     double* pose_bar) {
  constexpr int NPB = D == 3 ? kTile * kTile * kTile : kTile * kTile;
  const int64_t items = (int64_t)(*count) * NPB;
  // 3D: the 64 lanes of a wave take the 64 nodes of one block, hence one instance
  for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < items; it += (int64_t)gridDim.x * kBlock) {
    int inst, idx[3];
    int64_t node;
    active_node<D>(c, list[it / NPB], (int)(it % NPB), inst, idx, node);
    const int64_t gid = b.inst[inst].goff + node;
    double pb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool any = false;
    Node4<T> pr = {{T(0), T(0), T(0), T(0)}};
    if (it < pre_cap) pr = ld_node(pre + it * kNodeVals);
    T vb[3] = {T(0), T(0), T(0)};
    {
      T* gv = gvb + gid * kNodeVals;
      const Node4<T> o = ld_node(gv);
#pragma unroll
      for (int a = 0; a < D; ++a) vb[a] = o.v[a];
      if (o.v[0] != T(0) || o.v[1] != T(0) || o.v[2] != T(0)) {
#pragma unroll
        for (int a = 0; a < 3; ++a) gv[a] = T(0);
      }
    }
    const T m = pr.v[3];
    T ub[3] = {T(0), T(0), T(0)};
    T mb = T(0);
    if (m > T(0)) {
      bool wall = false;
#pragma unroll
      for (int a = 0; a < D; ++a) wall |= (idx[a] < c.bound) || (idx[a] >= c.n - c.bound);
      if (!wall) {
        T u[3] = {T(0), T(0), T(0)};
        const T dt = T(b.inst[inst].dt);
#pragma unroll
        for (int a = 0; a < D; ++a) u[a] = pr.v[a] / m;
        u[1] += dt * T(c.gravity);
#pragma unroll
        for (int a = 0; a < 3; ++a) ub[a] = vb[a];
        if (D == 3 && c.shovel) {
          const Blade<T> bl = load_blade<T>(b.poses, inst, c.max_steps, step);
          const T xi[3] = {T(idx[0]) * T(c.dx), T(idx[1]) * T(c.dx), T(idx[2]) * T(c.dx)};
          const T half[3] = {T(c.half[0]), T(c.half[1]), T(c.half[2])};
          SDF<T> f;
          sdf_eval<T>(bl, half, xi, f);
          if (f.phi < T(c.skin)) {
            T vs[3], vsb[3], nb[3];
            blade_velocity<T>(bl, xi, vs);
            coulomb_backward<T>(vs, f.n, T(c.mu_b), u, vb, ub, vsb, nb);
            // v_s = v_lin + (psi_dot (y - tip_y), -psi_dot (x - tip_x), 0)
            T tipb[3] = {T(0), T(0), T(0)}, psib = T(0);
            const T omb = vsb[0] * (xi[1] - bl.tip[1]) - vsb[1] * (xi[0] - bl.tip[0]);
            tipb[1] -= bl.omega * vsb[0];
            tipb[0] += bl.omega * vsb[1];
            sdf_normal_backward<T>(bl, half, xi, f, nb, tipb, psib);
            pb[0] = tipb[0]; pb[1] = tipb[1]; pb[2] = tipb[2]; pb[3] = psib;
            pb[4] = vsb[0]; pb[5] = vsb[1]; pb[6] = vsb[2]; pb[7] = omb;
            any = true;
          }
        }
        // m bar = -(u bar . mv) / m^2, formed as -(u bar . (mv / m)) / m: for a node
        // that holds only a sliver of B-spline weight, m^2 underflows in FP32
        const T im = T(1) / m;
        T dot = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) dot += ub[a] * (pr.v[a] * im);
        mb = -dot * im;
#pragma unroll
        for (int a = 0; a < D; ++a) ub[a] = ub[a] * im;
      }
    }
    gb[gid * kNodeVals + 0] = ub[0];
    gb[gid * kNodeVals + 1] = ub[1];
    gb[gid * kNodeVals + 2] = ub[2];
    gb[gid * kNodeVals + 3] = mb;
    if (D == 3 && c.shovel && __any(any)) {
      // the 64 lanes hold the nodes of one block: its sums go to the block's
      // partials in the deterministic mode
      double* dst = b.dpart ? b.dpart + (int64_t)list[it / NPB] * kDetVals
                            : pose_bar + ((int64_t)inst * c.max_steps + step) * 8;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double sum = wave_sum(pb[k]);
        if ((threadIdx.x & 63) == 0) {
          if (b.dpart) dst[k] = sum;
          else if (sum != 0.0) atomicAdd(dst + k, sum);
        }
      }
    }
  }
}

void launch_grid_adj(int prec, const KCfg& c, const Bufs& b, int step, const uint32_t* list, const uint32_t* count,
                     const void* pre, int64_t pre_cap, void* gvb, void* gb, double* pose_bar, hipStream_t s) {
  const unsigned nb = active_grid(c);
#define DDM_GA(T, DD)                                                                                             \
  hipLaunchKernelGGL((k_grid_adj<T, DD>), dim3(nb), dim3(kBlock), 0, s, c, b, step, list, count, (const T*)pre,  \
                     pre_cap, (T*)gvb, (T*)gb, pose_bar)
  if (prec == 0) {
    if (c.dim == 3) DDM_GA(float, 3); else DDM_GA(float, 2);
  } else {
    if (c.dim == 3) DDM_GA(double, 3); else DDM_GA(double, 2);
  }
#undef DDM_GA
  if (b.dpart && c.dim == 3 && c.shovel)
    launch_det_finish(c, b, true, 8, pose_bar + (int64_t)step * 8, (int64_t)c.max_steps * 8, s);
}

// ---------------------------------------------------------------------------
// Adjoint of P2G and of the constitutive update, in two kernels so that the
// 27-node gather and the SVD-frame adjoint do not hold registers at the same
// time.
//  k_p2g_adj_gather: rebuilds A = k tau + m_p C from the stored stress, gathers the
//    grid adjoints (m bar, mv bar) over the stencil and writes x bar (adding
//    to the G2P part already there), v bar, and A bar into the C bar rows;
//    the density adjoint V_p (m_p bar + A bar : C) is block-reduced.
//  k_p2g_adj_constit: tau bar = k A bar, back through the return map and the
//    SVD (isotropic-function adjoint) and F_tmp = (I + dt C)(I + G); writes
//    G bar and C bar = m_p A bar + dt F_tmp bar (I + G)^T; material adjoints
//    (mu, lambda, alpha, k_c) are block-reduced in double.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void ftmp_of(const P<T, D>& st, int64_t p, T dt, T Cm[3][3], T Gm[3][3], T Ft[3][3]) {
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
}

template <typename T, int D, bool SF>
__global__ void __launch_bounds__(kBlock) k_p2g_adj_gather(KCfg c, Bufs b, const void* stv, const T* __restrict__ tau,
                                                           const T* __restrict__ gbar, void* adj_cur, double* pacc) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc[1] = {0.0};
  if (p - I.off < I.n) {
    const P<T, D> st = pv<T, D>(stv, c.ntot);
    const Adj<T, D> ac = av<T, D>(adj_cur, c.ntot);
    Stencil<T, D> S;
    if (make_stencil<T, D>(st, p, c, S)) {
      const T dt = T(I.dt), mp = T(I.mp), dx = T(c.dx), inv_dx = T(c.inv_dx);
      // A = k tau + m_p C with the stress the recomputed forward step stored
      T Cm[3][3], vel[3], A[3][3];
      const T k_str = -dt * T(I.Vp) * T(4.0 * c.inv_dx * c.inv_dx);
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
          Cm[a][bb] = st.C(a, bb, p);
          A[a][bb] = k_str * tau[(int64_t)sym_row<D>(a, bb) * c.ntot + p] + mp * Cm[a][bb];
        }
#pragma unroll
      for (int a = 0; a < D; ++a) vel[a] = st.v(a, p);
      // Node o (weight w_o, offset r_o = (o - f) dx) received m_p w_o and
      // w_o t_o, t_o = m_p v + A r_o.  With g_m, g_v its mass and momentum
      // adjoints and G = sum w_o g_v:
      //   mass adjoint   sum w_o (g_m + v . g_v) = sum w_o g_m + v . G
      //   v bar          m_p G
      //   A bar          sum w_o g_v r_o^T
      //   x bar         += sum grad w_o (m_p g_m + g_v . t_o) - A^T G
      // The sums run along the last axis first and are factored by axis.
      // Density: every particle of an instance has the mass m_p = rho V_p,
      // so node o's mass m_o and the part mv_o - f_o of its momentum that is
      // not stress (f_o = sum_p w_op S_p r_op, S_p = k tau_p) are linear in
      // rho.  Without a gradient treatment of the grid adjoints the grid
      // update's adjoint gives g_m = -g_v . mv_o / m_o, and the sub-step's
      // density adjoint sum_o (g_m m_o + g_v . (mv_o - f_o)) / rho reduces to
      // -sum_o g_v . f_o / rho = -sum_p (S_p : A bar_p) / rho.  That form is
      // used then: the mass form sum_o w_o (g_m + g_v . (v + C r_o)) is a
      // near-cancelling sum whose terms carry the FP32 rounding of g_m and
      // g_v (of order eps |g_v| |v|).
      T xb[3];
#pragma unroll
      for (int a = 0; a < D; ++a) xb[a] = ac.x(a, p);     // G2P part, written by k_g2p_adj
      const T* g = gbar + I.goff * kNodeVals;
      T rr[3][3], dwi[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          rr[a][k] = a < D ? (T(k) - S.f[a]) * dx : T(0);
          dwi[a][k] = a < D ? S.dw[a][k] * inv_dx : T(0);
        }
      T mvv[3] = {T(0), T(0), T(0)}, Bl[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int a = 0; a < D; ++a) { mvv[a] = mp * vel[a]; Bl[a] = A[a][D - 1] * dx; }
      T G[3] = {T(0), T(0), T(0)}, Gm = T(0), xg[3] = {T(0), T(0), T(0)};
      T Ab[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
      for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < (D == 3 ? 3 : 1); ++o1) {
          // 3D: row (o0, o1) along axis 2; 2D: row o0 along axis 1
          const T wa = S.w[0][o0], wb = D == 3 ? S.w[1][o1] : T(1);
          const T wxy = wa * wb;
          const T a0 = dwi[0][o0] * wb, a1 = D == 3 ? wa * dwi[1][o1] : T(0);
          T t[3] = {T(0), T(0), T(0)};
#pragma unroll
          for (int a = 0; a < D; ++a)
            t[a] = mvv[a] + A[a][0] * rr[0][o0] + (D == 3 ? A[a][1] * rr[1][o1] : T(0)) + A[a][D - 1] * rr[D - 1][0];
          T u[3] = {T(0), T(0), T(0)}, ul[3] = {T(0), T(0), T(0)}, um = T(0), sw = T(0), sd = T(0);
#pragma unroll
          for (int ol = 0; ol < 3; ++ol) {
            const T wl = S.w[D - 1][ol];
            const int64_t nd = (D == 3 ? node_of<D>(S.base, o0, o1, ol, c.n) : node_of<D>(S.base, o0, ol, 0, c.n)) * kNodeVals;
            const Node4<T> gn = ld_node(g + nd);
            T sc = mp * gn.v[3];
#pragma unroll
            for (int a = 0; a < D; ++a) sc += gn.v[a] * t[a];
            sw += wl * sc;
            sd += dwi[D - 1][ol] * sc;
            um += wl * gn.v[3];
            const T wr = wl * rr[D - 1][ol];
#pragma unroll
            for (int a = 0; a < D; ++a) { u[a] += wl * gn.v[a]; ul[a] += wr * gn.v[a]; t[a] += Bl[a]; }
          }
          Gm += wxy * um;
          if (D == 3) {
            xg[0] += a0 * sw;
            xg[1] += a1 * sw;
            xg[2] += wxy * sd;
          } else {
            xg[0] += a0 * sw;
            xg[1] += wa * sd;
          }
          const T r0 = wxy * rr[0][o0], r1 = D == 3 ? wxy * rr[1][o1] : T(0);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            G[a] += wxy * u[a];
            Ab[a][0] += r0 * u[a];
            if (D == 3) Ab[a][1] += r1 * u[a];
            Ab[a][D - 1] += wxy * ul[a];
          }
        }
      T vb[3] = {T(0), T(0), T(0)};
      T mpb = Gm;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        mpb += vel[a] * G[a];
        vb[a] = mp * G[a];
        T atg = T(0);
#pragma unroll
        for (int bb = 0; bb < D; ++bb) atg += A[bb][a] * G[bb];
        xb[a] += xg[a] - atg;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        ac.x(a, p) = xb[a];
        ac.v(a, p) = vb[a];
#pragma unroll
        for (int bb = 0; bb < D; ++bb) { ac.C(a, bb, p) = Ab[a][bb]; mpb += Ab[a][bb] * Cm[a][bb]; }
      }
      if (SF) {
        T sab = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int bb = 0; bb < D; ++bb) sab += tau[(int64_t)sym_row<D>(a, bb) * c.ntot + p] * Ab[a][bb];
        acc[0] = -(double)(k_str * sab) * (I.Vp / I.mp);
      } else {
        acc[0] = (double)mpb * I.Vp;
      }
    }
  }
  block_accumulate<1>(acc, pacc + (int64_t)inst * 8 + 4, b.dpart);
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_p2g_adj_constit(KCfg c, Bufs b, const void* stv, const void* adj_next,
                                                            void* adj_cur, double* pacc) {
  const int inst = b.blk_inst[blockIdx.x];
  const InstDev& I = b.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  if (p - I.off < I.n) {
    const P<T, D> st = pv<T, D>(stv, c.ntot);
    const Adj<T, D> an = av<T, D>(adj_next, c.ntot), ac = av<T, D>(adj_cur, c.ntot);
    const T dt = T(I.dt), mp = T(I.mp);
    const T mu = T(I.mu), lam = T(I.lam), al = T(I.alpha), kc = T(I.kc);
    const T k_str = -dt * T(I.Vp) * T(4.0 * c.inv_dx * c.inv_dx);
    T Cm[3][3], Gm[3][3], Ft[3][3], Ab[3][3], taub[3][3], Fnb[3][3];
    ftmp_of<T, D>(st, p, dt, Cm, Gm, Ft);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        Ab[a][bb] = ac.C(a, bb, p);
        taub[a][bb] = k_str * Ab[a][bb];
        Fnb[a][bb] = an.G(a, bb, p);
      }
    Constit<T, D> cs;
    constit_forward<T, D>(Ft, mu, lam, al, kc, cs);
    T Ftb[3][3], mub = T(0), lamb = T(0), alb = T(0), kcb = T(0);
    constit_backward<T, D>(cs, mu, lam, al, kc, Fnb, taub, Ftb, mub, lamb, alb, kcb);
    // F_tmp = (I + dt C) F with F = I + G
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        T fb = Ftb[a][bb], cb = Ftb[a][bb];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          fb += dt * Cm[k][a] * Ftb[k][bb];
          cb += Ftb[a][k] * Gm[bb][k];
        }
        ac.G(a, bb, p) = fb;
        ac.C(a, bb, p) = mp * Ab[a][bb] + dt * cb;
      }
    acc[0] = (double)mub;
    acc[1] = (double)lamb;
    acc[2] = (double)alb;
    acc[3] = (double)kcb;
  }
  block_accumulate<4>(acc, pacc + (int64_t)inst * 8, b.dpart);
}

void launch_p2g_adj(int prec, const KCfg& c, const Bufs& b, int nblk, const void* st, const void* tau, const void* gb,
                    bool stress_form, const void* adj_next, void* adj_cur, double* pacc, hipStream_t s) {
#define DDM_P2GADJ(T, DD)                                                                                          \
  if (stress_form)                                                                                                 \
    hipLaunchKernelGGL((k_p2g_adj_gather<T, DD, true>), dim3(nblk), dim3(kBlock), 0, s, c, b, st,                  \
                       (const T*)tau, (const T*)gb, adj_cur, pacc);                                                \
  else                                                                                                             \
    hipLaunchKernelGGL((k_p2g_adj_gather<T, DD, false>), dim3(nblk), dim3(kBlock), 0, s, c, b, st,                 \
                       (const T*)tau, (const T*)gb, adj_cur, pacc);                                                \
  if (b.dpart) launch_det_finish(c, b, false, 1, pacc + 4, 8, s);                                                  \
  hipLaunchKernelGGL((k_p2g_adj_constit<T, DD>), dim3(nblk), dim3(kBlock), 0, s, c, b, st, adj_next, adj_cur, pacc); \
  if (b.dpart) launch_det_finish(c, b, false, 4, pacc, 8, s);
  if (prec == 0) {
    if (c.dim == 3) { DDM_P2GADJ(float, 3) } else { DDM_P2GADJ(float, 2) }
  } else {
    if (c.dim == 3) { DDM_P2GADJ(double, 3) } else { DDM_P2GADJ(double, 2) }
  }
#undef DDM_P2GADJ
}

// ---------------------------------------------------------------------------
// Final gradient per instance: chain (mu, lambda, alpha, k_c, rho) adjoints to
// (E, nu, phi_deg, rho) and the per-sub-step pose adjoints through the pose
// Jacobian d pose / d (depth, angle_deg, push, displace, push_angle_deg);
// scale by dloss.
// ---------------------------------------------------------------------------
__global__ void k_grad_final(KCfg c, const InstDev* inst, const double* pacc, const double* pose_bar,
                             const double* pose_jac, int n_steps, const double* dloss, double* grad) {
  constexpr int NS = kSkillParams;
  const int i = blockIdx.x;
  double s[NS] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int st = threadIdx.x; st < n_steps; st += blockDim.x) {
    const double* pb = pose_bar + ((int64_t)i * c.max_steps + st) * 8;
    const double* J = pose_jac + ((int64_t)i * c.max_steps + st) * 8 * NS;
    for (int k = 0; k < 8; ++k)
      for (int j = 0; j < NS; ++j) s[j] += pb[k] * J[k * NS + j];
  }
  __shared__ double red[kBlock / 64][NS];
  for (int j = 0; j < NS; ++j) {
    const double v = wave_sum(s[j]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][j] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const InstDev& I = inst[i];
    const double* a = pacc + (int64_t)i * 8;
    const double sc = dloss[i];
    double sk[NS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < (int)blockDim.x / 64; ++w)
      for (int j = 0; j < NS; ++j) sk[j] += red[w][j];
    double* gi = grad + (int64_t)i * kParams;
    gi[0] = sc * (a[0] * I.dmu_dE + a[1] * I.dlam_dE);
    gi[1] = sc * (a[0] * I.dmu_dnu + a[1] * I.dlam_dnu);
    gi[2] = sc * (a[2] * I.dal_dphi + a[3] * I.dkc_dphi);
    gi[3] = sc * a[4];
    for (int j = 0; j < NS; ++j) gi[4 + j] = sc * sk[j];
  }
}

void launch_grad_final(const KCfg& c, const InstDev* inst, const double* pacc, const double* pose_bar,
                       const double* pose_jac, int n_steps, const double* dloss, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_final, dim3(c.n_inst), dim3(kBlock), 0, s, c, inst, pacc, pose_bar, pose_jac, n_steps,
                     dloss, grad);
}

}  // namespace ddm
