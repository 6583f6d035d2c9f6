// Binning of particles: exact integer cell keys from the stored positions, a
// stable least-significant-digit radix sort (8-bit digits, wave64 ballot
// ranking), the state gather into sorted order, and the list of occupied
// tiles that the scatter kernels work on.
//
// Key of a live particle: inst * (n^D + 1) + tile * B^D + cell-in-tile, with
// tile and cell-in-tile lexicographic in (x, y[, z]) (last axis fastest) and
// B = kTile.  Padding slots get inst * (n^D + 1) + n^D, so every instance keeps
// its slot range and its padding stays at the end of it.
#include <hip/hip_runtime.h>

#include "ddm_kernels.hpp"

namespace ddm {

constexpr int kSortItems = 8;                       // keys per thread in a sort block
constexpr int kSortBlockKeys = kBlock * kSortItems; // 2048

// Base cell of one axis from a stored position (same rule as the stencil).
__device__ __forceinline__ bool cell_f32(uint32_t xr, const KCfg& c, int& base) {
  const uint64_t q = (uint64_t)xr << c.nlog2;
  if (q < 0x80000000ull) { base = 0; return false; }
  const uint64_t b = (q - 0x80000000ull) >> 32;
  if (b > (uint64_t)(c.n - 3)) { base = c.n - 3; return false; }
  base = (int)b;
  return true;
}
__device__ __forceinline__ bool cell_f64(double xr, const KCfg& c, int& base) {
  const double bf = floor(xr * c.inv_dx - 0.5);
  if (!(bf >= 0.0)) { base = 0; return false; }
  if (!(bf <= (double)(c.n - 3))) { base = c.n - 3; return false; }
  base = (int)bf;
  return true;
}

template <int PREC>
__global__ void k_keys(KCfg c, const int* blk_inst, const InstDev* inst, const void* state, uint32_t* keys,
                       uint32_t* vals, DevErr* err, const uint32_t* order) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t p = order ? (int64_t)order[j] : j;
  const int i = blk_inst[p / kBlock];
  const InstDev& I = inst[i];
  const uint32_t cells = (uint32_t)c.nodes;
  uint32_t key = (uint32_t)i * (cells + 1u) + cells;
  if (p - I.off < I.n) {
    const int nt = c.n / kTile;
    uint32_t t = 0, cl = 0;
    bool ok = true;
    for (int a = 0; a < c.dim; ++a) {
      int b;
      if (PREC == 0) ok &= cell_f32(static_cast<const uint32_t*>(state)[(int64_t)a * c.ntot + p], c, b);
      else ok &= cell_f64(static_cast<const double*>(state)[(int64_t)a * c.ntot + p], c, b);
      t = t * nt + b / kTile;
      cl = cl * kTile + b % kTile;
    }
    if (!ok) atomicOr(&err->flags, 2u);
    const uint32_t tcells = c.dim == 3 ? kTile * kTile * kTile : kTile * kTile;
    key = (uint32_t)i * (cells + 1u) + t * tcells + cl;
  }
  keys[j] = key;
  vals[j] = (uint32_t)p;
}

void launch_keys(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, uint32_t* keys, uint32_t* vals,
                 hipStream_t s, const uint32_t* order) {
  if (prec == 0) hipLaunchKernelGGL(k_keys<0>, dim3(nblk), dim3(kBlock), 0, s, c, b.blk_inst, b.inst, state, keys, vals, b.err, order);
  else hipLaunchKernelGGL(k_keys<1>, dim3(nblk), dim3(kBlock), 0, s, c, b.blk_inst, b.inst, state, keys, vals, b.err, order);
}

// Keys of the deterministic mode's first sort: the particle id (padding slots
// last), so that a stable sort by cell afterwards orders a cell's particles by id.
__global__ void k_pid_keys(const uint32_t* pid, uint32_t* keys, uint32_t* vals, int64_t ntot) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= ntot) return;
  const uint32_t id = pid[p];
  keys[p] = id == 0xFFFFFFFFu ? (uint32_t)ntot : id;
  vals[p] = (uint32_t)p;
}

void launch_pid_keys(const uint32_t* pid, uint32_t* keys, uint32_t* vals, int64_t ntot, hipStream_t s) {
  hipLaunchKernelGGL(k_pid_keys, dim3((unsigned)((ntot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, pid, keys, vals,
                     ntot);
}

// ---------------------------------------------------------------------------
// Radix sort pass: digit histogram per block, exclusive scan over
// hist[digit][block], stable scatter.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* keys, int64_t n, int shift, uint32_t* hist,
                                                       int nsb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys;
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t e = base + (int64_t)k * kBlock + threadIdx.x;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nsb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of a uint32 array in three launches (block scan, scan of
// block totals, add).  Block = 256 threads x 8 items.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t ws[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wid] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) off += ws[w];
    tot += ws[w];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_local(uint32_t* a, int64_t n, uint32_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys + (int64_t)threadIdx.x * kSortItems;
  uint32_t v[kSortItems], s = 0;
  for (int k = 0; k < kSortItems; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot);
  for (int k = 0; k < kSortItems; ++k) {
    if (base + k < n) a[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_sums(uint32_t* sums, int64_t m) {
  // one block; loops over chunks of kSortBlockKeys
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < m; c0 += kSortBlockKeys) {
    const int64_t base = c0 + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems], s = 0;
    for (int k = 0; k < kSortItems; ++k) {
      v[k] = base + k < m ? sums[base + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan(s, &tot);
    for (int k = 0; k < kSortItems; ++k) {
      if (base + k < m) sums[base + k] = run;
      run += v[k];
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_add(uint32_t* a, int64_t n, const uint32_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys + (int64_t)threadIdx.x * kSortItems;
  const uint32_t add = sums[blockIdx.x];
  for (int k = 0; k < kSortItems; ++k)
    if (base + k < n) a[base + k] += add;
}

static void excl_scan(uint32_t* a, int64_t n, uint32_t* sums, hipStream_t s) {
  const int64_t nb = (n + kSortBlockKeys - 1) / kSortBlockKeys;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kBlock), 0, s, a, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, a, n, sums);
}

// Stable scatter: elements of a block in the order e = base + k * 256 + tid,
// ranked among equal digits with wave ballots (peer masks) and per-wave
// digit counts in LDS.
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                          uint32_t* vout, int64_t n, int shift, const uint32_t* offs,
                                                          int nsb) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kBlock / 64][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * nsb + blockIdx.x];
  for (int w = 0; w < kBlock / 64; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t e = base + (int64_t)k * kBlock + threadIdx.x;
    const bool valid = e < n;
    const uint32_t key = valid ? kin[e] : 0u;
    const uint32_t val = valid ? vin[e] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank_w = (uint32_t)__popcll(peers & lt);
    const bool leader = valid && (peers & lt) == 0ull;
    if (leader) wcnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank_w;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    {
      uint32_t add = 0;
      for (int w = 0; w < kBlock / 64; ++w) { add += wcnt[w][threadIdx.x]; wcnt[w][threadIdx.x] = 0; }
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

int sort_passes(uint32_t max_key) {
  int bits = 0;
  while (bits < 32 && (max_key >> bits) != 0u) ++bits;
  return (bits + 7) / 8;
}

int64_t sort_hist_words(int64_t n) {
  const int64_t nsb = (n + kSortBlockKeys - 1) / kSortBlockKeys;
  return 256 * nsb;
}

int64_t sort_sum_words(int64_t n) {
  const int64_t h = sort_hist_words(n);
  return (h + kSortBlockKeys - 1) / kSortBlockKeys + 1;
}

// Sorts (keys[0], vals[0]) (ping-pong through keys[1], vals[1]); returns the
// index of the buffer pair holding the result.
int radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t n, uint32_t max_key, uint32_t* hist, uint32_t* sums,
                hipStream_t s) {
  const int passes = sort_passes(max_key);
  const int nsb = (int)((n + kSortBlockKeys - 1) / kSortBlockKeys);
  int cur = 0;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    hipLaunchKernelGGL(k_radix_hist, dim3(nsb), dim3(kBlock), 0, s, keys[cur], n, shift, hist, nsb);
    excl_scan(hist, (int64_t)256 * nsb, sums, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nsb), dim3(kBlock), 0, s, keys[cur], vals[cur], keys[1 - cur],
                       vals[1 - cur], n, shift, hist, nsb);
    cur = 1 - cur;
  }
  return cur;
}

// ---------------------------------------------------------------------------
// Gather of the state rows (and ids) into sorted order, and the inverse
// (scatter) used to carry adjoints back across a sort.
// ---------------------------------------------------------------------------
template <typename W>
__global__ void k_gather(const W* in, W* out, const uint32_t* perm, int rows, int64_t ntot, const uint32_t* pid_in,
                         uint32_t* pid_out) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= ntot) return;
  const int64_t src = perm[j];
  for (int r = 0; r < rows; ++r) out[(int64_t)r * ntot + j] = in[(int64_t)r * ntot + src];
  if (pid_out) pid_out[j] = pid_in[src];
}

template <typename W>
__global__ void k_scatter(const W* in, W* out, const uint32_t* perm, int rows, int64_t ntot) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= ntot) return;
  const int64_t dst = perm[j];
  for (int r = 0; r < rows; ++r) out[(int64_t)r * ntot + dst] = in[(int64_t)r * ntot + j];
}

void launch_gather(int elem_bytes, const void* in, void* out, const uint32_t* perm, int rows, int64_t ntot,
                   const uint32_t* pid_in, uint32_t* pid_out, hipStream_t s) {
  const unsigned nb = (unsigned)((ntot + kBlock - 1) / kBlock);
  if (elem_bytes == 4) hipLaunchKernelGGL(k_gather<uint32_t>, dim3(nb), dim3(kBlock), 0, s, (const uint32_t*)in, (uint32_t*)out, perm, rows, ntot, pid_in, pid_out);
  else hipLaunchKernelGGL(k_gather<uint64_t>, dim3(nb), dim3(kBlock), 0, s, (const uint64_t*)in, (uint64_t*)out, perm, rows, ntot, pid_in, pid_out);
}

void launch_unpermute(int elem_bytes, const void* in, void* out, const uint32_t* perm, int rows, int64_t ntot,
                      hipStream_t s) {
  const unsigned nb = (unsigned)((ntot + kBlock - 1) / kBlock);
  if (elem_bytes == 4) hipLaunchKernelGGL(k_scatter<uint32_t>, dim3(nb), dim3(kBlock), 0, s, (const uint32_t*)in, (uint32_t*)out, perm, rows, ntot);
  else hipLaunchKernelGGL(k_scatter<uint64_t>, dim3(nb), dim3(kBlock), 0, s, (const uint64_t*)in, (uint64_t*)out, perm, rows, ntot);
}

// ---------------------------------------------------------------------------
// Occupied tiles from the sorted keys: [start, end) slot ranges per tile.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t key_tile(uint32_t key, const KCfg& c, int tshift) {
  const uint32_t cells = (uint32_t)c.nodes;
  const uint32_t inst = key / (cells + 1u);
  const uint32_t local = key - inst * (cells + 1u);
  if (local >= cells) return -1;               // padding
  const int64_t tiles = c.nodes >> tshift;
  return (int64_t)inst * tiles + (local >> tshift);
}

__global__ void k_tile_bounds(KCfg c, const uint32_t* keys, int tshift, uint32_t* tstart, uint32_t* tend) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= c.ntot) return;
  const int64_t t = key_tile(keys[j], c, tshift);
  if (t < 0) return;
  const int64_t tp = j > 0 ? key_tile(keys[j - 1], c, tshift) : -2;
  const int64_t tn = j + 1 < c.ntot ? key_tile(keys[j + 1], c, tshift) : -2;
  if (tp != t) tstart[t] = (uint32_t)j;
  if (tn != t) tend[t] = (uint32_t)(j + 1);
}

// One record per occupied tile (a workgroup takes a whole tile, however many
// particles it holds), and the record of each tile in tslot.  The records
// are ordered by particle count, largest first, in buckets of 32 particles
// (kTileBuckets, the last open-ended): workgroups are dispatched in list
// order, so the longest tiles start first and the short ones fill the end of
// the launch (P2G 566 -> 532 us per launch on the 64-instance batch).
__device__ __forceinline__ int tile_bucket(uint32_t n) { return min(kTileBuckets - 1, (int)(n >> 5)); }

// Counts per bucket: a workgroup histogram in LDS, then one global add per
// bucket and workgroup.
__global__ void k_tile_buckets(int64_t total_tiles, const uint32_t* tstart, const uint32_t* tend, uint32_t* bucket) {
  __shared__ uint32_t h[kTileBuckets];
  if (threadIdx.x < kTileBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t e = t < total_tiles ? tend[t] : 0u;
  if (e != 0u) atomicAdd(&h[tile_bucket(e - tstart[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kTileBuckets && h[threadIdx.x] != 0u) atomicAdd(&bucket[threadIdx.x], h[threadIdx.x]);
}

// bucket[0, B): counts -> bucket[B, 2B): first record of each bucket, the
// largest bucket first; count = the number of records.
__global__ void k_tile_bucket_offsets(uint32_t* bucket, uint32_t* count) {
  if (threadIdx.x != 0) return;
  uint32_t acc = 0;
  for (int b = kTileBuckets - 1; b >= 0; --b) {
    bucket[kTileBuckets + b] = acc;
    acc += bucket[b];
  }
  *count = acc;
}

// Records: ranks within the workgroup from an LDS count per bucket, one
// global add per bucket and workgroup for the range of records.
__global__ void k_tile_list(int64_t total_tiles, const uint32_t* tstart, const uint32_t* tend, TileRec* list,
                            uint32_t* bucket, uint32_t* tslot) {
  __shared__ uint32_t h[kTileBuckets], base[kTileBuckets];
  if (threadIdx.x < kTileBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t e = t < total_tiles ? tend[t] : 0u;
  const uint32_t st = e != 0u ? tstart[t] : 0u;
  const int bk = tile_bucket(e - st);
  const uint32_t rank = e != 0u ? atomicAdd(&h[bk], 1u) : 0u;
  __syncthreads();
  if (threadIdx.x < kTileBuckets && h[threadIdx.x] != 0u)
    base[threadIdx.x] = atomicAdd(&bucket[kTileBuckets + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (e == 0u) return;
  const uint32_t idx = base[bk] + rank;
  list[idx] = TileRec{st, e, (uint32_t)t};
  tslot[t] = idx;
}

__global__ void k_tile_slots(TileList tl, int64_t max_records, uint32_t* tslot) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= max_records || r >= (int64_t)*tl.count) return;
  tslot[tl.list[r].tile] = (uint32_t)r;
}

void launch_tile_slots(const KCfg& c, const TileList& tl, int64_t max_records, uint32_t* tslot, hipStream_t s) {
  const int tshift = c.dim == 3 ? 6 : 4;
  const int64_t total_tiles = (c.nodes >> tshift) * c.n_inst;
  launch_fill_u32(tslot, total_tiles, kNoSlot, s);
  hipLaunchKernelGGL(k_tile_slots, dim3((unsigned)((max_records + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, tl,
                     max_records, tslot);
}

void launch_tile_list(const KCfg& c, const uint32_t* sorted_keys, uint32_t* tstart, uint32_t* tend, TileRec* list,
                      uint32_t* count, uint32_t* tslot, uint32_t* bucket, hipStream_t s) {
  const int tshift = c.dim == 3 ? 6 : 4;   // log2(kTile^D)
  const int64_t total_tiles = (c.nodes >> tshift) * c.n_inst;
  const unsigned ntb = (unsigned)((total_tiles + kBlock - 1) / kBlock);
  launch_fill_zero(tend, total_tiles, 4, s);
  launch_fill_zero(bucket, kTileBuckets, 4, s);
  launch_fill_u32(tslot, total_tiles, kNoSlot, s);
  hipLaunchKernelGGL(k_tile_bounds, dim3((unsigned)((c.ntot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, c,
                     sorted_keys, tshift, tstart, tend);
  hipLaunchKernelGGL(k_tile_buckets, dim3(ntb), dim3(kBlock), 0, s, total_tiles, tstart, tend, bucket);
  hipLaunchKernelGGL(k_tile_bucket_offsets, dim3(1), dim3(64), 0, s, bucket, count);
  hipLaunchKernelGGL(k_tile_list, dim3(ntb), dim3(kBlock), 0, s, total_tiles, tstart, tend, list, bucket, tslot);
}

// Active set after a binning: mark the 3^D blocks around every occupied tile,
// then list the marked blocks.
__global__ void k_mark_active(KCfg c, TileList tl, int64_t max_records, uint32_t* mask) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= max_records || r >= (int64_t)*tl.count) return;
  const int D = c.dim, nt = c.n / kTile;
  const uint32_t per = D == 3 ? (uint32_t)(nt * nt * nt) : (uint32_t)(nt * nt);
  const uint32_t gt = tl.list[r].tile;
  const uint32_t inst = gt / per;
  uint32_t t = gt - inst * per;
  int tc[3] = {0, 0, 0};
  for (int a = D - 1; a >= 0; --a) { tc[a] = (int)(t % (uint32_t)nt); t /= (uint32_t)nt; }
  for (int d0 = -1; d0 <= 1; ++d0)
    for (int d1 = -1; d1 <= 1; ++d1)
      for (int d2 = (D == 3 ? -1 : 0); d2 <= (D == 3 ? 1 : 0); ++d2) {
        const int q[3] = {tc[0] + d0, tc[1] + d1, tc[2] + d2};
        bool ok = true;
        for (int a = 0; a < D; ++a) ok &= q[a] >= 0 && q[a] < nt;
        if (!ok) continue;
        const uint32_t lb = D == 3 ? (uint32_t)((q[0] * nt + q[1]) * nt + q[2]) : (uint32_t)(q[0] * nt + q[1]);
        mask[inst * per + lb] = 1u;
      }
}

__global__ void k_list_active(int64_t total_tiles, const uint32_t* mask, uint32_t* list, uint32_t* count) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= total_tiles || mask[t] == 0u) return;
  list[atomicAdd(count, 1u)] = (uint32_t)t;
}

void launch_active_set(const KCfg& c, const TileList& tl, const ActiveSet& act, hipStream_t s) {
  const int tshift = c.dim == 3 ? 6 : 4;
  const int64_t total_tiles = (c.nodes >> tshift) * c.n_inst;
  const unsigned nb = (unsigned)((total_tiles + kBlock - 1) / kBlock);
  launch_fill_zero(act.mask, total_tiles, 4, s);
  launch_fill_zero(act.count, 1, 4, s);
  hipLaunchKernelGGL(k_mark_active, dim3(nb), dim3(kBlock), 0, s, c, tl, total_tiles, act.mask);
  hipLaunchKernelGGL(k_list_active, dim3(nb), dim3(kBlock), 0, s, total_tiles, act.mask, act.list, act.count);
}

}  // namespace ddm
