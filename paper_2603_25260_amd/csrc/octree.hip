// Octree construction, coordinate hash, 3x3x3 neighbourhoods and child
// expansion on gfx950 (Sec. S3.2 of the paper; neighbourhoods for the sparse
// convolutions of Sec. 3.3).  Integer-only; wave64 ballots and prefix counts.
#include <cstring>
#include <utility>

#include "lpcc_internal.h"

namespace lpcc {

// ---------------------------------------------------------------------------
// Morton keys: bit 3b+2 = x_b, 3b+1 = y_b, 3b = z_b, and a frame tag above
// the 3D coordinate bits so that several frames sort into one array.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

// ---------------------------------------------------------------------------
// LSD radix sort of the Morton keys (Sec. S3.2 sorts the coordinates in
// Morton order before the levels are derived).  Passes of at most 8 bits from
// the least significant end; each pass is stable, so the keys end sorted on
// all bits [0, end_bit).  A tile is kSortTile keys in striped order (item k of
// thread t is key k*256 + t of the tile).
// ---------------------------------------------------------------------------
SortPasses sort_passes(int end_bit) {
  SortPasses sp;
  memset(&sp, 0, sizeof(sp));
  end_bit = end_bit < 1 ? 1 : end_bit;
  sp.n = (end_bit + 7) / 8;
  const int w = (end_bit + sp.n - 1) / sp.n;
  for (int p = 0; p < sp.n; p++) {
    sp.shift[p] = p * w;
    sp.bits[p] = w < end_bit - p * w ? w : end_bit - p * w;
  }
  return sp;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift, int bits) {
  return (uint32_t)(key >> shift) & ((1u << bits) - 1u);
}

// Keys of the launch's frames: block b covers tile (first tile of the
// launch's key range) + b; its keys' pass-0 digits are counted per tile and
// every pass's digits in the totals (LDS first, then one global add per bin).
__global__ __launch_bounds__(256) void k_morton_sort0(const MortonFrames mf, int D, uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ err, const SortPasses sp,
                                                      uint32_t* __restrict__ hist, uint32_t* __restrict__ totals) {
  __shared__ uint32_t h[8][256];
  for (int k = threadIdx.x; k < 8 * 256; k += 256) (&h[0][0])[k] = 0u;
  __syncthreads();
  const int64_t lo = mf.start[0], hi = mf.start[mf.nf];
  const int64_t tile = lo / kSortTile + blockIdx.x;
  const uint32_t side = 1u << D;
  for (int k = 0; k < kSortItems; k++) {
    const int64_t i = tile * kSortTile + k * 256 + threadIdx.x;
    if (i < lo || i >= hi) continue;
    // frame of element i (constant indices into the argument arrays)
    int f = 0;
#pragma unroll
    for (int g = 1; g < kMortonGroup; g++)
      if (g < mf.nf && i >= mf.start[g]) f = g;
    const int32_t* src = mf.xyz[0];
    int64_t s0 = mf.start[0];
#pragma unroll
    for (int g = 1; g < kMortonGroup; g++)
      if (g == f) {
        src = mf.xyz[g];
        s0 = mf.start[g];
      }
    const GAS int32_t* p = gp(src) + 3 * (i - s0);
    int32_t x = p[0], y = p[1], z = p[2];
    if (x < 0 || y < 0 || z < 0 || (uint32_t)x >= side || (uint32_t)y >= side || (uint32_t)z >= side) {
      atomicOr(err + mf.f0 + f, ERR_COORD);
      x = y = z = 0;
    }
    const uint64_t tag = (uint64_t)(mf.f0 + f) << (3 * D);
    const uint64_t key = tag | (spread3((uint32_t)x) << 2) | (spread3((uint32_t)y) << 1) | spread3((uint32_t)z);
    gp(keys)[i] = key;
    for (int q = 0; q < sp.n; q++) atomicAdd(&h[q][digit_of(key, sp.shift[q], sp.bits[q])], 1u);
  }
  __syncthreads();
  const int b = threadIdx.x;
  for (int q = 0; q < sp.n; q++) {
    const uint32_t v = h[q][b];
    if (!v) continue;
    atomicAdd(totals + q * 256 + b, v);
    if (q == 0) atomicAdd(hist + tile * 256 + b, v);
  }
}

hipError_t launch_morton_sort0(const MortonFrames& mf, int D, uint64_t* keys, uint32_t* err, const SortPasses& sp,
                               uint32_t* hist, uint32_t* totals, hipStream_t s) {
  const int64_t lo = mf.start[0], hi = mf.start[mf.nf];
  if (hi <= lo) return hipSuccess;
  const int64_t blocks = (hi - 1) / kSortTile - lo / kSortTile + 1;
  hipLaunchKernelGGL(k_morton_sort0, dim3((unsigned)blocks), dim3(256), 0, s, mf, D, keys, err, sp, hist, totals);
  return hipGetLastError();
}

// In place: hist[t][d] <- first destination of tile t's keys of digit d
// (digits ascending, tiles ascending within a digit).  Block d scans digit
// d over the tiles: each thread sums a run of tiles, the 256 run sums are
// scanned in the block, and the runs are rewritten as running offsets
// starting from the digit's base (the keys of all smaller digits).
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* __restrict__ hist, int ntiles,
                                                   const uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t base;
  const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // base of digit d: the sum of the totals of the smaller digits
  const uint32_t tv = tid < d ? gp(totals)[tid] : 0u;
  const uint32_t bi = wave_scan_incl(tv);
  if (lane == 63) wsum[wave] = bi;
  __syncthreads();
  if (tid == 0) base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  const uint32_t b0 = base;
  __syncthreads();
  const int per = (ntiles + 255) / 256;
  const int t0 = min(ntiles, tid * per), t1 = min(ntiles, t0 + per);
  uint32_t sum = 0;
  for (int t = t0; t < t1; t++) sum += gp(hist)[(int64_t)t * 256 + d];
  const uint32_t inc = wave_scan_incl(sum);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off = b0 + inc - sum;
  for (int w = 0; w < wave; w++) off += wsum[w];
  for (int t = t0; t < t1; t++) {
    const int64_t o = (int64_t)t * 256 + d;
    const uint32_t v = gp(hist)[o];
    gp(hist)[o] = off;
    off += v;
  }
}

// Digit counts of one pass per tile of kSortTile keys (LDS histogram, one
// store per bin).
__global__ __launch_bounds__(256) void k_sort_count(const uint64_t* __restrict__ kin, int64_t n, int shift, int bits,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t tile = blockIdx.x;
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    const int64_t i = tile * kSortTile + k * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(gp(kin)[i], shift, bits)], 1u);
  }
  __syncthreads();
  gp(hist)[tile * 256 + threadIdx.x] = h[threadIdx.x];
}

// One pass: every key's destination is the first destination of its tile's
// digit plus its rank among the tile's keys of that digit.  Ranks within a
// wave come from a ballot match over the digit bits; the counts of every
// (item, wave, digit) are turned into running offsets by one thread per
// digit.  With offs_ready the tile offsets come from k_sort_scan, else the
// pass sums the counts of the tiles before it and the totals of the smaller
// digits itself; such small sorts also add the next pass's digit counts per
// destination tile here (few tiles: few contended counters), larger ones
// count them in a pass of their own.
__global__ __launch_bounds__(256) void k_sort_scatter(const uint64_t* __restrict__ kin, uint64_t* __restrict__ kout,
                                                      int64_t n, int shift, int bits, const uint32_t* __restrict__ hist,
                                                      int offs_ready, const uint32_t* __restrict__ totals,
                                                      uint32_t* __restrict__ hist_next, int shift_n, int bits_n,
                                                      uint32_t* __restrict__ err) {
  __shared__ uint32_t cnt[kSortItems][4][256];
  __shared__ uint32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = blockIdx.x;
  for (int k = tid; k < kSortItems * 4 * 256; k += 256) (&cnt[0][0][0])[k] = 0u;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint64_t key[kSortItems];
  uint32_t dig[kSortItems], rk[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    const int64_t i = tile * kSortTile + k * 256 + tid;
    key[k] = i < n ? gp(kin)[i] : 0ull;
    dig[k] = digit_of(key[k], shift, bits);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    const bool valid = tile * kSortTile + k * 256 + tid < n;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; b++) {
      const bool bit = (dig[k] >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    rk[k] = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0ull) cnt[k][wave][dig[k]] = (uint32_t)__popcll(peers);
  }
  // first destination of digit `tid` in this tile
  const uint32_t tot = gp(totals)[tid];
  const uint32_t inc = wave_scan_incl(tot);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off;
  if (offs_ready) {
    off = gp(hist)[tile * 256 + tid];
  } else {
    off = inc - tot;
    for (int w = 0; w < wave; w++) off += wsum[w];
    for (int64_t t = 0; t < tile; t++) off += gp(hist)[t * 256 + tid];
  }
#pragma unroll
  for (int k = 0; k < kSortItems; k++)
#pragma unroll
    for (int w = 0; w < 4; w++) {
      const uint32_t c = cnt[k][w][tid];
      cnt[k][w][tid] = off;
      off += c;
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    if (tile * kSortTile + k * 256 + tid >= n) continue;
    const uint64_t dest = (uint64_t)cnt[k][wave][dig[k]] + rk[k];
    if (dest >= (uint64_t)n) {  // only if the counts were inconsistent
      atomicOr(err, ERR_SORT);
      continue;
    }
    gp(kout)[dest] = key[k];
    if (hist_next != nullptr)
      atomicAdd(hist_next + (dest / kSortTile) * 256 + digit_of(key[k], shift_n, bits_n), 1u);
  }
}

hipError_t launch_sort_pass(const uint64_t* kin, uint64_t* kout, int64_t n, const SortPasses& sp, int p,
                            uint32_t* hist, const uint32_t* totals, uint32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  uint32_t* hp = hist + (int64_t)p * ntiles * 256;
  const bool scan = ntiles > kSortFusedTiles;
  const bool last = p + 1 >= sp.n;
  // pass 0's per-tile counts come with the keys; a large sort counts every
  // later pass over the order the previous pass left, a small one had them
  // added by the previous pass
  if (p > 0 && scan)
    hipLaunchKernelGGL(k_sort_count, dim3((unsigned)ntiles), dim3(256), 0, s, kin, n, sp.shift[p], sp.bits[p], hp);
  if (scan) hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, hp, (int)ntiles, totals + p * 256);
  uint32_t* next = (!scan && !last) ? hp + ntiles * 256 : nullptr;
  hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)ntiles), dim3(256), 0, s, kin, kout, n, sp.shift[p], sp.bits[p],
                     (const uint32_t*)hp, scan ? 1 : 0, totals + p * 256, next, last ? 0 : sp.shift[p + 1],
                     last ? 0 : sp.bits[p + 1], err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Level build over sorted keys.  For element i let d*(i) be the shallowest
// depth at which it starts a new node: 0 at a frame start (the tags differ),
// D+1 for a duplicate, else D - floor(b/3) with b the highest bit in which it
// differs from its predecessor.  Element i is the first element of a depth-d
// node iff d*(i) <= d, so node indices are prefix counts of (d* <= d).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dstar(const uint64_t* keys, int64_t i, int D) {
  if (i == 0) return 0;
  uint64_t x = keys[i] ^ keys[i - 1];
  if (x == 0) return D + 1;
  int b = 63 - __clzll((long long)x);
  int d = D - b / 3;
  return d < 0 ? 0 : d;
}

constexpr int kLevelThreads = 256;


// hist[tile][v] = #elements of the tile with d* <= v (v = 0..D)
__global__ void k_level_hist(const uint64_t* __restrict__ keys, int64_t n, int D, int tile,
                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kMaxD + 2];
  for (int v = threadIdx.x; v <= D + 1; v += blockDim.x) h[v] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * tile;
  for (int k = threadIdx.x; k < tile; k += blockDim.x) {
    int64_t i = base + k;
    if (i < n) atomicAdd(&h[dstar(keys, i, D)], 1u);
  }
  __syncthreads();
  // cumulative over depth: hist[tile][d] = #elements of the tile with d* <= d
  for (int v = threadIdx.x; v <= D; v += blockDim.x) {
    uint32_t c = 0;
    for (int u = 0; u <= v; u++) c += h[u];
    hist[(int64_t)blockIdx.x * (D + 1) + v] = c;
  }
}

hipError_t launch_level_hist(const uint64_t* keys, int64_t n, int D, int tile, uint32_t* hist, hipStream_t s) {
  int64_t nb = (n + tile - 1) / tile;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_hist, dim3((unsigned)nb), dim3(kLevelThreads), 0, s, keys, n, D, tile, hist);
  return hipGetLastError();
}

// In place: hist[t][d] <- #elements of tiles < t with d* <= d (exclusive over
// tiles; the histogram is already cumulative over depth).  totals[d] = N_d.
// One block per depth, so the depths are scanned side by side: every thread
// sums a run of tiles, a block-wide exclusive scan (wave shuffles, then the
// four wave totals) gives each run its offset, the run is rewritten.
__global__ __launch_bounds__(kLevelThreads) void k_level_scan(uint32_t* __restrict__ hist, int nb, int D,
                                                             uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[kLevelThreads / 64];
  const int d = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nb + kLevelThreads - 1) / kLevelThreads;
  const int t0 = tid * per, t1 = min(nb, t0 + per);
  uint32_t run = 0;
  for (int t = t0; t < t1; t++) run += hist[(int64_t)t * (D + 1) + d];
  const uint32_t inc = wave_scan_incl(run);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t ex = inc - run;
  for (int w = 0; w < wave; w++) ex += wsum[w];
  if (tid == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kLevelThreads / 64; w++) tot += wsum[w];
    totals[d] = tot;
  }
  for (int t = t0; t < t1; t++) {
    const int64_t o = (int64_t)t * (D + 1) + d;
    const uint32_t v = hist[o];
    hist[o] = ex;
    ex += v;
  }
}

hipError_t launch_level_scan(uint32_t* hist, int nb, int D, uint32_t* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_level_scan, dim3(D + 1), dim3(kLevelThreads), 0, s, hist, nb, D, totals);
  return hipGetLastError();
}

// Writes, for every depth d, the node keys V_d (key >> 3(D-d), tag kept),
// the occupancy codes X_{d} (atomic OR of 1 << child slot into the parent's
// byte) and the first-child index of every node.  Tiles hold `tile`
// elements, processed in rounds of 256 in order.
__global__ void k_level_write(const uint64_t* __restrict__ keys, int64_t n, int D, int tile,
                              const uint32_t* __restrict__ offs, const uint32_t* __restrict__ totals,
                              LevelOut lo) {
  __shared__ uint32_t wtot[4][kMaxD + 1];
  __shared__ uint32_t run[kMaxD + 1];
  // occupancy words of the round's parents, combined here before one global
  // OR per word: the parents of a round's 256 elements at depth d-1 span at
  // most 256 consecutive nodes, i.e. at most 65 words from word wb[d]
  constexpr int kCW = 66;
  __shared__ uint32_t cw[kMaxD + 1][kCW];
  __shared__ uint32_t wb[kMaxD + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  if (threadIdx.x <= D) run[threadIdx.x] = offs[(int64_t)blockIdx.x * (D + 1) + threadIdx.x];
  // cstart[d][N_d] = N_{d+1}: the sentinel after the last node of every depth
  if (blockIdx.x == 0 && threadIdx.x < D) {
    const uint32_t nd = totals[threadIdx.x], nd1 = totals[threadIdx.x + 1];
#pragma unroll
    for (int d = 0; d < kMaxD; d++)  // constant indices into the pointer table
      if (d == (int)threadIdx.x) lo.cstart[d][nd] = (int32_t)nd1;
  }
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * tile;
  for (int k0 = 0; k0 < tile; k0 += blockDim.x) {
    int64_t i = base + k0 + threadIdx.x;
    bool valid = i < n;
    int ds = valid ? dstar(keys, i, D) : D + 2;
    uint64_t key = valid ? keys[i] : 0;
    uint32_t excl[kMaxD + 1];
    for (int d = 0; d <= D; d++) {
      uint64_t m = __ballot(ds <= d);
      excl[d] = __popcll(m & lt);
      if (lane == 0) wtot[wave][d] = __popcll(m);
    }
    for (int k = threadIdx.x; k < (D + 1) * kCW; k += blockDim.x) cw[k / kCW][k % kCW] = 0;
    __syncthreads();
    uint32_t node[kMaxD + 1];
    if (valid) {
      for (int d = 0; d <= D; d++) {
        uint32_t before = run[d];
        for (int w = 0; w < wave; w++) before += wtot[w][d];
        // index of the depth-d node holding element i
        node[d] = before + excl[d] + (ds <= d ? 1u : 0u) - 1u;
      }
      // the round's first element holds the lowest parent of every depth
      if (threadIdx.x == 0)
        for (int d = 1; d <= D; d++) wb[d] = node[d - 1] >> 2;
    }
    __syncthreads();
    if (valid) {
      if (ds == 0) {  // first element of a frame: record its node per depth
        const uint64_t f = (3 * D >= 64) ? 0 : (key >> (3 * D));
        for (int d = 0; d <= D; d++) lo.frame_off[f * (D + 1) + d] = node[d];
      }
      for (int d = 0; d <= D; d++) {
        if (ds > d) continue;
        lo.key[d][node[d]] = key >> (3 * (D - d));
        if (d < D) lo.cstart[d][node[d]] = (int32_t)node[d + 1];
        if (d >= 1) {
          uint32_t slot = (uint32_t)((key >> (3 * (D - d))) & 7u);
          uint32_t p = node[d - 1];
          atomicOr(&cw[d][(p >> 2) - wb[d]], (1u << slot) << (8 * (p & 3u)));
        }
      }
    }
    __syncthreads();
    // one global OR per touched word (words at the round's edges may be
    // shared with the neighbouring rounds and blocks)
    for (int k = threadIdx.x; k < D * kCW; k += blockDim.x) {
      const int d = 1 + k / kCW, w = k % kCW;
      const uint32_t v = cw[d][w];
      if (v) atomicOr((uint32_t*)(lo.code[d - 1]) + wb[d] + w, v);
    }
    __syncthreads();
    if (threadIdx.x <= D) {
      uint32_t add = 0;
      for (int w = 0; w < 4; w++) add += wtot[w][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

hipError_t launch_level_write(const uint64_t* keys, int64_t n, int D, int tile, const uint32_t* hist,
                              const uint32_t* totals, const LevelOut& lo, hipStream_t s) {
  int64_t nb = (n + tile - 1) / tile;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_write, dim3((unsigned)nb), dim3(kLevelThreads), 0, s, keys, n, D, tile, hist, totals,
                     lo);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota_u64(uint64_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint64_t)i;
}
hipError_t launch_iota_u64(uint64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coordinate hash: open addressing, linear probing, 2^k >= 2N slots of
// {u64 key, i32 row}; empty slots hold all-ones.  Lookups return the same
// row whatever the insertion order.
// ---------------------------------------------------------------------------
constexpr uint64_t kEmpty = ~0ull;
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t hmix(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ uint64_t hslot(uint64_t k, uint64_t mask) { return hmix(k) & mask; }

__device__ __forceinline__ void hash_put(uint64_t k, int32_t row, uint64_t* table, uint64_t mask) {
  uint64_t slot = hslot(k, mask);
  for (uint64_t probe = 0; probe <= mask; probe++) {
    unsigned long long prev = kEmpty;
    __hip_atomic_compare_exchange_strong((GAS unsigned long long*)&table[2 * slot], &prev, (unsigned long long)k,
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == kEmpty || prev == k) {
      ((GAS int32_t*)(table + 2 * slot + 1))[0] = row;
      return;
    }
    slot = (slot + 1) & mask;
  }
}

__global__ void k_hash_insert(const uint64_t* __restrict__ keys, int64_t n, uint64_t* table, uint64_t mask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  hash_put(keys[i], (int32_t)i, table, mask);
}

hipError_t launch_hash_insert(const uint64_t* keys, int64_t n, uint64_t* table, uint64_t mask, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_insert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, table, mask);
  return hipGetLastError();
}

// Neighbour table: a wave serves two nodes, lanes 0-26 and 32-58 one tap
// each: neighbour (dx,dy,dz) of tap 9(dx+1)+3(dy+1)+(dz+1).
// kmap[tap * kstride + node] = the neighbour's row, or -1 when empty or
// outside [0,2^j)^3; kmap[27 * kstride + node] = the node's presence mask
// (bit tap set when that neighbour exists; the node itself is tap 13),
// gathered from the wave's ballot.  Every lane probes on its own, so the
// probes of a node are in flight together.
__device__ __forceinline__ void kmap_pair(const uint64_t* __restrict__ keys, int64_t n, int64_t wv, int j,
                                          const uint64_t* __restrict__ table, uint64_t mask,
                                          int32_t* __restrict__ kmap, int64_t kstride) {
  const int lane = threadIdx.x & 63;
  const int64_t i = 2 * wv + (lane >> 5);
  const int t = lane & 31;
  const bool valid = t < 27 && i < n;
  int32_t r = -1;
  if (valid) {
    const uint64_t key = gp(keys)[i];
    const uint64_t low = j > 0 ? (key & ((1ull << (3 * j)) - 1)) : 0;
    const uint64_t tag = key ^ low;
    const int x = (int)compact3(low >> 2) + t / 9 - 1;
    const int y = (int)compact3(low >> 1) + (t / 3) % 3 - 1;
    const int z = (int)compact3(low) + t % 3 - 1;
    const int side = 1 << j;
    if (x >= 0 && y >= 0 && z >= 0 && x < side && y < side && z < side) {
      const uint64_t q = tag | (spread3((uint32_t)x) << 2) | (spread3((uint32_t)y) << 1) | spread3((uint32_t)z);
      uint64_t slot = hslot(q, mask);
      for (uint64_t probe = 0; probe <= mask; probe++) {
        const u64x2 e = ((const GAS u64x2*)table)[slot];
        if (e.x == q) {
          r = (int32_t)(uint32_t)e.y;
          break;
        }
        if (e.x == kEmpty) break;
        slot = (slot + 1) & mask;
      }
    }
    gp(kmap)[(int64_t)t * kstride + i] = r;
  }
  const uint64_t m = __ballot(r >= 0);
  if (t == 0 && i < n) gp(kmap)[27 * kstride + i] = (int32_t)(uint32_t)(m >> (lane & 32));
}

__global__ __launch_bounds__(256) void k_kmap(const uint64_t* __restrict__ keys, int64_t n, int j,
                                              const uint64_t* __restrict__ table, uint64_t mask,
                                              int32_t* __restrict__ kmap, int64_t kstride) {
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (2 * wv >= n) return;  // wave-uniform
  kmap_pair(keys, n, wv, j, table, mask, kmap, kstride);
}

// Several depths per launch: block b belongs to the last job whose first
// block is <= b (jobs are in increasing block order).
__device__ __forceinline__ int job_of(const HashJob* __restrict__ jobs, int njobs, bool kmap_blocks) {
  int q = 0;
  for (int k = 1; k < njobs; k++) {
    const int b0 = kmap_blocks ? jobs[k].blk_kmap : jobs[k].blk_insert;
    if ((int)blockIdx.x >= b0) q = k;
  }
  return q;
}

__global__ __launch_bounds__(kHashBlock) void k_hash_insert_multi(const HashJob* __restrict__ jobs, int njobs) {
  const HashJob J = jobs[job_of(jobs, njobs, false)];
  const int64_t i = (int64_t)((int)blockIdx.x - J.blk_insert) * kHashBlock + threadIdx.x;
  if (i >= J.n) return;
  hash_put(gp(J.keys)[i], (int32_t)i, J.table, J.mask);
}

__global__ __launch_bounds__(kHashBlock) void k_kmap_multi(const HashJob* __restrict__ jobs, int njobs) {
  const HashJob J = jobs[job_of(jobs, njobs, true)];
  const int64_t wv = ((int64_t)((int)blockIdx.x - J.blk_kmap) * kHashBlock + threadIdx.x) >> 6;
  if (2 * wv >= J.n) return;  // wave-uniform
  kmap_pair(J.keys, J.n, wv, J.j, J.table, J.mask, J.kmap, J.kstride);
}

hipError_t launch_hash_multi(const HashJob* jobs_dev, int njobs, int insert_blocks, int kmap_blocks,
                             hipStream_t s) {
  if (njobs <= 0 || insert_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_insert_multi, dim3(insert_blocks), dim3(kHashBlock), 0, s, jobs_dev, njobs);
  hipLaunchKernelGGL(k_kmap_multi, dim3(kmap_blocks), dim3(kHashBlock), 0, s, jobs_dev, njobs);
  return hipGetLastError();
}

hipError_t launch_kmap(const uint64_t* keys, int64_t n, int j, const uint64_t* table, uint64_t mask,
                       int32_t* kmap, int64_t kstride, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kmap, dim3((unsigned)((n + 7) / 8)), dim3(256), 0, s, keys, n, j, table, mask, kmap,
                     kstride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Neighbour table of depth j from the table of depth j-1, without a hash.
// The neighbour of child c (slot o of parent p) at offset delta lies, per
// axis, in the depth-(j-1) cell p + floor((o + delta) / 2), in that cell's
// child slot (o + delta) mod 2.  The cell is p's own neighbour at that offset
// (the table of depth j-1), and the child exists when that slot's bit is set
// in the cell's occupancy code; its row is the cell's first-child row plus
// the number of set bits below the slot, since children are stored in
// ascending slot order (Sec. S3.2).  Cells outside the cube are absent at
// depth j-1, so their children are absent too: the table equals the one the
// hash lookups give, entry for entry.
//
// A block takes kTreeParents consecutive parents; their children are the
// consecutive rows [cstart[p0], cstart[p_end]).  One lane per child reads the
// 2x2x2 cells its 27 neighbours fall in: cell a = (ax, ay, az) in {0,1}^3
// sits at parent offset (o - 1 + a) per axis, tap 9(ox+ax) + 3(oy+ay) +
// (oz+az) of the parent.  The stores are coalesced: lanes hold consecutive
// rows of one tap.
// ---------------------------------------------------------------------------
constexpr int kTreeParents = 256;

// Cell index along one axis for child-tap component T (0, 1, 2 = delta -1,
// 0, +1) of a child at slot bit o: delta -1 stays in cell 0, +1 in cell 1,
// and 0 in cell 1 - o; the slot inside the cell is o for T = 1, else 1 - o.
template <int T>
__device__ __forceinline__ int tree_cell(int o) { return T == 0 ? 0 : (T == 2 ? 1 : 1 - o); }
template <int T>
__device__ __forceinline__ int tree_slot(int o) { return T == 1 ? o : 1 - o; }

template <int TX, int TY, int TZ>
__device__ __forceinline__ int32_t tree_row(const uint32_t (&cc)[8], const int32_t (&cs)[8], int ox, int oy,
                                            int oz) {
  const int a = tree_cell<TX>(ox) * 4 + tree_cell<TY>(oy) * 2 + tree_cell<TZ>(oz);
  // select the cell by explicit compares (an index into a register array
  // would go through scratch); cells this tap cannot reach fold away
  uint32_t code = cc[(TX == 2 ? 4 : 0) + (TY == 2 ? 2 : 0) + (TZ == 2 ? 1 : 0)];
  int32_t first = cs[(TX == 2 ? 4 : 0) + (TY == 2 ? 2 : 0) + (TZ == 2 ? 1 : 0)];
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const bool reach = (TX == 1 || ((k >> 2) & 1) == (TX == 2)) && (TY == 1 || ((k >> 1) & 1) == (TY == 2)) &&
                       (TZ == 1 || (k & 1) == (TZ == 2));
    if (reach) {
      code = a == k ? cc[k] : code;
      first = a == k ? cs[k] : first;
    }
  }
  const int s = tree_slot<TX>(ox) * 4 + tree_slot<TY>(oy) * 2 + tree_slot<TZ>(oz);
  return ((code >> s) & 1u) ? first + __popc(code & ((1u << s) - 1u)) : -1;
}

// A row at or past the depth's node count (kstride) only arises when the
// decoded codes claim more children than the stream's header (a corrupt
// stream or the wrong model): it is stored as absent, so that no gather
// reads past the depth's feature rows (the hash lookups can only return
// inserted rows).
template <int T>
__device__ __forceinline__ void tree_tap(const uint32_t (&cc)[8], const int32_t (&cs)[8], int ox, int oy, int oz,
                                         GAS int32_t* __restrict__ out, int64_t kstride, uint32_t& m) {
  int32_t r = tree_row<T / 9, (T / 3) % 3, T % 3>(cc, cs, ox, oy, oz);
  r = (r >= 0 && (int64_t)r < kstride) ? r : -1;
  out[(int64_t)T * kstride] = r;
  m |= (r >= 0 ? 1u : 0u) << T;
}

template <int... T>
__device__ __forceinline__ void tree_taps(std::integer_sequence<int, T...>, const uint32_t (&cc)[8],
                                          const int32_t (&cs)[8], int ox, int oy, int oz,
                                          GAS int32_t* __restrict__ out, int64_t kstride, uint32_t& m) {
  (tree_tap<T>(cc, cs, ox, oy, oz, out, kstride, m), ...);
}

__global__ __launch_bounds__(256) void k_kmap_tree(const int32_t* __restrict__ pkmap, int64_t pstride,
                                                   const uint8_t* __restrict__ pcode,
                                                   const int32_t* __restrict__ pcstart, int64_t np,
                                                   int32_t* __restrict__ kmap, int64_t kstride) {
  __shared__ uint16_t who[8 * kTreeParents];  // (parent in block << 3) | slot, per child row
  const int64_t p0 = (int64_t)blockIdx.x * kTreeParents;
  const int64_t pe = min(p0 + (int64_t)kTreeParents, np);
  const int64_t p = p0 + threadIdx.x;
  const int32_t c0 = gp(pcstart)[p0];
  // children past the table (a stream whose codes claim more children than
  // its header) are not written; the expansion reports that stream
  const int64_t c1 = min((int64_t)gp(pcstart)[pe], kstride);
  if (p < pe) {
    uint32_t code = gp(pcode)[p];
    int32_t r = gp(pcstart)[p] - c0;
    while (code) {
      if (r >= 0 && r < 8 * kTreeParents) who[r] = (uint16_t)((threadIdx.x << 3) | (__ffs(code) - 1));
      r++;
      code &= code - 1;
    }
  }
  __syncthreads();
  const int nk = (int)min(c1 - (int64_t)c0, (int64_t)8 * kTreeParents);
  for (int k = threadIdx.x; k < nk; k += 256) {
    const uint32_t w = who[k];
    if ((int64_t)(w >> 3) >= pe - p0) continue;  // only with codes and first-child rows that disagree
    const int64_t pp = p0 + (w >> 3);
    const int ox = (w >> 2) & 1, oy = (w >> 1) & 1, oz = w & 1;
    const int tb = ox * 9 + oy * 3 + oz;
    int32_t q[8];
#pragma unroll
    for (int a = 0; a < 8; a++) q[a] = gp(pkmap)[(int64_t)(tb + (a >> 2) * 9 + ((a >> 1) & 1) * 3 + (a & 1)) * pstride + pp];
    uint32_t cc[8];
    int32_t cs[8];
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const int32_t qi = q[a] >= 0 ? q[a] : 0;  // absent cells read row 0 and are masked
      const uint32_t c = gp(pcode)[qi];
      cs[a] = gp(pcstart)[qi];
      cc[a] = q[a] >= 0 ? c : 0u;
    }
    uint32_t m = 0;
    GAS int32_t* out = gp(kmap) + c0 + k;
    tree_taps(std::make_integer_sequence<int, 27>{}, cc, cs, ox, oy, oz, out, kstride, m);
    out[27 * kstride] = (int32_t)m;
  }
}

hipError_t launch_kmap_tree(const int32_t* pkmap, int64_t np, const uint8_t* pcode, const int32_t* pcstart,
                            int32_t* kmap, int64_t n, hipStream_t s) {
  if (n <= 0 || np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kmap_tree, dim3((unsigned)((np + kTreeParents - 1) / kTreeParents)), dim3(256), 0, s, pkmap,
                     np, pcode, pcstart, np, kmap, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Child expansion (decode): children of parent p are (key_p << 3) | o for the
// set bits o of X[p], ascending, which keeps Morton order (Sec. S3.2).
// ---------------------------------------------------------------------------
// In place: per-chunk child counts -> exclusive offsets; checks the total.

__global__ void k_expand_scan(uint32_t* __restrict__ sums, int nb, int64_t expected, uint32_t* err) {
  __shared__ uint32_t part[256];
  int tid = threadIdx.x;
  int per = (nb + 255) / 256;
  int t0 = tid * per, t1 = min(nb, t0 + per);
  uint32_t run = 0;
  for (int t = t0; t < t1; t++) run += sums[t];
  part[tid] = run;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < 256; k++) { uint32_t v = part[k]; part[k] = acc; acc += v; }
    if ((int64_t)acc != expected) atomicOr(err, ERR_COUNT);
  }
  __syncthreads();
  uint32_t acc = part[tid];
  for (int t = t0; t < t1; t++) { uint32_t v = sums[t]; sums[t] = acc; acc += v; }
}

// One block per decoded chunk.  The chunk's first child row is the sum of
// the child counts of the chunks before it: summed here when there are few
// chunks, else `csum` already holds exclusive offsets (k_expand_scan).
constexpr int kExpandDirect = 2048;

__global__ __launch_bounds__(256) void k_expand_chunks(const Chunk* __restrict__ chunks, int nchunks,
                                                       const uint64_t* __restrict__ pkeys,
                                                       const uint8_t* __restrict__ codes, int64_t n,
                                                       const uint32_t* __restrict__ csum, int sums_are_offsets,
                                                       uint64_t* __restrict__ ckeys, int32_t* __restrict__ cstart,
                                                       int64_t expected, uint64_t* table, uint64_t mask,
                                                       uint32_t* err) {
  __shared__ uint32_t wtot[4];
  __shared__ uint32_t run;
  __shared__ uint64_t kids[8 * 256];  // child keys of the current round, in child order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cb = blockIdx.x;
  const Chunk ch = chunks[cb];
  // the first round's codes and parent keys are requested before the child
  // offset of the chunk is summed, so the two memory round trips overlap
  const int64_t i_first = ch.node0 + threadIdx.x;
  const bool v_first = (int)threadIdx.x < ch.count && i_first < n;
  const uint32_t code_first = v_first ? codes[i_first] : 0u;
  const uint64_t pk_first = v_first ? pkeys[i_first] : 0ull;
  if (sums_are_offsets) {
    if (threadIdx.x == 0) run = csum[cb];
  } else {
    uint32_t part = 0;
    for (int k = threadIdx.x; k < cb; k += 256) part += csum[k];
    part = wave_scan_incl(part);  // lane 63: the wave's sum
    if (lane == 63) wtot[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) run = wtot[0] + wtot[1] + wtot[2] + wtot[3];
  }
  __syncthreads();
  for (int k0 = 0; k0 < ch.count; k0 += 256) {
    const int64_t i = ch.node0 + k0 + threadIdx.x;
    const bool valid = k0 + (int)threadIdx.x < ch.count && i < n;
    const uint32_t code = k0 == 0 ? code_first : (valid ? codes[i] : 0u);
    const uint32_t c = __popc(code);
    const uint32_t inc = wave_scan_incl(c);
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t before = run;
    for (int w = 0; w < wave; w++) before += wtot[w];
    const uint32_t first = before + inc - c;
    const uint32_t r0 = run;  // first child of this round
    if (valid) {
      cstart[i] = (int32_t)first;
      const uint64_t pk = k0 == 0 ? pk_first : pkeys[i];
      uint32_t r = first - r0;
      for (int o = 0; o < 8; o++)
        if ((code >> o) & 1u) kids[r++] = (pk << 3) | (uint64_t)o;
      if (i == n - 1) {
        cstart[n] = (int32_t)(first + c);
        if ((int64_t)(first + c) != expected) atomicOr(err, ERR_COUNT);
      }
    }
    __syncthreads();
    // one thread per child: coalesced key stores and independent insertions
    const uint32_t nk = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    for (uint32_t j = threadIdx.x; j < nk; j += 256) {
      const uint32_t r = r0 + j;
      if ((int64_t)r >= expected) break;
      const uint64_t k = kids[j];
      ckeys[r] = k;
      if (table != nullptr) hash_put(k, (int32_t)r, table, mask);
    }
    __syncthreads();
    if (threadIdx.x == 0) run = r0 + nk;
    __syncthreads();
  }
}

hipError_t launch_expand_chunks(const Chunk* chunks, int nchunks, const uint64_t* pkeys, const uint8_t* codes,
                                int64_t n, uint32_t* csum, uint64_t* ckeys, int32_t* cstart,
                                int64_t n_child_expected, uint64_t* table, uint64_t mask, uint32_t* err,
                                hipStream_t s) {
  if (nchunks <= 0 || n <= 0) return hipSuccess;
  int offs = 0;
  if (nchunks > kExpandDirect) {
    hipLaunchKernelGGL(k_expand_scan, dim3(1), dim3(256), 0, s, csum, nchunks, n_child_expected, err);
    offs = 1;
  }
  hipLaunchKernelGGL(k_expand_chunks, dim3(nchunks), dim3(256), 0, s, chunks, nchunks, pkeys, codes, n,
                     (const uint32_t*)csum, offs, ckeys, cstart, n_child_expected, table, mask, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Base geometry (the levels that are not modelled are coded from the
// frequencies of their own symbols).  One thread per base node.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int base_depth_of(const BaseLevels& bl, int64_t i) {
  int d = 0;
  while (d + 1 < bl.nb && i >= bl.start[d + 1]) d++;
  return d;
}

__global__ void k_base_hist(const BaseLevels bl, uint32_t* __restrict__ hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bl.start[bl.nb]) return;
  const int d = base_depth_of(bl, i);
  const int64_t k = i - bl.start[d];
  if (bl.count != nullptr && k >= (int64_t)gp(bl.count)[d]) return;
  const int f = (int)(gp(bl.key[d])[k] >> (3 * d));
  if (f >= bl.nf) return;
  atomicAdd(&hist[((int64_t)f * bl.nb + d) * 256 + gp(bl.code[d])[k]], 1u);
}

hipError_t launch_base_hist(const BaseLevels& bl, uint32_t* hist, hipStream_t s) {
  const int64_t n = bl.start[bl.nb];
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_base_hist, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bl, hist);
  return hipGetLastError();
}

__global__ void k_base_sf(const BaseLevels bl, const int32_t* __restrict__ cdf, uint32_t* __restrict__ sf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bl.start[bl.nb]) return;
  const int d = base_depth_of(bl, i);
  const int64_t k = i - bl.start[d];
  const int f = min((int)(gp(bl.key[d])[k] >> (3 * d)), bl.nf - 1);
  const GAS int32_t* row = gp(cdf) + ((int64_t)f * bl.nb + d) * 256;
  const int sym = max((int)gp(bl.code[d])[k] - 1, 0);
  const uint32_t lo = (uint32_t)row[sym], hi = (uint32_t)row[sym + 1];
  gp(sf)[i] = lo | ((hi - lo) << 16);
}

hipError_t launch_base_sf(const BaseLevels& bl, const int32_t* cdf, uint32_t* sf, hipStream_t s) {
  const int64_t n = bl.start[bl.nb];
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_base_sf, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bl, cdf, sf);
  return hipGetLastError();
}

// 64 lanes per node, 8 bytes each
__global__ void k_base_rows(const uint64_t* __restrict__ keys, int64_t n, int d, int nb, int nf,
                            const uint16_t* __restrict__ rows16, uint16_t* __restrict__ cdf16) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t >> 6;
  const int l = (int)(t & 63);
  if (i >= n) return;
  const int f = min((int)(gp(keys)[i] >> (3 * d)), nf - 1);
  const GAS uint64_t* src = (const GAS uint64_t*)(rows16 + ((int64_t)f * nb + d) * 256);
  ((GAS uint64_t*)(cdf16 + i * 256))[l] = src[l];
}

hipError_t launch_base_rows(const uint64_t* keys, int64_t n, int d, int nb, int nf, const uint16_t* rows16,
                            uint16_t* cdf16, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_base_rows, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, keys, n, d, nb, nf,
                     rows16, cdf16);
  return hipGetLastError();
}

__global__ void k_keys_to_xyz(const uint64_t* __restrict__ keys, int64_t n, int D, int32_t* __restrict__ xyz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i] & ((D >= 21) ? ~0ull : ((1ull << (3 * D)) - 1));
  xyz[3 * i] = (int32_t)compact3(k >> 2);
  xyz[3 * i + 1] = (int32_t)compact3(k >> 1);
  xyz[3 * i + 2] = (int32_t)compact3(k);
}

hipError_t launch_keys_to_xyz(const uint64_t* keys, int64_t n, int D, int32_t* xyz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys_to_xyz, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, D, xyz);
  return hipGetLastError();
}

}  // namespace lpcc
