// Compaction and stable counting sort of the particle slots by cell, run every
// sort_every steps so that deposits of a workgroup fall on few nodes.
//
// Tiles of T consecutive slots (T = 4,096 or 8,192).  A tile's per-cell counts go to a
// bin-major matrix hist[c * nt + t]; an exclusive scan of that matrix in its
// flat order gives, for every (cell, tile), the first destination slot, so
// holes are dropped and equal cells keep their order.  The matrix and the
// totals of its scan blocks are zero between sorts (zeroed with the
// discharge's buffer; the scan leaves 0 in empty entries and the scatter
// zeroes each entry it reads and the block totals), so the counts write
// only their nonzero entries and add them to their block's total, and no
// clearing or reduction pass is needed.  The scatter gives a
// tile to a workgroup: each wave counts its quarter of the tile, a per-cell
// prefix over the waves gives each wave its own cursors, and the rank of an
// item among earlier items of the same cell comes from wave ballots over the
// key bits, in rounds of 64 items processed in order.
#include "hd_device.h"

namespace hd {

namespace {

constexpr int kScanItems = 16;                         // per thread
constexpr int kScanBlock = kThreads * kScanItems;      // elements per scan block
constexpr int kWavesPerBlock = kThreads / 64;
constexpr int kScatterWindow = 1024;  // cells per window of the scatter's cursor arrays
// Cursor words per wave of the scatter.
inline int scatter_stride(int nc_max) { return nc_max + 1 < kScatterWindow ? nc_max + 1 : kScatterWindow; }

// Sort tiles of T items (at least kSortTile, the tile the count matrix and
// the tile ranges are allocated for): larger tiles mean fewer (cell, tile)
// entries, smaller ones more tiles to spread over the workgroups.  The
// sort's result does not depend on T.
template <int T, class P>
__device__ __forceinline__ uint32_t n_tiles(const Disch<P>& d) {
  return (d.st->n_main + (uint32_t)T - 1u) / (uint32_t)T;
}

// kScanItems consecutive matrix entries from base (a multiple of 16), as
// 16-byte vectors where the whole vector lies below n.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void load_items(const Gp<uint32_t>* h, uint64_t base, uint64_t n,
                                           uint32_t (&v)[kScanItems]) {
#pragma unroll
  for (int q = 0; q < kScanItems / 4; ++q) {
    const uint64_t i = base + 4u * (uint64_t)q;
    if (i + 4 <= n) {
      const u32x4 x = *reinterpret_cast<const Gp<u32x4>*>(h + i);
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) v[4 * q + k] = (i + k < n) ? h[i + k] : 0u;
    }
  }
}
// Stores back the scanned entries of load_items, skipping every 16-byte
// vector whose counts are all zero: those entries are zero and stay zero
// (an empty (cell, tile) keeps 0), so only the few vectors that hold a
// count are written.
__device__ __forceinline__ void store_items(Gp<uint32_t>* h, uint64_t base, uint64_t n,
                                            const uint32_t (&v)[kScanItems],
                                            const uint32_t (&cnt)[kScanItems]) {
#pragma unroll
  for (int q = 0; q < kScanItems / 4; ++q) {
    const uint64_t i = base + 4u * (uint64_t)q;
    if (i + 4 <= n) {
      if (cnt[4 * q] | cnt[4 * q + 1] | cnt[4 * q + 2] | cnt[4 * q + 3])
        *reinterpret_cast<Gp<u32x4>*>(h + i) = u32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i + k < n && cnt[4 * q + k]) h[i + k] = v[4 * q + k];
    }
  }
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of a block of kScanBlock elements (kScanItems consecutive per
// thread); returns the block total.  sh holds kWavesPerBlock words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t (&v)[kScanItems], uint32_t* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t x = v[k];
    v[k] = s;
    s += x;
  }
  const uint32_t inc = wave_incl_scan(s);
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    const uint32_t x = sh[w];
    if (w < wv) base += x;
    tot += x;
  }
  __syncthreads();
  const uint32_t ex = base + inc - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) v[k] += ex;
  return tot;
}

// Work units (sort tiles, scan blocks) of all discharges due for a sort are
// numbered one after another, so that the workgroups of a launch share the
// whole batch's work whatever the sizes of its discharges (taking the
// discharges in turn left most workgroups idle on the small ones): the
// first unit of discharge i is pre[i] and the total pre[D], in LDS
// (D + 1 words), computed by every workgroup from the discharges' states.
template <int T, class P>
__device__ __forceinline__ uint32_t tiles_due(const Disch<P>& d) {
  return d.st->sort_due ? n_tiles<T>(d) : 0u;
}
template <int T, class P>
__device__ __forceinline__ uint32_t scan_blocks(const Disch<P>& d) {
  const uint64_t n = (uint64_t)d.nc * n_tiles<T>(d);
  return (uint32_t)((n + kScanBlock - 1) / kScanBlock);
}
template <int T, class P>
__device__ __forceinline__ uint32_t scan_blocks_due(const Disch<P>& d) {
  return d.st->sort_due ? scan_blocks<T>(d) : 0u;
}
template <class P, class U>
__device__ void unit_prefix(const Disch<P>* __restrict__ ds, int D, uint32_t* pre, U units) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t carry = 0;
    for (int b = 0; b < D; b += 64) {
      const int i = b + lane;
      const uint32_t v = i < D ? units(ds[i]) : 0u;
      const uint32_t inc = wave_incl_scan(v);
      if (i < D) pre[i + 1] = carry + inc;
      carry += __shfl(inc, 63, 64);
    }
    if (lane == 0) pre[0] = 0u;
  }
  __syncthreads();
}

template <class P, int T>
__global__ __launch_bounds__(kThreads) void k_sort_count(const Disch<P>* __restrict__ ds, int D,
                                                         int stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_lo[kWavesPerBlock], sh_hi[kWavesPerBlock];
  constexpr uint32_t kQuarter = (uint32_t)T / kWavesPerBlock;  // slots per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // one histogram of stride (>= the largest nc + 1) words for the whole
  // launch, shared by the four waves (LDS atomics) and zero between tiles,
  // so that the LDS of a large grid still lets several workgroups share a
  // CU; the unit prefix follows it
  uint32_t* h = reinterpret_cast<uint32_t*>(smem);
  uint32_t* pre = h + (size_t)stride;
  for (int c = (int)threadIdx.x; c < stride; c += kThreads) h[c] = 0u;
  unit_prefix(ds, D, pre, [](const Disch<P>& d) { return tiles_due<T>(d); });
  const uint32_t total = pre[D];
  int di = 0;
  // The four waves of a workgroup share a tile, a quarter each, so that a
  // tile's loads and counts are spread over four waves rather than
  // serialised in one.
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    while (pre[di + 1] <= g) ++di;
    const Disch<P>& d = ds[di];
    const State* st = d.st;
    const uint32_t t = g - pre[di];
    const uint32_t n = st->n_main, nt = n_tiles<T>(d);
    const int nc = d.nc;
    const Gp<int32_t>* cell = gptr(d.cell[st->buf]);
    Gp<uint32_t>* hist = gptr(d.hist);
    const uint32_t b = t * (uint32_t)T + (uint32_t)wv * kQuarter;
    const uint32_t e = min(n, b + kQuarter);
    // 4 consecutive slots per lane per 256-slot round, all rounds loaded
    // before they are counted (the capacity is a multiple of the tile, so
    // every vector load stays inside the array)
    constexpr int kRounds = (int)(kQuarter / 256u);
    int32_t c4[kRounds][4];
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const uint32_t i = b + 256u * (uint32_t)q + 4u * (uint32_t)lane;
      if (i < e) gld4(cell + i, c4[q]);
    }
    // the tile's cell range first
    int lo = nc, hi = -1;
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const uint32_t i = b + 256u * (uint32_t)q + 4u * (uint32_t)lane;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = c4[q][k];
        if (i + (uint32_t)k < e && c >= 0) {
          lo = min(lo, c);
          hi = max(hi, c);
        }
      }
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    if (lane == 0) {
      sh_lo[wv] = lo;
      sh_hi[wv] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
      lo = min(lo, sh_lo[w]);
      hi = max(hi, sh_hi[w]);
    }
    // Cells lo .. lo + 7 are counted in 8-bit fields of one register per
    // lane (at most 16 items per lane), then in 16-bit fields summed over
    // the wave (at most kQuarter per cell); other cells go straight to the
    // histogram.  With nearly sorted cells an atomic per item would have
    // all 64 lanes on one address.
    uint64_t a8 = 0;
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const uint32_t i = b + 256u * (uint32_t)q + 4u * (uint32_t)lane;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = c4[q][k];
        if (i + (uint32_t)k < e && c >= 0) {
          const uint32_t o = (uint32_t)(c - lo);
          if (o < 8u)
            a8 += 1ull << (8u * o);
          else
            atomicAdd(&h[c], 1u);
        }
      }
    }
    const uint32_t w0 = (uint32_t)a8, w1 = (uint32_t)(a8 >> 32);
    const uint64_t s0 = wave_sum_u64((uint64_t)(w0 & 0xffu) | ((uint64_t)((w0 >> 8) & 0xffu) << 16) |
                                     ((uint64_t)((w0 >> 16) & 0xffu) << 32) | ((uint64_t)(w0 >> 24) << 48));
    const uint64_t s1 = wave_sum_u64((uint64_t)(w1 & 0xffu) | ((uint64_t)((w1 >> 8) & 0xffu) << 16) |
                                     ((uint64_t)((w1 >> 16) & 0xffu) << 32) | ((uint64_t)(w1 >> 24) << 48));
    if (lane < 8 && lo + lane < nc) {
      const uint32_t v = (uint32_t)(((lane < 4) ? s0 : s1) >> (16 * (lane & 3))) & 0xffffu;
      if (v) atomicAdd(&h[lo + lane], v);
    }
    __syncthreads();
    // the tile's count of each cell
    for (int c = lo + (int)threadIdx.x; c <= hi; c += kThreads) {
      const uint32_t v = h[c];
      h[c] = 0u;
      if (v) {
        hist[(size_t)c * nt + t] = v;
        // the total of the scan block holding this entry
        atomicAdd(&d.bin_start[((size_t)c * nt + t) / (size_t)kScanBlock], v);
      }
    }
    if (threadIdx.x == 0) {
      gptr(d.tile_rng)[2 * t] = lo;
      gptr(d.tile_rng)[2 * t + 1] = hi;
    }
    __syncthreads();  // histograms and ranges are reused by the next tile
  }
}

template <class P, int T>
__global__ __launch_bounds__(kThreads) void k_scan_down(const Disch<P>* __restrict__ ds, int D) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t sh[kWavesPerBlock];
  __shared__ uint32_t sh_off[kWavesPerBlock];
  uint32_t* pre = reinterpret_cast<uint32_t*>(smem);
  // a discharge due for a sort with no slots in use sorts to nothing
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < D; i += kThreads) {
      State* st = ds[i].st;
      if (st->sort_due && scan_blocks<T>(ds[i]) == 0) st->n_live_sorted = 0;
    }
  unit_prefix(ds, D, pre, [](const Disch<P>& d) { return scan_blocks_due<T>(d); });
  const uint32_t total = pre[D];
  int di = 0;
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    while (pre[di + 1] <= g) ++di;
    const Disch<P>& d = ds[di];
    State* st = d.st;
    const uint64_t n = (uint64_t)d.nc * n_tiles<T>(d);
    const uint32_t nb = pre[di + 1] - pre[di], blk = g - pre[di];
    uint32_t v[kScanItems];
    const uint64_t base = (uint64_t)blk * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
    load_items(gptr(d.hist), base, n, v);
    // the block's offset: the totals of the blocks before it (each block
    // sums them itself instead of a separate pass scanning the totals)
    uint32_t part = 0;
    for (uint32_t b2 = threadIdx.x; b2 < blk; b2 += (uint32_t)kThreads) part += d.bin_start[b2];
    part = wave_sum_u32(part);
    if ((threadIdx.x & 63) == 0) sh_off[threadIdx.x >> 6] = part;
    uint32_t cnt[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) cnt[k] = v[k];
    const uint32_t tot = block_excl_scan(v, sh);  // its barriers also publish sh_off
    uint32_t off = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) off += sh_off[w];
    if (blk == nb - 1 && threadIdx.x == 0) st->n_live_sorted = off + tot;
    // an empty (cell, tile) keeps 0: no item reads its start, and the
    // matrix is then zero again once the scatter has read the others
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = cnt[k] ? v[k] + off : 0u;
    store_items(gptr(d.hist), base, n, v, cnt);
    __syncthreads();  // sh_off is rewritten for the next block
  }
}

template <class P, int T>
__global__ __launch_bounds__(kThreads) void k_sort_scatter(const Disch<P>* __restrict__ ds, int D,
                                                           int stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr uint32_t kQuarter = (uint32_t)T / kWavesPerBlock;  // slots per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t lt = lanemask_lt();
  // run[w][c - lo]: cursor of wave w for cell c; the unit prefix follows
  uint32_t* run = reinterpret_cast<uint32_t*>(smem);
  uint32_t* pre = run + (size_t)kWavesPerBlock * (size_t)stride;
  // the scan blocks' totals are zero again for the next sort's counts: one
  // flat index over the due discharges' blocks (their counts read in
  // parallel, not one discharge's state after another)
  unit_prefix(ds, D, pre, [](const Disch<P>& d) { return scan_blocks_due<T>(d); });
  {
    const uint32_t nz = pre[D];
    int dz = 0;
    for (uint32_t u = blockIdx.x * kThreads + threadIdx.x; u < nz; u += gridDim.x * kThreads) {
      while (pre[dz + 1] <= u) ++dz;
      ds[dz].bin_start[u - pre[dz]] = 0u;
    }
  }
  __syncthreads();  // pre[] is reused for the tiles
  unit_prefix(ds, D, pre, [](const Disch<P>& d) { return tiles_due<T>(d); });
  const uint32_t total = pre[D];
  int di = 0;
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    while (pre[di + 1] <= g) ++di;
    const Disch<P>& d = ds[di];
    const State* st = d.st;
    const uint32_t t = g - pre[di];
    const uint32_t n = st->n_main, nt = n_tiles<T>(d);
    const int nc = d.nc;
    const int nbits = 32 - __clz((uint32_t)nc);  // keys 0 .. nc (nc marks a hole)
    const int src = st->buf, dst = src ^ 1;
    const Gp<int32_t>* cell = gptr(d.cell[src]);
    const Gp<P>* s_off = gptr(d.off[src]);
    const Gp<P>* s_vx = gptr(d.vx[src]);
    const Gp<P>* s_vy = gptr(d.vy[src]);
    const Gp<P>* s_vz = gptr(d.vz[src]);
    const Gp<uint32_t>* s_id = gptr(d.id[src]);
    Gp<int32_t>* d_cell = gptr(d.cell[dst]);
    Gp<P>* d_off = gptr(d.off[dst]);
    Gp<P>* d_vx = gptr(d.vx[dst]);
    Gp<P>* d_vy = gptr(d.vy[dst]);
    Gp<P>* d_vz = gptr(d.vz[dst]);
    Gp<uint32_t>* d_id = gptr(d.id[dst]);
    const int lo = gptr(d.tile_rng)[2 * t], hi = gptr(d.tile_rng)[2 * t + 1];
    const uint32_t b = t * (uint32_t)T + (uint32_t)wv * kQuarter;
    const uint32_t e = min(n, b + kQuarter);
    uint32_t* myrun = run + wv * stride;
    // The tile's cells in windows of at most stride cells (one window for
    // all but the most spread-out tiles: the LDS then fits several
    // workgroups per CU at the largest grids); a tile of holes only has none.
    for (int wlo = lo; wlo <= hi; wlo += stride) {
      const int whi = min(hi, wlo + stride - 1);
      const int span = whi - wlo + 1;
      // counts of this wave's quarter in the window
      for (int c = lane; c < span; c += 64) myrun[c] = 0u;
      __builtin_amdgcn_wave_barrier();
      {
        constexpr int kRounds = (int)(kQuarter / 256u);
        int32_t c4[kRounds][4];
#pragma unroll
        for (int q = 0; q < kRounds; ++q) {
          const uint32_t i = b + 256u * (uint32_t)q + 4u * (uint32_t)lane;
          if (i < e) gld4(cell + i, c4[q]);
        }
        // cells wlo .. wlo + 7 in packed fields as in the count (at most 16
        // items per lane, kQuarter per cell), the others by atomics
        uint64_t a8 = 0;
#pragma unroll
        for (int q = 0; q < kRounds; ++q) {
          const uint32_t i = b + 256u * (uint32_t)q + 4u * (uint32_t)lane;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (i + (uint32_t)k < e && c4[q][k] >= 0) {
              const uint32_t o = (uint32_t)(c4[q][k] - wlo);
              if (o < (uint32_t)span) {
                if (o < 8u)
                  a8 += 1ull << (8u * o);
                else
                  atomicAdd(&myrun[o], 1u);
              }
            }
        }
        const uint32_t w0 = (uint32_t)a8, w1 = (uint32_t)(a8 >> 32);
        const uint64_t s0 = wave_sum_u64((uint64_t)(w0 & 0xffu) | ((uint64_t)((w0 >> 8) & 0xffu) << 16) |
                                         ((uint64_t)((w0 >> 16) & 0xffu) << 32) | ((uint64_t)(w0 >> 24) << 48));
        const uint64_t s1 = wave_sum_u64((uint64_t)(w1 & 0xffu) | ((uint64_t)((w1 >> 8) & 0xffu) << 16) |
                                         ((uint64_t)((w1 >> 16) & 0xffu) << 32) | ((uint64_t)(w1 >> 24) << 48));
        if (lane < 8) {
          const uint32_t v = (uint32_t)(((lane < 4) ? s0 : s1) >> (16 * (lane & 3))) & 0xffffu;
          if (v) myrun[lane] += v;
        }
      }
      __syncthreads();
      // cursors: the tile's first slot for the cell, then the earlier waves
      // (only cells present in the tile: the range can be wide and sparse)
      for (int c = threadIdx.x; c < span; c += kThreads) {
        uint32_t k[kWavesPerBlock], tot = 0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) {
          k[w] = run[w * stride + c];
          tot += k[w];
        }
        if (tot == 0) continue;
        uint32_t r = gptr(d.hist)[(size_t)(wlo + c) * nt + t];
        gptr(d.hist)[(size_t)(wlo + c) * nt + t] = 0u;  // zero for the next sort's counts
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) {
          run[w * stride + c] = r;
          r += k[w];
        }
      }
      __syncthreads();
      // rounds of 64 items whose loads are issued together; the source
      // arrays are read once per window, with the nontemporal hint, so that
      // they do not displace the destination's partly written lines from
      // the caches; items of other windows wait for theirs
      constexpr int R = 8;
      for (uint32_t r = b; r < e; r += 64u * R) {
        int key[R];
        P o_[R], x_[R], y_[R], z_[R];
        uint32_t id_[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const uint32_t i = r + 64u * q + (uint32_t)lane;
          key[q] = nc;
          if (i < e) {
            const int c = __builtin_nontemporal_load(cell + i);
            key[q] = c >= 0 ? c : nc;
            o_[q] = __builtin_nontemporal_load(s_off + i);
            x_[q] = __builtin_nontemporal_load(s_vx + i);
            y_[q] = __builtin_nontemporal_load(s_vy + i);
            z_[q] = __builtin_nontemporal_load(s_vz + i);
            id_[q] = __builtin_nontemporal_load(s_id + i);
          }
        }
        uint32_t dest[R];
        bool here[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int k = key[q];
          const int k0 = __builtin_amdgcn_readfirstlane(k);
          uint64_t peers = ~0ull;
          if (__ballot(k == k0) != ~0ull) {
            for (int bit = 0; bit < nbits; ++bit) {
              const bool on = (k >> bit) & 1;
              const uint64_t m = __ballot(on);
              peers &= on ? m : ~m;
            }
          }
          const uint32_t rank = (uint32_t)__popcll(peers & lt);
          const uint32_t cntk = (uint32_t)__popcll(peers);
          dest[q] = 0;
          here[q] = k >= wlo && k <= whi;  // holes (nc) are never in a window
          if (here[q]) {
            const uint32_t base = myrun[k - wlo];
            if (rank == 0) myrun[k - wlo] = base + cntk;
            dest[q] = base + rank;
          }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (here[q]) {
            const uint32_t o = dest[q];
            d_cell[o] = key[q];
            d_off[o] = o_[q];
            d_vx[o] = x_[q];
            d_vy[o] = y_[q];
            d_vz[o] = z_[q];
            d_id[o] = id_[q];
          }
        }
      }
      __syncthreads();  // the window's cursors are rewritten by the next one
    }
    __syncthreads();  // cursors are rewritten for the next tile
  }
}

template <class P>
__global__ void k_sort_finish(const Disch<P>* __restrict__ ds, int D) {
  const int di = blockIdx.x * blockDim.x + threadIdx.x;
  if (di >= D) return;
  State* st = ds[di].st;
  if (!st->sort_due) return;
  st->buf ^= 1;
  const uint32_t n = st->n_live_sorted;
  st->n_main = n;
  st->sort_due = 0;
  // Checkpoint the coming interval's start when it is close to capacity:
  // fewer free slots than twice the last interval's growth plus the most
  // secondaries an interval can bring (both walls, every step).
  const Disch<P>& d = ds[di];
  const uint32_t grow = n > st->prev_n_main ? n - st->prev_n_main : 0u;
  const uint64_t need = 2ull * grow + 2ull * (uint64_t)kSeeMax * (uint64_t)d.sort_every;
  st->ckpt_due = (uint64_t)n + need > (uint64_t)d.capacity ? 1 : 0;
  st->prev_n_main = n;
}

// Checkpoint of a sort interval's start, for rolling back an interval whose
// particles overflow the capacity.  restore = 0, at the interval's start:
// when the start was judged close to capacity (ckpt_due) the live slots
// [0, n_main) go to the other particle buffer (unused until the interval's
// sort, which an overflow suppresses) and the grid region and the State to
// the checkpoint area; otherwise the checkpoint is marked invalid.
// restore = 1: everything is copied back (the State last, by one thread;
// the copies read only the checkpoint).
template <class P>
__global__ __launch_bounds__(kThreads) void k_checkpoint(const Disch<P>* __restrict__ ds, int D,
                                                         int restore) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t gsz = (size_t)gridDim.x * blockDim.x;
  // restore = 0: the decisions of kThreads discharges at a time are read in
  // parallel (1: take a checkpoint, 2: mark it invalid, 0: keep it), so that
  // a batch does not wait for one state's round trip per discharge
  __shared__ uint8_t take[kThreads];
  for (int g0 = 0; g0 < D; g0 += kThreads) {
    const int ng = min(kThreads, D - g0);
    if (!restore) {
      uint8_t f = 0;
      if ((int)threadIdx.x < ng) {
        State* st = ds[g0 + (int)threadIdx.x].st;
        const int err = st->error;
        const int due = st->ckpt_due;
        const int64_t left = st->steps_left;
        // an interval stopped by an error keeps its checkpoint
        f = err ? 0 : ((due && left > 0) ? 1 : 2);
        if (f == 2 && blockIdx.x == 0) st->ckpt_valid = 0;
      }
      take[threadIdx.x] = f;
      __syncthreads();
    }
    for (int di = g0; di < g0 + ng; ++di) {
      const Disch<P>& d = ds[di];
      State* st = d.st;
      State* sv = reinterpret_cast<State*>(d.ckpt + d.grid_bytes);
      if (!restore) {
        if (take[di - g0] != 1) continue;
      } else if (!st->ckpt_valid) {
        continue;
      }
      const int cur = restore ? sv->buf : st->buf;
      const size_t n = restore ? sv->n_main : st->n_main;
      const int src = restore ? cur ^ 1 : cur, dst = src ^ 1;
      for (size_t i = gid; i < n; i += gsz) {
        d.cell[dst][i] = d.cell[src][i];
        d.off[dst][i] = d.off[src][i];
        d.vx[dst][i] = d.vx[src][i];
        d.vy[dst][i] = d.vy[src][i];
        d.vz[dst][i] = d.vz[src][i];
        d.id[dst][i] = d.id[src][i];
      }
      uint4* grid = reinterpret_cast<uint4*>(d.cnt[0]);
      uint4* keep = reinterpret_cast<uint4*>(d.ckpt);
      const size_t words = d.grid_bytes / 16;
      for (size_t w = gid; w < words; w += gsz) {
        if (restore)
          grid[w] = keep[w];
        else
          keep[w] = grid[w];
      }
      if (gid == 0) {
        if (!restore) {
          *sv = *st;
          st->ckpt_valid = 1;
          st->ckpt_step = st->step;
        } else {
          State x = *sv;
          x.ckpt_valid = 1;  // the checkpoint still holds this state
          x.ckpt_step = x.step;
          *st = x;
        }
      }
    }
    if (!restore) __syncthreads();  // take[] is refilled for the next discharges
  }
}

}  // namespace

template <class P, int T>
void launch_sort_tiles(const Disch<P>* d_dev, int D, int grid, int nc_max, hipStream_t s) {
  const size_t pre = (size_t)(D + 1) * 4u;
  const size_t lds_count = (size_t)(nc_max + 1) * 4u + pre;
  hipLaunchKernelGGL((k_sort_count<P, T>), dim3(grid), dim3(kThreads), lds_count, s, d_dev, D,
                     nc_max + 1);
  hipLaunchKernelGGL((k_scan_down<P, T>), dim3(grid), dim3(kThreads), pre, s, d_dev, D);
  const int sw = scatter_stride(nc_max);
  const size_t lds_scatter = (size_t)kWavesPerBlock * (size_t)sw * 4u + pre;
  hipLaunchKernelGGL((k_sort_scatter<P, T>), dim3(grid), dim3(kThreads), lds_scatter, s, d_dev, D,
                     sw);
}

// tile: items per sort tile, kSortTile or twice that (checked by the
// caller).
template <class P>
hipError_t launch_sort_impl(const Disch<P>* d_dev, int D, int grid, int tile, int nc_max,
                            hipStream_t s) {
  if (tile == 2 * kSortTile)
    launch_sort_tiles<P, 2 * kSortTile>(d_dev, D, grid, nc_max, s);
  else
    launch_sort_tiles<P, kSortTile>(d_dev, D, grid, nc_max, s);
  hipLaunchKernelGGL(k_sort_finish<P>, dim3((D + 63) / 64), dim3(64), 0, s, d_dev, D);
  return hipGetLastError();
}

template <class P>
hipError_t launch_checkpoint(const Disch<P>* d_dev, int D, int restore, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_checkpoint<P>, dim3(grid), dim3(kThreads), 0, s, d_dev, D, restore);
  return hipGetLastError();
}

template <class P, int T>
hipError_t sort_set_lds_tiles(int nc_max, int D) {
  const int pre = (D + 1) * 4;
  const int lds = kWavesPerBlock * scatter_stride(nc_max) * 4 + pre;
  hipError_t e = hipFuncSetAttribute((const void*)k_sort_count<P, T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (nc_max + 1) * 4 + pre);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_scan_down<P, T>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, pre);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_sort_scatter<P, T>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <class P>
hipError_t sort_set_lds(int nc_max, int D) {
  hipError_t e = sort_set_lds_tiles<P, kSortTile>(nc_max, D);
  if (e == hipSuccess) e = sort_set_lds_tiles<P, 2 * kSortTile>(nc_max, D);
  return e;
}

// LDS of the sort's count and scatter launches.
size_t sort_lds_bytes(int nc_max, int D) {
  const size_t pre = (size_t)(D + 1) * 4u;
  const size_t count = (size_t)(nc_max + 1) * 4u + pre;
  const size_t scatter = (size_t)kWavesPerBlock * (size_t)scatter_stride(nc_max) * 4u + pre;
  return count > scatter ? count : scatter;
}

// Scan-partials entries needed per discharge.
size_t sort_parts(size_t nc, size_t tiles) { return (nc * tiles + kScanBlock - 1) / kScanBlock + 1; }

template hipError_t launch_sort_impl<float>(const Disch<float>*, int, int, int, int, hipStream_t);
template hipError_t launch_checkpoint<float>(const Disch<float>*, int, int, int, hipStream_t);
template hipError_t launch_checkpoint<double>(const Disch<double>*, int, int, int, hipStream_t);
template hipError_t launch_sort_impl<double>(const Disch<double>*, int, int, int, int,
                                            hipStream_t);
template hipError_t sort_set_lds<float>(int, int);
template hipError_t sort_set_lds<double>(int, int);

}  // namespace hd
