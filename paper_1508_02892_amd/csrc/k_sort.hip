// Compaction and stable counting sort of the particle slots by cell, run every
// sort_every steps so that deposits of a workgroup fall on few nodes.
//
// Tiles of kSortTile consecutive slots are owned by one wave each.  A tile's
// per-cell counts go to a bin-major matrix hist[c * nt + t]; an exclusive scan
// of that matrix in its flat order gives, for every (cell, tile), the first
// destination slot, so holes are dropped and equal cells keep their order.
// Within a tile, the rank of an item among earlier items of the same cell
// comes from wave ballots over the key bits plus a per-cell running count in
// LDS; rounds of 64 items are processed in order.
#include "hd_device.h"

namespace hd {

namespace {

constexpr int kScanItems = 16;                         // per thread
constexpr int kScanBlock = kThreads * kScanItems;      // elements per scan block
constexpr int kWavesPerBlock = kThreads / 64;

template <class P>
__device__ __forceinline__ uint32_t n_tiles(const Disch<P>& d) {
  return (d.st->n_main + (uint32_t)kSortTile - 1u) / (uint32_t)kSortTile;
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_sort_clear(const Disch<P>* __restrict__ ds, int D) {
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    if (!d.st->sort_due) continue;
    const uint64_t n = (uint64_t)d.nc * n_tiles(d);
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kThreads)
      d.hist[i] = 0u;
  }
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_sort_count(const Disch<P>* __restrict__ ds, int D) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * kWavesPerBlock + wv, nw = gridDim.x * kWavesPerBlock;
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    const State* st = d.st;
    if (!st->sort_due) continue;
    const uint32_t n = st->n_main, nt = n_tiles(d);
    const int nc = d.nc;
    uint32_t* h = reinterpret_cast<uint32_t*>(smem) + (size_t)wv * (size_t)(nc + 1);
    const int32_t* cell = d.cell[st->buf];
    for (uint32_t t = gw; t < nt; t += nw) {
      for (int c = lane; c < nc; c += 64) h[c] = 0u;
      int lo = nc, hi = -1;
      const uint32_t b = t * (uint32_t)kSortTile;
      const uint32_t e = min(n, b + (uint32_t)kSortTile);
      for (uint32_t i = b + (uint32_t)lane; i < e; i += 64) {
        const int c = cell[i];
        if (c >= 0) {
          atomicAdd(&h[c], 1u);
          lo = min(lo, c);
          hi = max(hi, c);
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
      }
      for (int c = lo + lane; c <= hi; c += 64) {
        const uint32_t v = h[c];
        if (v) d.hist[(size_t)c * nt + t] = v;
      }
      if (lane == 0) {
        d.tile_rng[2 * t] = lo;
        d.tile_rng[2 * t + 1] = hi;
      }
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

template <class P>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const Disch<P>* __restrict__ ds, int D) {
  __shared__ uint32_t sh[kWavesPerBlock];
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    if (!d.st->sort_due) continue;
    const uint64_t n = (uint64_t)d.nc * n_tiles(d);
    const uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    for (uint32_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
      uint32_t v[kScanItems];
      const uint64_t base = (uint64_t)blk * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
#pragma unroll
      for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? d.hist[base + k] : 0u;
      const uint32_t tot = block_excl_scan(v, sh);
      if (threadIdx.x == 0) d.bin_start[blk] = tot;
    }
  }
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_scan_top(const Disch<P>* __restrict__ ds) {
  __shared__ uint32_t sh[kWavesPerBlock];
  const Disch<P>& d = ds[blockIdx.x];
  State* st = d.st;
  if (!st->sort_due) return;
  const uint64_t n = (uint64_t)d.nc * n_tiles(d);
  const uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
  uint32_t run = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += (uint32_t)kScanBlock) {
    uint32_t v[kScanItems];
    const uint32_t base = b0 + threadIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < nb) ? d.bin_start[base + k] : 0u;
    const uint32_t tot = block_excl_scan(v, sh);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < nb) d.bin_start[base + k] = v[k] + run;
    run += tot;
  }
  if (threadIdx.x == 0) st->n_live_sorted = run;
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_scan_down(const Disch<P>* __restrict__ ds, int D) {
  __shared__ uint32_t sh[kWavesPerBlock];
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    if (!d.st->sort_due) continue;
    const uint64_t n = (uint64_t)d.nc * n_tiles(d);
    const uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    for (uint32_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
      uint32_t v[kScanItems];
      const uint64_t base = (uint64_t)blk * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
#pragma unroll
      for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? d.hist[base + k] : 0u;
      (void)block_excl_scan(v, sh);
      const uint32_t off = d.bin_start[blk];
#pragma unroll
      for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) d.hist[base + k] = v[k] + off;
    }
  }
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_sort_scatter(const Disch<P>* __restrict__ ds, int D) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * kWavesPerBlock + wv, nw = gridDim.x * kWavesPerBlock;
  const uint64_t lt = lanemask_lt();
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    const State* st = d.st;
    if (!st->sort_due) continue;
    const uint32_t n = st->n_main, nt = n_tiles(d);
    const int nc = d.nc;
    const int nbits = 32 - __clz((uint32_t)nc);  // keys 0 .. nc (nc marks a hole)
    uint32_t* run = reinterpret_cast<uint32_t*>(smem) + (size_t)wv * (size_t)(nc + 1);
    const int src = st->buf, dst = src ^ 1;
    const int32_t* cell = d.cell[src];
    for (uint32_t t = gw; t < nt; t += nw) {
      // per-cell cursor = first destination of this tile's items of that cell
      const int lo = d.tile_rng[2 * t], hi = d.tile_rng[2 * t + 1];
      for (int c = lo + lane; c <= hi; c += 64) run[c] = d.hist[(size_t)c * nt + t];
      const uint32_t b = t * (uint32_t)kSortTile;
      const uint32_t e = min(n, b + (uint32_t)kSortTile);
      constexpr int R = 4;  // rounds of 64 items whose loads are issued together
      for (uint32_t r = b; r < e; r += 64u * R) {
        int key[R];
        P o_[R], x_[R], y_[R], z_[R];
        uint32_t id_[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const uint32_t i = r + 64u * q + (uint32_t)lane;
          key[q] = nc;
          if (i < e) {
            const int c = cell[i];
            key[q] = c >= 0 ? c : nc;
            o_[q] = d.off[src][i];
            x_[q] = d.vx[src][i];
            y_[q] = d.vy[src][i];
            z_[q] = d.vz[src][i];
            id_[q] = d.id[src][i];
          }
        }
        uint32_t dest[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int k = key[q];
          const int k0 = __shfl(k, 0, 64);
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
          if (k < nc) {
            const uint32_t base = run[k];
            if (rank == 0) run[k] = base + cntk;
            dest[q] = base + rank;
          }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (key[q] < nc) {
            const uint32_t o = dest[q];
            d.cell[dst][o] = key[q];
            d.off[dst][o] = o_[q];
            d.vx[dst][o] = x_[q];
            d.vy[dst][o] = y_[q];
            d.vz[dst][o] = z_[q];
            d.id[dst][o] = id_[q];
          }
        }
      }
    }
  }
}

template <class P>
__global__ void k_sort_finish(const Disch<P>* __restrict__ ds, int D) {
  const int di = blockIdx.x * blockDim.x + threadIdx.x;
  if (di >= D) return;
  State* st = ds[di].st;
  if (!st->sort_due) return;
  st->buf ^= 1;
  st->n_main = st->n_live_sorted;
  st->sort_due = 0;
}

}  // namespace

template <class P>
hipError_t launch_sort_impl(const Disch<P>* d_dev, int D, int grid, int nc_max, hipStream_t s) {
  const size_t lds = (size_t)kWavesPerBlock * (size_t)(nc_max + 1) * 4u;
  hipLaunchKernelGGL(k_sort_clear<P>, dim3(grid), dim3(kThreads), 0, s, d_dev, D);
  hipLaunchKernelGGL(k_sort_count<P>, dim3(grid), dim3(kThreads), lds, s, d_dev, D);
  hipLaunchKernelGGL(k_scan_reduce<P>, dim3(grid), dim3(kThreads), 0, s, d_dev, D);
  hipLaunchKernelGGL(k_scan_top<P>, dim3(D), dim3(kThreads), 0, s, d_dev);
  hipLaunchKernelGGL(k_scan_down<P>, dim3(grid), dim3(kThreads), 0, s, d_dev, D);
  hipLaunchKernelGGL(k_sort_scatter<P>, dim3(grid), dim3(kThreads), lds, s, d_dev, D);
  hipLaunchKernelGGL(k_sort_finish<P>, dim3((D + 63) / 64), dim3(64), 0, s, d_dev, D);
  return hipGetLastError();
}

template <class P>
hipError_t sort_set_lds(int nc_max) {
  const int lds = kWavesPerBlock * (nc_max + 1) * 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_sort_count<P>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_sort_scatter<P>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// Scan-partials entries needed per discharge.
size_t sort_parts(size_t nc, size_t tiles) { return (nc * tiles + kScanBlock - 1) / kScanBlock + 1; }

template hipError_t launch_sort_impl<float>(const Disch<float>*, int, int, int, hipStream_t);
template hipError_t launch_sort_impl<double>(const Disch<double>*, int, int, int, hipStream_t);
template hipError_t sort_set_lds<float>(int);
template hipError_t sort_set_lds<double>(int);

}  // namespace hd
