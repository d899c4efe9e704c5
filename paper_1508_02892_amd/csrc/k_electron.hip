// Fused electron step (Sec. II.A): leapfrog push with linear gather, removal
// at the electrodes, null-collision Monte Carlo and cloud-in-cell deposit,
// plus the ion-fluid update of the same step (Secs. II.B-C) in dedicated
// workgroups that run concurrently with the particle workgroups.
//
// Particle workgroups are persistent: the chunks of all active discharges are
// laid end to end and split into contiguous ranges, one per workgroup.  For
// each discharge it touches, a workgroup keeps the collision table, a
// fixed-point deposit grid, the EEDF histogram and event counters in LDS and
// flushes them once.  Collisions are compacted into an LDS queue (in particle
// order, by a ballot prefix sum) so that the rare scattering work runs on
// fully occupied lanes; children of ionizations are staged per chunk in
// parent order.
#include "hd.h"
#include "hd_device.h"

namespace hd {

namespace {

constexpr double kECharge = 1.602176634e-19;
// Workgroups are kElecThreads (eight waves) or, in the wide variants,
// kElecThreadsWide (sixteen waves, one workgroup per CU where the LDS of a
// large grid leaves room for only one narrow one); a chunk is four particles
// per thread, so 2,048 or 4,096 slots.
constexpr int kElecThreadsWide = 2 * kElecThreads;
constexpr int kWQ = 128;                   // per-wave collision queue entries
constexpr int kTabLds = 1024;              // collision-table rows kept in LDS (0 .. 102.3 eV
                                           // at 10 points per eV); higher rows via the cache
constexpr uint32_t kKidsLds = 256;         // sub-chunk child counts of a segment kept in LDS
static_assert(kKidsLds <= (uint32_t)kElecThreads, "the LDS counts are scanned in one round");

// Workgroup barrier that orders LDS accesses only: the wave's global stores
// may still be in flight when it passes, where __syncthreads waits for them.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// A pointer that is the same in every lane, moved to scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

// A collision waiting to be scattered.  meta: bits 0-7 channel, bit 8 set if
// a child is created, bits 16-23 the child's index within the sub-chunk.
template <class P>
struct alignas(16) QEntry {
  P vx, vy, vz, off;
  uint32_t id;
  int32_t c;
  uint32_t slot;
  uint32_t meta;
};

struct ElecArgs {
  int D;
  int tab_max;    // max ne*K over the batch
  int nn_max;     // max nodes
  int nb1_max;    // max eedf bins + 1
  int fluid_nn;   // max nodes of a full-fluid discharge (its solver lives in LDS), 0 if none
  int K_max;      // max channels
  int tab_rows;   // collision-table rows held in LDS (tab_rows_lds)
  int waves;      // waves per workgroup (8, or 16 in the wide variants)
};

struct Lds {
  uint32_t tab, ep, bins, q, eedf, ctr, pre, kids, total;
  uint32_t rows;  // collision-table rows held in LDS
};

// LDS counters: [0, kMaxK) collisions per channel, then these.
enum { kCtrAbsL = kMaxK, kCtrAbsR, kCtrCreated, kCtrOverflow, kCtrPushed, kCtrN };

template <class P>
__host__ __device__ inline Lds lds_layout(const ElecArgs& a) {
  auto al = [](uint32_t x) { return (x + 15u) & ~15u; };
  const uint32_t rows = (uint32_t)a.tab_rows;
  // min(ne, rows) * K of any discharge is at most this
  const uint32_t tab_lds = (uint32_t)a.tab_max < rows * (uint32_t)a.K_max
                               ? (uint32_t)a.tab_max : rows * (uint32_t)a.K_max;
  Lds L;
  L.rows = rows;
  L.tab = 0;
  L.ep = al(L.tab + tab_lds * (uint32_t)sizeof(P));
  L.bins = al(L.ep + (uint32_t)a.nn_max * (uint32_t)sizeof(P));
  L.q = al(L.bins + (uint32_t)a.nn_max * 8u);
  L.eedf = al(L.q + (uint32_t)a.waves * (uint32_t)kWQ * (uint32_t)sizeof(QEntry<P>));
  L.ctr = al(L.eedf + (uint32_t)a.nb1_max * 4u);
  L.pre = al(L.ctr + (uint32_t)kCtrN * 4u);
  L.kids = al(L.pre + (uint32_t)(a.D + 1) * 4u);
  L.total = al(L.kids + kKidsLds * 4u);
  // a, b, c, r of Eq (2.3) and the reduced system of the partitioned solve
  const uint32_t fluid = a.fluid_nn ? (4u * (uint32_t)a.fluid_nn + 7u * (uint32_t)kTriRed) * 8u : 0u;
  if (fluid > L.total) L.total = al(fluid);
  return L;
}

// The collision table keeps its first kTabLds rows in LDS, fewer when that
// would leave room for only one narrow workgroup per CU (many channels, large
// grids) while fewer rows make room for two (one wide workgroup: the whole
// CU's LDS): rows above come through the cache, which only the rare fast
// electrons read.  Chosen on the host.
constexpr uint32_t kTwoPerCu = (80u << 10) - 1024u;   // LDS per workgroup for two per CU
constexpr uint32_t kOnePerCu = (160u << 10) - 1024u;  // LDS of a wide workgroup
constexpr uint32_t kTabMinLds = 128;

template <class P>
ElecArgs elec_args(int D, int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max,
                   int waves) {
  ElecArgs a{D, tab_max, nn_max, nb1_max, fluid_nn, K_max, kTabLds, waves};
  const Lds L = lds_layout<P>(a);
  const uint32_t budget = waves > kElecThreads / 64 ? kOnePerCu : kTwoPerCu;
  const uint32_t fluid = fluid_nn ? (4u * (uint32_t)fluid_nn + 7u * (uint32_t)kTriRed) * 8u : 0u;
  if (L.total > budget && fluid <= budget) {
    const uint32_t rest = L.total - L.ep;  // everything but the table
    const uint32_t row = (uint32_t)K_max * (uint32_t)sizeof(P);
    const uint32_t rows = rest < budget ? (budget - rest) / row : 0u;
    if (rows >= kTabMinLds && rows < (uint32_t)kTabLds) a.tab_rows = (int)rows;
  }
  return a;
}

__device__ __forceinline__ void lds_add_i64(int64_t* p, uint64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

// What a workgroup needs while working on one discharge, read once from the
// descriptor: LDS arrays, the particle arrays of the current buffer and the
// constants of the push, the null-collision test and the EEDF.
template <class P>
struct Seg {
  const P* tab;       // LDS rows [0, tab_rows) of the cumulative probabilities
  const P* ep;        // LDS copy of E' = (-e/m_e) dt E at the nodes
  int64_t* bins;      // LDS deposit grid
  uint32_t* eedf;     // LDS histogram
  uint32_t* ctr;      // LDS counters
  const Gp<P>* tab_g; // full table
  Gp<int32_t>* cell;
  Gp<P>* off;
  Gp<P>* vx;
  Gp<P>* vy;
  Gp<P>* vz;
  Gp<uint32_t>* id;
  P kdz, Pmax, KE, inv_dE, keedf;
  int tab_rows, nc, ne, K, nbins;
  uint32_t ion_mask;  // bit k: channel k is an ionization
  uint32_t att_mask;  // bit k: channel k is an attachment
  uint32_t seed_lo, seed_hi, step, n_main;
  uint32_t* kl;       // LDS copy of the segment's first kKidsLds sub-chunk child counts
  uint32_t kbase;     // index of the segment's first sub-chunk
  bool sample;
};

template <class P>
__device__ __forceinline__ int eedf_bin(P vx, P vy, P vz, const Seg<P>& g) {
  const P en = g.KE * ((vx * vx + vy * vy) + vz * vz);
  const P x = en * g.keedf;
  return (x < (P)g.nbins) ? (int)x : g.nbins;
}

// Scattering of one queued collision (elastic / excitation / ionization /
// attachment).  The particle's new velocity goes straight to its slot; an
// ionization's new electron goes to the staging area of its sub-chunk, with
// its deposit, ion source (of the channel's product species) and EEDF
// sample; an attached electron's slot becomes a hole and its charge joins
// the negative-ion source at its position (it was not deposited).
// With SW the new velocity goes back into the queue entry, for the slot's
// own lane to pick up, instead of to the particle arrays.
template <class P, bool ATT, bool SW>
__device__ void handle(const Disch<P>& d, const Seg<P>& g, QEntry<P>& e) {
  StreamT<true> s(d.seed, kTagElectron, e.id, g.step);
  for (int w = 0; w < Uni<P>::kWords; ++w) (void)s.word();  // R used by the null test
  const int ch = (int)(e.meta & 0xFFu);
  const P vx = e.vx, vy = e.vy, vz = e.vz;
  const P v2 = (vx * vx + vy * vy) + vz * vz;
  const P en = d.KE * v2;
  const int kind = d.kind[ch];
  P nx, ny, nz, ox, oy, oz;
  if (ATT && kind == 3) {
    const int64_t W1 = cic_w1<P>(e.off);
    const int64_t W0 = ((int64_t)1 << 32) - W1;
    int64_t* src = d.ion_src + (size_t)d.product[ch] * (size_t)d.nn;
    atomic_add_i64(&src[e.c], W0);
    atomic_add_i64(&src[e.c + 1], W1);
    g.cell[e.slot] = -1;
    atomicAdd(&g.ctr[ch], 1u);
    return;
  }
  if (kind == 0) {
    sphere<P>(s, nx, ny, nz);
    const P vm = sqrt(v2);
    const P cosx = ((vx * nx + vy * ny) + vz * nz) / vm;
    const P fac = (P)1 - d.delta_k[ch] * ((P)1 - cosx);
    const P vn = sqrt(v2 * fac);
    ox = vn * nx;
    oy = vn * ny;
    oz = vn * nz;
  } else if (kind == 1) {
    sphere<P>(s, nx, ny, nz);
    P er = en - d.thr[ch];
    if (er < (P)0) er = (P)0;
    const P vn = sqrt(er * d.invKE);
    ox = vn * nx;
    oy = vn * ny;
    oz = vn * nz;
  } else {
    sphere<P>(s, nx, ny, nz);
    const P us = Uni<P>::get(s);
    P er = en - d.thr[ch];
    if (er < (P)0) er = (P)0;
    const P es = us * er;
    const P ep = er - es;
    const P vn = sqrt(ep * d.invKE);
    ox = vn * nx;
    oy = vn * ny;
    oz = vn * nz;
    P mx, my, mz;
    sphere<P>(s, mx, my, mz);
    const P vc = sqrt(es * d.invKE);
    const P cvx = vc * mx, cvy = vc * my, cvz = vc * mz;
    const uint32_t kslot = e.slot / (uint32_t)kSub * (uint32_t)kSub + (e.meta >> 16);
    gptr(d.kc)[kslot] = e.c;
    gptr(d.koff)[kslot] = e.off;
    gptr(d.kvx)[kslot] = cvx;
    gptr(d.kvy)[kslot] = cvy;
    gptr(d.kvz)[kslot] = cvz;
    const int64_t W1 = cic_w1<P>(e.off);
    const int64_t W0 = ((int64_t)1 << 32) - W1;
    lds_add_i64(&g.bins[e.c], (uint64_t)W0);
    lds_add_i64(&g.bins[e.c + 1], (uint64_t)W1);
    int64_t* src = d.ion_src + (size_t)d.product[ch] * (size_t)d.nn;
    atomic_add_i64(&src[e.c], W0);
    atomic_add_i64(&src[e.c + 1], W1);
    if (g.sample) atomicAdd(&g.eedf[eedf_bin<P>(cvx, cvy, cvz, g)], 1u);
    atomicAdd(&g.ctr[kCtrCreated], 1u);
  }
  if constexpr (SW) {
    e.vx = ox;
    e.vy = oy;
    e.vz = oz;
  } else {
    g.vx[e.slot] = ox;
    g.vy[e.slot] = oy;
    g.vz[e.slot] = oz;
  }
  if (g.sample) atomicAdd(&g.eedf[eedf_bin<P>(ox, oy, oz, g)], 1u);
  atomicAdd(&g.ctr[ch], 1u);
}

// One wave scatters the first n (<= 64) queue entries, then moves the rest
// (< 64) to the front.  The queue belongs to this wave alone.
template <class P, bool ATT>
__device__ __forceinline__ void drain(const Disch<P>& d, const Seg<P>& g, QEntry<P>* q,
                                      uint32_t& qn, uint32_t n) {
  const uint32_t lane = (uint32_t)(threadIdx.x & 63);
  if (lane < n) handle<P, ATT, false>(d, g, q[lane]);
  const uint32_t rest = qn - n;
  QEntry<P> t;
  if (lane < rest) t = q[n + lane];
  if (lane < rest) q[lane] = t;
  qn = rest;
}

// Channel of a collision candidate: the first k whose interpolated cumulative
// probability exceeds R (-1: null collision).  All K comparisons are made and
// the first true one is taken, so the loop has the same trip count on every
// lane.
template <class P, int KC, bool VEC>
__device__ __forceinline__ int select_channel(const Seg<P>& g, P u0, P vx, P vy, P vz,
                                              bool& ovf) {
  const int K = KC > 0 ? KC : g.K;  // KC: channel count fixed at compile time (0: any)
  const P v2 = (vx * vx + vy * vy) + vz * vz;
  const P en = g.KE * v2;
  const P sx = en * g.inv_dE;
  int i;
  P t;
  ovf = sx >= (P)(g.ne - 1);
  if (ovf) {
    i = g.ne - 2;
    t = (P)1;
  } else {
    i = (int)sx;
    t = sx - (P)i;
  }
  auto scan = [&](auto ra) {
    uint32_t hit = 0;
    if constexpr (KC > 0) {
      P pa[KC], pb[KC];
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        pa[k] = ra[k];
        pb[k] = ra[KC + k];
      }
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const P pk = pa[k] + t * (pb[k] - pa[k]);
        hit |= (u0 < pk ? 1u : 0u) << k;
      }
    } else {
#pragma unroll 4
      for (int k = 0; k < K; ++k) {  // unrolled so that the row loads issue together
        const P pa = ra[k];
        const P pb = ra[K + k];
        const P pk = pa + t * (pb - pa);
        hit |= (u0 < pk ? 1u : 0u) << k;
      }
    }
    return hit ? __builtin_ctz(hit) : -1;
  };
  // rows i and i+1 from LDS when both are there, else through the cache
  if (i + 1 < g.tab_rows) {
    if constexpr (KC == 0 && VEC) {
      // rows of a whole number of 16-byte vectors (K a multiple of 4 in
      // FP32, of 2 in FP64) start 16-byte aligned: one LDS read per vector
      // (left out where the registers are short: the segment-write variant)
      constexpr int kL = 16 / (int)sizeof(P);
      if (K % kL == 0) {
        typedef __attribute__((ext_vector_type(kL))) P V;
        const P* ra = g.tab + i * K;
        // Each interpolated value a + t (b - a), 0 <= t <= 1, is at most
        // max(a, b)(1 + 3u) with u the unit roundoff, and the cumulative rows
        // peak at their last channel: at or above this bound no channel is
        // hit, so most null candidates skip the loop.
        constexpr double kSlack = sizeof(P) == 4 ? 0x1p-21 : 0x1p-50;
        const P top = fmax(ra[K - 1], ra[2 * K - 1]) * (P)(1.0 + kSlack);
        if (!(u0 < top)) return -1;
        uint32_t hit = 0;
#pragma unroll 1
        for (int k = 0; k < K; k += kL) {
          const V a = *reinterpret_cast<const V*>(ra + k);
          const V b = *reinterpret_cast<const V*>(ra + K + k);
#pragma unroll
          for (int l = 0; l < kL; ++l) {
            const P pk = a[l] + t * (b[l] - a[l]);
            hit |= (u0 < pk ? 1u : 0u) << (k + l);
          }
        }
        return hit ? __builtin_ctz(hit) : -1;
      }
    }
    return scan(g.tab + i * K);
  }
  return scan(g.tab_g + (size_t)i * K);
}

// Event counts of one wave, accumulated over a segment.  Each lane counts its
// own particles (a vector add per event) instead of a ballot and popcount per
// slot, whose 64-bit masks the compiler otherwise keeps in scalar registers.
struct WaveCounts {  // per lane; summed over the wave once per segment
  uint32_t absl = 0, absr = 0, ovf = 0, pushed = 0;
};

// One thread's four slots of a chunk as loaded from HBM.
template <class P>
struct ChunkIn {
  uint32_t id[4];
  int32_t c[4];
  P off[4], vz[4], vx[4], vy[4];
};

// Issue the loads of chunk lc (ids first: the random numbers need only them).
// NP: nontemporal hint on ids, cells and offsets; NV: on the velocities.
template <class P, bool NP, bool NV, int W>
__device__ __forceinline__ void chunk_load(const Seg<P>& g, uint32_t lc, ChunkIn<P>& x) {
  const uint32_t i0 = lc * (uint32_t)(W * kSub) + (uint32_t)threadIdx.x * (uint32_t)kPerThread;
  gld4<NP>(g.id + i0, x.id);
  __builtin_amdgcn_sched_barrier(0);  // keep the id load ahead of the others
  gld4<NP>(g.cell + i0, x.c);
  gld4<NP>(g.off + i0, x.off);
  gld4<NV>(g.vz + i0, x.vz);
  gld4<NV>(g.vx + i0, x.vx);
  gld4<NV>(g.vy + i0, x.vy);
}

// One wave's 256 slots of a chunk: push, removal and write-back, then the
// null-collision test and channel, the deposit at x^{n+1}; collisions are
// queued.  No workgroup barrier is involved.
//
// How a chunk's particle data arrive (the vector-memory counter counts
// loads and stores alike, and while both are outstanding the compiler can
// only wait for all of them):
// LM = 0: the previous chunk's stores drain first, then this chunk's loads
//   go out, so that each use below waits for its own load (the ids first,
//   for the random numbers) instead of for all of them.
// LM = 1: nx holds this chunk's loads, issued one chunk earlier; after the
//   drain (which now also covers them) the next chunk's loads go out into
//   nx, so that they arrive while this chunk computes (24 more registers).
// LM = 2: the loads go out at once, without the drain; the first use waits
//   for them and for the previous chunk's stores together, so that the
//   store and load latencies overlap.
// M = LM + 4 NP + 8 NV + 16 SW: with NP the loads and write-backs of ids,
// cells and offsets carry the nontemporal hint (streamed once per launch),
// with NV those of the velocities too.  Velocities without the hint stay in
// the caches, where the collision handler's scattered velocity writes then
// land (as partial writes to lines that have left the caches they cost a
// read-modify-write in memory), and at particle counts whose velocities fit
// the MALL, they stay there between steps.  With SW the chunk's collisions
// are all handled before its velocities are written: the new velocities
// return to their lanes, v_z is written whole, and v_x, v_y are written for
// every 16-particle (64-byte) segment that holds a collision, so that no
// write is narrower than a segment.
template <class P, int KC, int M, int W>
__device__ void wave_chunk(const Disch<P>& d, const Seg<P>& g, uint32_t lc, QEntry<P>* q,
                           uint32_t& qn, WaveCounts& wc, ChunkIn<P>& nx, bool more) {
  constexpr int LM = M & 3;
  constexpr bool NP = (M & 4) != 0, NV = (M & 8) != 0, SW = (M & 16) != 0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const uint32_t i0 = lc * (uint32_t)(W * kSub) + (uint32_t)tid * (uint32_t)kPerThread;
  if constexpr (LM != 2) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) only
  ChunkIn<P> in;
  if constexpr (LM == 1) {
    in = nx;
    if (more) chunk_load<P, NP, NV, W>(g, lc + 1u, nx);
    __builtin_amdgcn_sched_barrier(0);
  } else {
    chunk_load<P, NP, NV, W>(g, lc, in);
  }
  int32_t(&c)[4] = in.c;
  P(&off)[4] = in.off;
  P(&vx)[4] = in.vx;
  P(&vy)[4] = in.vy;
  P(&vz)[4] = in.vz;
  const uint32_t(&id)[4] = in.id;
  // the null-collision numbers first: one Philox block of stream (tag 0,
  // id, step) per slot needs only the ids, so it runs while the other
  // particle arrays are still arriving
  P u0[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t w0, w1, w2, w3;
    philox4x32_10_v(id[j], g.step, 0u, kTagElectron, g.seed_lo, g.seed_hi, w0, w1, w2, w3);
    if constexpr (sizeof(P) == 4)
      u0[j] = (P)u01_f32(w0);
    else
      u0[j] = (P)u01_f64(w0, w1);
  }
  bool alive[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    // leapfrog push with the linear gather of E', written with selects
    // (dead slots keep their contents)
    const bool live = (i0 + (uint32_t)j < g.n_main) && (c[j] >= 0);
    const int32_t cc = live ? c[j] : 0;
    const P e0 = g.ep[cc];
    const P e1 = g.ep[cc + 1];
    const P t1 = e1 - e0;
    const P gg = e0 + off[j] * t1;
    const P vzn = vz[j] + gg;
    const P s = off[j] + vzn * g.kdz;
    const P f = floor(s);
    const bool outl = !(f >= (P)(-cc));
    const bool outr = !outl && (f >= (P)(g.nc - cc));
    const bool stay = live && !outl && !outr;
    const P on0 = s - f;
    const bool wrap = on0 == (P)1;
    const int32_t cn = cc + (stay ? (int32_t)f : 0) + (wrap ? 1 : 0);
    wc.pushed += live ? 1u : 0u;
    wc.absl += (live && outl) ? 1u : 0u;
    wc.absr += (live && outr) ? 1u : 0u;
    vz[j] = live ? vzn : vz[j];
    c[j] = stay ? cn : (live ? -1 : c[j]);
    off[j] = stay ? (wrap ? (P)0 : on0) : off[j];
    alive[j] = stay;
  }
  // write back (vx, vy unchanged; collided particles get theirs when
  // scattered); issued early so that they retire behind the Philox work
  gst4<NP>(g.cell + i0, c);
  gst4<NP>(g.off + i0, off);
  if constexpr (!SW) gst4<NV>(g.vz + i0, vz);
  int ch[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    // null-collision test
    ch[j] = -1;
    bool ovf = false;
    if (alive[j] && u0[j] < g.Pmax) ch[j] = select_channel<P, KC, !SW>(g, u0[j], vx[j], vy[j], vz[j], ovf);
    wc.ovf += ovf ? 1u : 0u;
    // an attached electron leaves before the deposit (its charge goes to
    // the negative ion when the collision is handled); the three-channel
    // path serves only tables without attachment
    if constexpr (KC == 0)
      if (g.att_mask && ch[j] >= 0 && ((g.att_mask >> ch[j]) & 1u)) alive[j] = false;
  }
  // deposit at x^{n+1}.  W0 + W1 = 2^32 per particle, so a run of m
  // particles in one cell adds m 2^32 - sum W1 to its left node and sum W1
  // to its right node.  Runs of equal cells are merged per thread, then over
  // the wave when the whole wave sits in one cell (sorted particles).
  int rc = -1;
  uint64_t a1 = 0;
  uint32_t m = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!alive[j]) continue;
    const uint64_t W1 = cic_w1u<P>(off[j]);
    if (c[j] == rc) {
      a1 += W1;
      m += 1;
    } else {
      if (rc >= 0) {
        lds_add_i64(&g.bins[rc], ((uint64_t)m << 32) - a1);
        lds_add_i64(&g.bins[rc + 1], a1);
      }
      rc = c[j];
      a1 = W1;
      m = 1;
    }
  }
  const uint64_t act = __ballot(rc >= 0);
  if (act) {
    const int lead = __ffsll((unsigned long long)act) - 1;
    const int rl = __builtin_amdgcn_readlane(rc, lead);
    if (__ballot(rc >= 0 && rc != rl) == 0) {
      const uint64_t s1 = wave_sum_u64(rc >= 0 ? a1 : 0);
      const uint32_t sm = wave_sum_u32(rc >= 0 ? m : 0);
      if (lane == lead) {
        lds_add_i64(&g.bins[rl], ((uint64_t)sm << 32) - s1);
        lds_add_i64(&g.bins[rl + 1], s1);
      }
    } else if (rc >= 0) {
      lds_add_i64(&g.bins[rc], ((uint64_t)m << 32) - a1);
      lds_add_i64(&g.bins[rc + 1], a1);
    }
  }
  // EEDF of the survivors that did not collide
  if (g.sample) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (alive[j] && ch[j] < 0) atomicAdd(&g.eedf[eedf_bin<P>(vx[j], vy[j], vz[j], g)], 1u);
  }
  // children are numbered in particle order within the sub-chunk
  const uint64_t lt = lanemask_lt();
  uint32_t kid = 0, nk = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool ion = ch[j] >= 0 && ((g.ion_mask >> ch[j]) & 1u);
    const uint64_t mk = __ballot(ion);
    kid += (uint32_t)__popcll(mk & lt);
    nk += (uint32_t)__popcll(mk);
  }
  if (lane == 0) {
    const uint32_t u = lc * (uint32_t)W + (uint32_t)wv;
    gptr(d.chunk_kids)[u] = nk;
    if (u - g.kbase < kKidsLds) g.kl[u - g.kbase] = nk;
  }
  // queue the collisions, one slot index j at a time, and scatter in 64s
  // SW: byte j of qp is the queue index of this lane's slot j while its
  // collision waits (0xFF: none); handle the first n entries, bring their
  // new velocities back to the slots' lanes, then move the rest to the front
  uint32_t qp = 0xFFFFFFFFu;
  auto batch = [&](uint32_t n) {
    if ((uint32_t)lane < n) handle<P, KC == 0, true>(d, g, q[lane]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t at = (qp >> (8 * j)) & 0xFFu;
      if (at < n) {
        vx[j] = q[at].vx;
        vy[j] = q[at].vy;
        vz[j] = q[at].vz;
        qp |= 0xFFu << (8 * j);
      } else if (at != 0xFFu) {
        qp -= n << (8 * j);
      }
    }
    const uint32_t rest = qn - n;
    QEntry<P> t;
    if ((uint32_t)lane < rest) t = q[n + (uint32_t)lane];
    __builtin_amdgcn_wave_barrier();
    if ((uint32_t)lane < rest) q[lane] = t;
    __builtin_amdgcn_wave_barrier();
    qn = rest;
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool col = ch[j] >= 0;
    const uint64_t mk = __ballot(col);
    if (mk == 0) continue;
    if (col) {
      const bool ion = (g.ion_mask >> ch[j]) & 1u;
      const uint32_t at = qn + (uint32_t)__popcll(mk & lt);
      QEntry<P>& e = q[at];
      e.vx = vx[j];
      e.vy = vy[j];
      e.vz = vz[j];
      e.off = off[j];
      e.id = id[j];
      e.c = c[j];
      e.slot = i0 + (uint32_t)j;
      e.meta = (uint32_t)ch[j] | (ion ? (0x100u | (kid << 16)) : 0u);
      kid += ion ? 1u : 0u;
      if constexpr (SW) qp = (qp & ~(0xFFu << (8 * j))) | (at << (8 * j));
    }
    qn += (uint32_t)__popcll(mk);
    if (qn >= 64u) {
      if constexpr (SW)
        batch(64u);
      else
        drain<P, KC == 0>(d, g, q, qn, 64u);
    }
  }
  if constexpr (SW) {
    if (qn) batch(qn);  // the rest of this chunk's collisions
    gst4<NV>(g.vz + i0, vz);
    const bool hit = (ch[0] >= 0) || (ch[1] >= 0) || (ch[2] >= 0) || (ch[3] >= 0);
    const uint64_t seg = __ballot(hit) >> ((uint32_t)lane & ~3u);
    if (seg & 0xFull) {  // a collision among the 16 slots of these four lanes
      gst4<NV>(g.vx + i0, vx);
      gst4<NV>(g.vy + i0, vy);
    }
  }
}

// Copies na elements of sa to da and nb of sb to db (LDS), issuing all of a
// thread's loads of a round before its first store, so that a segment's set-up
// waits for one memory round trip per round instead of one per element.
template <int NT, class T>
__device__ __forceinline__ void lds_copy2(T* da, const Gp<T>* sa, int na, T* db,
                                          const Gp<T>* sb, int nb) {
  constexpr int B = 8;  // elements per thread and array per round
  constexpr int nt = NT;
  const int tid = threadIdx.x;
  const int n = na > nb ? na : nb;
  for (int r = 0; r < n; r += B * nt) {
    T va[B], vb[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = r + u * nt + tid;
      if (i < na) va[u] = sa[i];
      if (i < nb) vb[u] = sb[i];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = r + u * nt + tid;
      if (i < na) da[i] = va[u];
      if (i < nb) db[i] = vb[u];
    }
  }
}

// Block-wide exclusive scan of one value per thread of a workgroup of W
// waves; writes the total to *total.  sh: W words of LDS.
template <int W>
__device__ __forceinline__ uint32_t wg_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  lds_barrier();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t s = sh[w];
    if (w < wv) base += s;
    tot += s;
  }
  lds_barrier();
  *total = tot;
  return base + x - v;
}

// Chunks [lc0, lc1) of discharge d by particle workgroup pb; chunk0 is the
// launch-wide index of the discharge's first chunk and per the chunks per
// workgroup (chunks of this launch's workgroup size).
template <class P, int M, int W>
__device__ void segment(const Disch<P>& d, uint32_t lc0, uint32_t lc1, unsigned char* smem,
                        const Lds& L, uint32_t pb, uint32_t chunk0, uint32_t per) {
  const int tid = threadIdx.x, wv = tid >> 6, nt = W * 64;
  P* tab = reinterpret_cast<P*>(smem + L.tab);
  P* ep = reinterpret_cast<P*>(smem + L.ep);
  State* st = d.st;
  Seg<P> g;
  g.tab = tab;
  g.ep = ep;
  g.bins = reinterpret_cast<int64_t*>(smem + L.bins);
  g.eedf = reinterpret_cast<uint32_t*>(smem + L.eedf);
  g.ctr = reinterpret_cast<uint32_t*>(smem + L.ctr);
  g.tab_g = gptr(d.tab);
  const int buf = st->buf;
  g.cell = gptr(d.cell[buf]);
  g.off = gptr(d.off[buf]);
  g.vx = gptr(d.vx[buf]);
  g.vy = gptr(d.vy[buf]);
  g.vz = gptr(d.vz[buf]);
  g.id = gptr(d.id[buf]);
  g.kdz = d.kdz;
  g.Pmax = d.Pmax;
  g.KE = d.KE;
  g.inv_dE = d.inv_dE;
  g.keedf = d.keedf;
  g.tab_rows = d.ne < (int)L.rows ? d.ne : (int)L.rows;
  g.nc = d.nc;
  g.ne = d.ne;
  g.K = d.K;
  g.nbins = d.nbins;
  g.ion_mask = d.ion_mask;
  g.att_mask = d.att_mask;
  g.seed_lo = (uint32_t)d.seed;
  g.seed_hi = (uint32_t)(d.seed >> 32);
  g.step = (uint32_t)st->step;
  g.n_main = st->n_main;
  g.sample = ((st->step + 1) % d.eedf_every) == 0;
  g.kl = reinterpret_cast<uint32_t*>(smem + L.kids);
  g.kbase = lc0 * (uint32_t)W;
  QEntry<P>* q = reinterpret_cast<QEntry<P>*>(smem + L.q) + (size_t)wv * kWQ;
  lds_copy2<W * 64>(tab, gptr(d.tab), g.tab_rows * d.K, ep, gptr(d.Ep), d.nn);
  for (int i = tid; i < d.nn; i += nt) g.bins[i] = 0;
  for (int i = tid; i <= d.nbins; i += nt) g.eedf[i] = 0;
  if (tid < kCtrN) g.ctr[tid] = 0;
  // the deposit grid's pointer goes to scalar registers now, so that no wait
  // for it (and for the particle stores in flight behind it) is left for the
  // flush at the end
  int64_t* cnt = uniform_ptr(d.cnt[st->cbuf ^ 1]);
  lds_barrier();  // LDS stores wait for the loads they copy
  uint32_t qn = 0;
  WaveCounts wc;
  ChunkIn<P> nx;
  if constexpr ((M & 3) == 1) chunk_load<P, (M & 4) != 0, (M & 8) != 0, W>(g, lc0, nx);
  if (g.K == 3 && g.att_mask == 0) {  // elastic, excitation, ionization: unrolled
    for (uint32_t lc = lc0; lc < lc1; ++lc)
      wave_chunk<P, 3, M, W>(d, g, lc, q, qn, wc, nx, lc + 1u < lc1);
    if (qn) drain<P, false>(d, g, q, qn, qn);
  } else {
    for (uint32_t lc = lc0; lc < lc1; ++lc)
      wave_chunk<P, 0, M, W>(d, g, lc, q, qn, wc, nx, lc + 1u < lc1);
    if (qn) drain<P, true>(d, g, q, qn, qn);
  }
  wc.absl = wave_sum_u32(wc.absl);
  wc.absr = wave_sum_u32(wc.absr);
  wc.ovf = wave_sum_u32(wc.ovf);
  wc.pushed = wave_sum_u32(wc.pushed);
  if ((tid & 63) == 0) {
    if (wc.absl) atomicAdd(&g.ctr[kCtrAbsL], wc.absl);
    if (wc.absr) atomicAdd(&g.ctr[kCtrAbsR], wc.absr);
    if (wc.ovf) atomicAdd(&g.ctr[kCtrOverflow], wc.ovf);
    if (wc.pushed) atomicAdd(&g.ctr[kCtrPushed], wc.pushed);
  }
  // Offsets of the segment's children relative to the segment (exclusive
  // scan of the sub-chunk counts) and the segment's total, ahead of the
  // flushes so that nothing waits for their atomics.  The counts come from
  // LDS when the segment has at most kKidsLds sub-chunks; otherwise from
  // memory, after a barrier that waits for every wave's stores.
  const uint32_t k0 = lc0 * (uint32_t)W, k1 = lc1 * (uint32_t)W;
  const bool kids_lds = k1 - k0 <= kKidsLds;
  if (kids_lds)
    lds_barrier();
  else
    __syncthreads();
  {
    __shared__ uint32_t sh[W];
    Gp<uint32_t>* kbase = gptr(d.chunk_base);
    uint32_t carry = 0;
    if (kids_lds) {  // at most kKidsLds <= kElecThreads counts: one round
      const uint32_t k = k0 + (uint32_t)tid;
      const uint32_t v = k < k1 ? g.kl[tid] : 0u;
      const uint32_t ex = wg_scan<W>(v, sh, &carry);
      if (k < k1) kbase[k] = ex;
    } else {
      const Gp<uint32_t>* kids = gptr(d.chunk_kids);
      for (uint32_t kb = k0; kb < k1; kb += (uint32_t)nt) {
        const uint32_t k = kb + (uint32_t)tid;
        const uint32_t v = k < k1 ? kids[k] : 0u;
        uint32_t tot;
        const uint32_t ex = wg_scan<W>(v, sh, &tot);
        if (k < k1) kbase[k] = carry + ex;
        carry += tot;
      }
    }
    if (tid == 0) {
      gptr(d.seg)[pb] = carry;
      if (lc0 == 0) {  // in chunks of kTile slots, whatever this launch's chunk
        constexpr uint32_t r = (uint32_t)(W * kSub / kTile);
        st->seg_off = chunk0 * r;
        st->seg_per = per * r;
      }
    }
  }
  for (int i = tid; i < d.nn; i += nt) {
    const int64_t v = g.bins[i];
    if (v) atomic_add_i64(&cnt[i], v);
  }
  if (g.sample)
    for (int i = tid; i <= d.nbins; i += nt)
      if (g.eedf[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&d.eedf[i]),
                               (unsigned long long)g.eedf[i]);
  const uint32_t* ctr = g.ctr;
  if (tid < d.K && ctr[tid]) atomicAdd(reinterpret_cast<unsigned long long*>(&st->coll[tid]),
                                       (unsigned long long)ctr[tid]);
  if (tid == kCtrAbsL && ctr[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->absorbed[0]), (unsigned long long)ctr[tid]);
  if (tid == kCtrAbsR && ctr[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->absorbed[1]), (unsigned long long)ctr[tid]);
  if (tid == kCtrCreated && ctr[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->created), (unsigned long long)ctr[tid]);
  if (tid == kCtrOverflow && ctr[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->overflow), (unsigned long long)ctr[tid]);
  if (tid == kCtrPushed && ctr[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->pushed), (unsigned long long)ctr[tid]);
  lds_barrier();  // the next segment of this workgroup reuses the LDS
}

// ---- ion fluid -----------------------------------------------------------

__device__ __forceinline__ double dmin0(double e) { return (0.0 < e) ? 0.0 : e; }  // min(e, 0)
__device__ __forceinline__ double dmax0(double e) { return (e < 0.0) ? 0.0 : e; }  // max(e, 0)

template <class P>
__device__ __forceinline__ double ion_temperature(const Disch<P>& d, double mu, double E) {
  const double x = mu * fabs(E);
  return d.TN + d.kappa * (x * x);
}

// Fitted He+ transport in He at atmospheric pressure (Sec. III): mobility
// versus |E| (Table 2, branch change at E0 = 1.47e6 V/m) and momentum-exchange
// frequency versus |u| (Table 3, branch change at u0 = 2e3 m/s).  The
// non-integer powers go through fit_log / fit_exp.
__device__ __forceinline__ double fit_pow(double x, double y) {
  return x > 0.0 ? fit_exp(y * fit_log(x)) : 0.0;
}

// Table 2 [m^2/(V s)]
__device__ __forceinline__ double mobility_fit(double E) {
  const double a = fabs(E), E0 = 1.47e6;
  if (a < E0) return 1e-3 * (1.18 - 0.185 * (a / E0));
  return 1e-3 * (0.94 * fit_pow(E0 / a, 0.3));
}

// Table 3 [1/s]
__device__ __forceinline__ double nu_fit(double u) {
  const double a = fabs(u), u0 = 2e3;
  if (a < u0) return 1e10 * (2.07 + 0.88 * fit_pow(a / u0, 1.89));
  return 1e10 * (1.54 + 1.36 * (a / u0));
}

// Drift-diffusion, explicit: Eq (2.5) with Eqs (2.7)-(2.8) and central
// differences, field-switched drift flux at the walls, then Eq (2.4) with
// half cells at the walls.  The mobility is constant or, with the fitted
// transport, Table 2 at each node's own field.  Gamma goes through LDS; n is
// updated in place after a barrier (each node then reads only its own old
// density).
template <class P>
__device__ void fluid_dd(const Disch<P>& d, double* lds) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn;
  double* __restrict__ ni = d.ni;
  const double* __restrict__ E = d.E;
  double* G = lds;
  const bool fit = d.ion_model == HD_ION_DD_FIT_MU;
  for (int j = tid; j < nn; j += (int)blockDim.x) {
    const double ej = E[j];
    const double mu = fit ? mobility_fit(ej) : d.mu;
    double g;
    if (j == 0) {
      g = (mu * ni[0]) * dmin0(ej);
    } else if (j == nc) {
      g = (mu * ni[nc]) * dmax0(ej);
    } else {
      const double nl = ni[j - 1], nj = ni[j], nr = ni[j + 1];
      const double T = ion_temperature(d, mu, ej);
      const double Dc = (mu * T) / kECharge;
      g = (mu * nj) * ej - (Dc * (nr - nl)) * d.inv_2dz;
    }
    G[j] = g;
  }
  __syncthreads();
  for (int j = tid; j < nn; j += (int)blockDim.x) {
    double v;
    if (j == 0)
      v = ni[0] - d.dt_dz * (G[1] - G[0]);
    else if (j == nc)
      v = ni[nc] - d.dt_dz * (G[nc] - G[nc - 1]);
    else
      v = ni[j] - d.dt_2dz * (G[j + 1] - G[j - 1]);
    ni[j] = v;
    d.gam[j] = G[j];
  }
  if (tid == 0) {
    d.st->wall[0] = G[0];
    d.st->wall[1] = G[nc];
  }
  __syncthreads();
}

// Full fluid: Eq (2.3) for Gamma^{n+1/2} with lagged nu and semi-implicit
// advection (tridiagonal, partitioned solve), drift wall fluxes with
// mu = e/(M nu) (Eq 2.6), then Eq (2.4).  nu is constant or, with the fitted
// transport, Table 3 at each node's lagged u.  Each row reads the old n,
// Gamma and E of its neighbours directly and re-derives their nu (the
// per-node values would not fit in LDS beside the coefficients at the
// largest grids); the coefficients live in LDS for the solve.
template <class P>
__device__ __forceinline__ double lagged_u(const Disch<P>& d, double n, double g) {
  return (n > d.nfloor) ? g / n : 0.0;
}

template <class P>
__device__ void fluid_full(const Disch<P>& d, double* lds) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn, m = nc - 1;
  double* __restrict__ ni = d.ni;
  double* __restrict__ gam = d.gam;
  const double* __restrict__ E = d.E;
  const bool fit = d.ion_model == HD_ION_FULL_FIT_NU;
  // mu = e/(M nu) at a node with lagged speed u
  auto mu_at = [&](double u) { return fit ? kECharge / (d.M * nu_fit(u)) : d.mu_full; };
  double* La = lds;
  double* Lb = La + nn;
  double* Lc = Lb + nn;
  double* Lr = Lc + nn;
  for (int j = 1 + tid; j <= m; j += (int)blockDim.x) {
    const double nl = ni[j - 1], nj = ni[j], nr = ni[j + 1];
    const double gl_ = gam[j - 1], gj = gam[j], gr_ = gam[j + 1];
    const double el = E[j - 1], ej = E[j], er = E[j + 1];
    const double ul = lagged_u(d, nl, gl_), ur = lagged_u(d, nr, gr_);
    const double nu = fit ? nu_fit(lagged_u(d, nj, gj)) : d.nu;
    const double Tl = ion_temperature(d, mu_at(ul), el), Tr = ion_temperature(d, mu_at(ur), er);
    const int k = j - 1;
    La[k] = -d.dt_2dz * ul;
    Lb[k] = 1.0 + nu * d.hdt;
    Lc[k] = d.dt_2dz * ur;
    Lr[k] = (gj * (1.0 - nu * d.hdt) + (d.e_M_dt * nj) * ej) - d.dt_2dzM * (nr * Tr - nl * Tl);
  }
  const double gl = (mu_at(lagged_u(d, ni[0], gam[0])) * ni[0]) * dmin0(E[0]);
  const double gr = (mu_at(lagged_u(d, ni[nc], gam[nc])) * ni[nc]) * dmax0(E[nc]);
  __syncthreads();
  if (tid == 0) {
    Lr[0] = Lr[0] - La[0] * gl;
    Lr[m - 1] = Lr[m - 1] - Lc[m - 1] * gr;
    d.st->wall[0] = gl;
    d.st->wall[1] = gr;
  }
  solve_tridiag_block<2>(m, La, Lb, Lc, Lr, lds + 4 * nn);  // Gamma^{n+1/2} -> Lb
  for (int j = tid; j < nn; j += (int)blockDim.x) {
    // Gamma^{n+1/2} at j-1, j, j+1 (walls: gl, gr) and the continuity update
    auto G = [&](int i) { return i == 0 ? gl : (i == nc ? gr : Lb[i - 1]); };
    double v;
    if (j == 0)
      v = ni[0] - d.dt_dz * (G(1) - G(0));
    else if (j == nc)
      v = ni[nc] - d.dt_dz * (G(nc) - G(nc - 1));
    else
      v = ni[j] - d.dt_2dz * (G(j + 1) - G(j - 1));
    ni[j] = v;
    gam[j] = G(j);
  }
  __syncthreads();
}

// Several drift-diffusion species (ion model 4): the mobility of species q
// at field E from its table on log-spaced E/N, linear in ln(E/N), end values
// outside.
template <class P>
__device__ __forceinline__ double species_mu(const Disch<P>& d, int q, double E) {
  const double* tab = d.mu_tab + (size_t)q * kMaxMu;
  const double x = (fabs(E) / d.n_gas) * 1e21;
  if (!(x > d.mu_lo[q])) return tab[0];
  const double u = (fit_log(x) - d.mu_L0[q]) * d.mu_inv_dL[q];
  if (!(u > 0.0)) return tab[0];
  const int n = d.n_mu[q];
  if (!(u < (double)(n - 1))) return tab[n - 1];
  const int k = (int)u;
  const double t = u - (double)k;
  return tab[k] + t * (tab[k + 1] - tab[k]);
}

// Each species in turn: Gamma_j = Z mu n_j E_j - D_j (n_{j+1} - n_{j-1})/(2 dz)
// with D = mu T / e and T from Eq (2.8) with the species' mass; at the walls
// the drift flux only when it points into the wall; then Eq (2.4).  The
// net charge flux sum_s Z_s Gamma_s at the walls goes to the state (absorbed
// power) and the positive-ion flux into each wall (emission).
template <class P>
__device__ void fluid_species(const Disch<P>& d, double* lds) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn;
  const double* __restrict__ E = d.E;
  double* G = lds;
  double w0 = 0.0, w1 = 0.0, f0 = 0.0, f1 = 0.0;
  for (int q = 0; q < d.S; ++q) {
    double* __restrict__ ni = d.ni + (size_t)q * nn;
    double* __restrict__ gam = d.gam + (size_t)q * nn;
    const double Zd = (double)d.Z[q];
    const double kap = d.kappa_s[q];
    for (int j = tid; j < nn; j += (int)blockDim.x) {
      const double ej = E[j];
      const double mu = species_mu(d, q, ej);
      double g;
      if (j == 0) {
        g = dmin0(((Zd * mu) * ni[0]) * ej);
      } else if (j == nc) {
        g = dmax0(((Zd * mu) * ni[nc]) * ej);
      } else {
        const double nl = ni[j - 1], nj = ni[j], nr = ni[j + 1];
        const double x = mu * fabs(ej);
        const double T = d.TN + kap * (x * x);
        const double Dc = (mu * T) / kECharge;
        g = ((Zd * mu) * nj) * ej - (Dc * (nr - nl)) * d.inv_2dz;
      }
      G[j] = g;
    }
    __syncthreads();
    for (int j = tid; j < nn; j += (int)blockDim.x) {
      double v;
      if (j == 0)
        v = ni[0] - d.dt_dz * (G[1] - G[0]);
      else if (j == nc)
        v = ni[nc] - d.dt_dz * (G[nc] - G[nc - 1]);
      else
        v = ni[j] - d.dt_2dz * (G[j + 1] - G[j - 1]);
      ni[j] = v;
      gam[j] = G[j];
    }
    if (tid == 0) {
      w0 = w0 + Zd * G[0];
      w1 = w1 + Zd * G[nc];
      if (d.Z[q] > 0) {
        f0 = f0 + dmax0(-G[0]);
        f1 = f1 + dmax0(G[nc]);
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    d.st->wall[0] = w0;
    d.st->wall[1] = w1;
    d.st->see_flux[0] = f0;
    d.st->see_flux[1] = f1;
  }
}

// Blocks [0, D) advance the ion fluid of discharge blockIdx.x; the others
// share the particle chunks of all discharges in contiguous segments.
template <class P, int M, int W>
__device__ __forceinline__ void electron_body(const Disch<P>* __restrict__ ds, const ElecArgs& a,
                                              unsigned char* smem) {
  const int D = a.D;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < D) {
    const Disch<P>& d = ds[blockIdx.x];
    if (d.st->steps_left > 0) {
      if (d.ion_model == HD_ION_DD_SPECIES)
        fluid_species<P>(d, reinterpret_cast<double*>(smem));
      else if (d.ion_model == HD_ION_DD_CONST_MU || d.ion_model == HD_ION_DD_FIT_MU)
        fluid_dd<P>(d, reinterpret_cast<double*>(smem));
      else
        fluid_full<P>(d, reinterpret_cast<double*>(smem));
    }
    return;
  }
  const Lds L = lds_layout<P>(a);
  uint32_t* pre = reinterpret_cast<uint32_t*>(smem + L.pre);
  // chunks of discharge i (none when it has no steps left)
  auto chunks = [&](int i) {
    const State* st = ds[i].st;
    const int64_t left = st->steps_left;  // both loads issued together
    const uint32_t n_main = st->n_main;
    constexpr uint32_t chunk = (uint32_t)(W * kSub);
    const uint32_t nch = (n_main + chunk - 1u) / chunk;
    return nch & (left > 0 ? ~0u : 0u);
  };
  if (D <= 4) {  // a few discharges: a serial prefix in LDS
    if (tid < D) pre[tid + 1] = chunks(tid);
    if (tid == 0) pre[0] = 0;
    lds_barrier();
    if (tid == 0)
      for (int i = 0; i < D; ++i) pre[i + 1] += pre[i];
  } else if (tid < 64) {  // a batch: wave scans of 64 discharges at a time
    uint32_t carry = 0;
    for (int b = 0; b < D; b += 64) {
      const int i = b + tid;
      const uint32_t v = i < D ? chunks(i) : 0u;
      uint32_t x = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (tid >= o) x += y;
      }
      if (i < D) pre[i + 1] = carry + x;
      carry += __shfl(x, 63, 64);
    }
    if (tid == 0) pre[0] = 0;
  }
  lds_barrier();
  const uint32_t total = pre[D];
  const uint32_t G = gridDim.x - (uint32_t)D, pb = blockIdx.x - (uint32_t)D;
  const uint32_t per = (total + G - 1u) / G;
  uint32_t g0 = pb * per;
  const uint32_t g1 = min(total, g0 + per);
  if (g0 >= g1) return;
  int di = 0;
  while (pre[di + 1] <= g0) ++di;
  while (g0 < g1) {
    const uint32_t end = min(g1, pre[di + 1]);
    // a discharge with no chunks (idle, or an empty slot whose descriptor
    // has no arrays) between two others gets no segment
    if (end > g0)
      segment<P, M, W>(ds[di], g0 - pre[di], end - pre[di], smem, L, pb, pre[di], per);
    g0 = end;
    ++di;
  }
}

// FP32: at most 128 VGPRs so that four waves share each SIMD.  Each kernel
// but the register-prefetch one has a wide twin (suffix _w): the same body
// with 1,024-thread workgroups, one per CU, for grids whose LDS leaves room
// for only one narrow workgroup per CU.
template <int M, int W>
__device__ __forceinline__ void f32_body(const Disch<float>* __restrict__ ds, const ElecArgs& a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<float, M, W>(ds, a, smem);
}
#define HD_F32_KERNEL(NAME, M)                                                                \
  __global__ __launch_bounds__(kElecThreads) __attribute__((amdgpu_waves_per_eu(4))) void     \
  NAME(const Disch<float>* __restrict__ ds, ElecArgs a) {                                    \
    f32_body<M, 8>(ds, a);                                                                   \
  }                                                                                          \
  __global__ __launch_bounds__(kElecThreadsWide) __attribute__((amdgpu_waves_per_eu(4))) void \
  NAME##_w(const Disch<float>* __restrict__ ds, ElecArgs a) {                                \
    f32_body<M, 16>(ds, a);                                                                  \
  }
HD_F32_KERNEL(k_electron_f32, 0)
// loads issued without draining the stores first
HD_F32_KERNEL(k_electron_f32_nd, 2)
// nontemporal particle loads and write-backs (for particle stores far beyond
// the MALL), with and without the drain; then the same with the velocities
// left to the caches
HD_F32_KERNEL(k_electron_f32_nt, 12)
HD_F32_KERNEL(k_electron_f32_nd_nt, 14)
HD_F32_KERNEL(k_electron_f32_np, 4)
HD_F32_KERNEL(k_electron_f32_nd_np, 6)
// all particle traffic nontemporal and each chunk's collisions handled
// before its velocities are written (whole segments only)
HD_F32_KERNEL(k_electron_f32_nt_sw, 28)
#undef HD_F32_KERNEL

// FP32 with the next chunk's loads in flight: at most 168 VGPRs, three
// waves per SIMD.
__global__ __launch_bounds__(kElecThreads) __attribute__((amdgpu_waves_per_eu(3))) void
k_electron_f32_pf(const Disch<float>* __restrict__ ds, ElecArgs a) {
  f32_body<1, 8>(ds, a);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64(const Disch<double>* __restrict__ ds,
                                                               ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 0, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_pf(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 1, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_nd(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 2, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_nt(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 12, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_nd_nt(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 14, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_np(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 4, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_nd_np(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 6, 8>(ds, a, smem);
}

__global__ __launch_bounds__(kElecThreads) void k_electron_f64_nt_sw(
    const Disch<double>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  electron_body<double, 28, 8>(ds, a, smem);
}

// Kernels of one precision, by how the particle data arrive and leave:
// 0 drain then load, 1 next chunk prefetched, 2 no drain; 3 and 4 as 0 and 2
// with nontemporal particle traffic; 5 and 6 as 0 and 2 with nontemporal
// traffic of ids, cells and offsets only; 7 as 3 with each chunk's
// velocities written after its collisions.  Launch variants 8-15 are the
// same kernels with wide workgroups.
constexpr int kElecKernels = 8;                    // kernels per precision
constexpr int kElecVariants = kElecWide + kElecKernels;  // and each with wide workgroups
template <class P>
struct ElecKernel;
template <>
struct ElecKernel<float> {
  static constexpr decltype(&k_electron_f32) fn[kElecKernels] = {
      k_electron_f32,       k_electron_f32_pf, k_electron_f32_nd,    k_electron_f32_nt,
      k_electron_f32_nd_nt, k_electron_f32_np, k_electron_f32_nd_np, k_electron_f32_nt_sw};
  static constexpr decltype(&k_electron_f32) wide[kElecKernels] = {
      k_electron_f32_w,       nullptr,           k_electron_f32_nd_w,    k_electron_f32_nt_w,
      k_electron_f32_nd_nt_w, k_electron_f32_np_w, k_electron_f32_nd_np_w, k_electron_f32_nt_sw_w};
};
template <>
struct ElecKernel<double> {
  static constexpr decltype(&k_electron_f64) fn[kElecKernels] = {
      k_electron_f64,       k_electron_f64_pf, k_electron_f64_nd,    k_electron_f64_nt,
      k_electron_f64_nd_nt, k_electron_f64_np, k_electron_f64_nd_np, k_electron_f64_nt_sw};
  static constexpr decltype(&k_electron_f64) wide[kElecKernels] = {};
};

// The kernel of a launch variant (nullptr: no such kernel).
template <class P>
auto elec_kernel(int variant) {
  return variant >= kElecWide ? ElecKernel<P>::wide[variant - kElecWide] : ElecKernel<P>::fn[variant];
}

}  // namespace

// Variant v < kElecWide: kernel v with kElecThreads per workgroup;
// kElecWide + v: its wide twin with kElecThreadsWide (FP32 only: the FP64
// kernels and the register-prefetch kernel use more registers than sixteen
// waves per CU allow, so they have none and those variants are rejected).
inline int elec_threads(int variant) {
  return variant >= kElecWide ? kElecThreadsWide : kElecThreads;
}

template <class P>
size_t electron_lds_bytes(int D, int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max,
                          int variant) {
  return lds_layout<P>(elec_args<P>(D, tab_max, nn_max, nb1_max, fluid_nn, K_max,
                                    elec_threads(variant) / 64)).total;
}

template <class P>
hipError_t launch_electron_impl(const Disch<P>* d_dev, int D, int grid, int tab_max, int nn_max,
                                int nb1_max, int fluid_nn, int K_max, int variant, hipStream_t s) {
  if (variant < 0 || variant >= kElecVariants) return hipErrorInvalidValue;
  const int nt = elec_threads(variant);
  const ElecArgs a = elec_args<P>(D, tab_max, nn_max, nb1_max, fluid_nn, K_max, nt / 64);
  const size_t lds = lds_layout<P>(a).total;
  const auto fk = elec_kernel<P>(variant);
  if (!fk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fk, dim3(grid), dim3(nt), lds, s, d_dev, a);
  return hipGetLastError();
}

template <class P>
int electron_occupancy(int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max, int D,
                       int variant) {
  int nb = 0;
  if (variant < 0 || variant >= kElecVariants) return 0;
  const size_t lds = electron_lds_bytes<P>(D, tab_max, nn_max, nb1_max, fluid_nn, K_max, variant);
  const auto fk = elec_kernel<P>(variant);
  if (!fk) return 0;  // no wide twin
  if (hipFuncSetAttribute((const void*)fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
      hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk, elec_threads(variant), lds) !=
      hipSuccess)
    return 0;
  return nb;
}

int electron_variants() { return kElecVariants; }

template size_t electron_lds_bytes<float>(int, int, int, int, int, int, int);
template size_t electron_lds_bytes<double>(int, int, int, int, int, int, int);
template hipError_t launch_electron_impl<float>(const Disch<float>*, int, int, int, int, int, int,
                                                int, int, hipStream_t);
template hipError_t launch_electron_impl<double>(const Disch<double>*, int, int, int, int, int,
                                                 int, int, int, hipStream_t);
template int electron_occupancy<float>(int, int, int, int, int, int, int);
template int electron_occupancy<double>(int, int, int, int, int, int, int);

}  // namespace hd
