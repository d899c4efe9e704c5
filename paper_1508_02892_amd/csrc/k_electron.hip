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
#include "hd_device.h"

namespace hd {

namespace {

constexpr double kECharge = 1.602176634e-19;

template <class P>
struct QEntry {
  P vx, vy, vz, off;
  uint32_t id;
  int32_t c;
  int32_t ch;
  int32_t kid;  // child slot in the chunk's staging area, -1 if none
};

struct ElecArgs {
  int D;
  int tab_max;    // max ne*K over the batch
  int nn_max;     // max nodes
  int nb1_max;    // max eedf bins + 1
  int fluid_nn;   // max nodes of a full-fluid discharge (its solver lives in LDS), 0 if none
};

struct Lds {
  uint32_t tab, bins, q, eedf, ctr, pre, wsum, total;
};

// LDS counters: [0, kMaxK) collisions per channel, then these.
enum { kCtrAbsL = kMaxK, kCtrAbsR, kCtrCreated, kCtrOverflow, kCtrPushed, kCtrN };

template <class P>
__host__ __device__ inline Lds lds_layout(const ElecArgs& a) {
  auto al = [](uint32_t x) { return (x + 15u) & ~15u; };
  Lds L;
  L.tab = 0;
  L.bins = al(L.tab + (uint32_t)a.tab_max * (uint32_t)sizeof(P));
  L.q = al(L.bins + (uint32_t)a.nn_max * 8u);
  L.eedf = al(L.q + (uint32_t)kQueue * (uint32_t)sizeof(QEntry<P>));
  L.ctr = al(L.eedf + (uint32_t)a.nb1_max * 4u);
  L.pre = al(L.ctr + (uint32_t)kCtrN * 4u);
  L.wsum = al(L.pre + (uint32_t)(a.D + 1) * 4u);
  L.total = al(L.wsum + 16u * 4u);
  const uint32_t fluid = 4u * (uint32_t)a.fluid_nn * 8u;  // a, b, c/c', r/d' of Eq (2.3)
  if (fluid > L.total) L.total = al(fluid);
  return L;
}

template <class P>
__device__ __forceinline__ void sphere(Stream& s, P& nx, P& ny, P& nz) {
  for (int t = 0; t < kSphereTries; ++t) {
    const P a = (P)2 * Uni<P>::get(s) - (P)1;
    const P b = (P)2 * Uni<P>::get(s) - (P)1;
    const P q = a * a + b * b;
    if (q < (P)1) {
      const P r = (P)2 * sqrt((P)1 - q);
      nx = a * r;
      ny = b * r;
      nz = (P)1 - (P)2 * q;
      return;
    }
  }
  nx = (P)0;
  ny = (P)0;
  nz = (P)1;
}

template <class P>
__device__ __forceinline__ int eedf_bin(P vx, P vy, P vz, const Disch<P>& d) {
  const P en = d.KE * ((vx * vx + vy * vy) + vz * vz);
  const P x = en * d.keedf;
  return (x < (P)d.nbins) ? (int)x : d.nbins;
}

// Scattering of one queued collision (elastic / excitation / ionization).
template <class P>
__device__ void handle(const Disch<P>& d, QEntry<P>& e, uint32_t lc, uint32_t step, bool sample,
                       int64_t* bins, uint32_t* eedf, uint32_t* ctr) {
  Stream s(d.seed, kTagElectron, e.id, step);
  for (int w = 0; w < Uni<P>::kWords; ++w) (void)s.word();  // R used by the null test
  const P vx = e.vx, vy = e.vy, vz = e.vz;
  const P v2 = (vx * vx + vy * vy) + vz * vz;
  const P en = d.KE * v2;
  const int kind = d.kind[e.ch];
  P nx, ny, nz;
  if (kind == 0) {
    sphere<P>(s, nx, ny, nz);
    const P vm = sqrt(v2);
    const P cosx = ((vx * nx + vy * ny) + vz * nz) / vm;
    const P fac = (P)1 - d.delta * ((P)1 - cosx);
    const P vn = sqrt(v2 * fac);
    e.vx = vn * nx;
    e.vy = vn * ny;
    e.vz = vn * nz;
  } else if (kind == 1) {
    sphere<P>(s, nx, ny, nz);
    P er = en - d.thr[e.ch];
    if (er < (P)0) er = (P)0;
    const P vn = sqrt(er * d.invKE);
    e.vx = vn * nx;
    e.vy = vn * ny;
    e.vz = vn * nz;
  } else {
    sphere<P>(s, nx, ny, nz);
    const P us = Uni<P>::get(s);
    P er = en - d.thr[e.ch];
    if (er < (P)0) er = (P)0;
    const P es = us * er;
    const P ep = er - es;
    const P vn = sqrt(ep * d.invKE);
    e.vx = vn * nx;
    e.vy = vn * ny;
    e.vz = vn * nz;
    P mx, my, mz;
    sphere<P>(s, mx, my, mz);
    const P vc = sqrt(es * d.invKE);
    const P cvx = vc * mx, cvy = vc * my, cvz = vc * mz;
    const uint32_t slot = lc * (uint32_t)kTile + (uint32_t)e.kid;
    d.kc[slot] = e.c;
    d.koff[slot] = e.off;
    d.kvx[slot] = cvx;
    d.kvy[slot] = cvy;
    d.kvz[slot] = cvz;
    const int64_t W1 = cic_w1<P>(e.off);
    const int64_t W0 = ((int64_t)1 << 32) - W1;
    atomicAdd(reinterpret_cast<unsigned long long*>(&bins[e.c]), (unsigned long long)W0);
    atomicAdd(reinterpret_cast<unsigned long long*>(&bins[e.c + 1]), (unsigned long long)W1);
    atomic_add_i64(&d.ion_src[e.c], W0);
    atomic_add_i64(&d.ion_src[e.c + 1], W1);
    if (sample) atomicAdd(&eedf[eedf_bin<P>(cvx, cvy, cvz, d)], 1u);
    atomicAdd(&ctr[kCtrCreated], 1u);
  }
  atomicAdd(&ctr[e.ch], 1u);
}

// The four consecutive slots a thread owns in a chunk.
template <class P>
struct Slots {
  int32_t c[4];
  P off[4], vx[4], vy[4], vz[4];
  uint32_t id[4];
};

template <class P>
__device__ __forceinline__ void load_slots(const Disch<P>& d, int buf, uint32_t lc, Slots<P>& s) {
  const uint32_t i0 = lc * (uint32_t)kTile + (uint32_t)threadIdx.x * (uint32_t)kPerThread;
  ld4(d.cell[buf] + i0, s.c);
  ld4(d.off[buf] + i0, s.off);
  ld4(d.vx[buf] + i0, s.vx);
  ld4(d.vy[buf] + i0, s.vy);
  ld4(d.vz[buf] + i0, s.vz);
  ld4(d.id[buf] + i0, s.id);
}

// One chunk of kTile consecutive particle slots.
template <class P>
__device__ void chunk(const Disch<P>& d, uint32_t lc, uint32_t step, uint32_t n_main, int buf,
                      bool sample, const P* tab, int64_t* bins, QEntry<P>* q, uint32_t* eedf,
                      uint32_t* ctr, uint32_t* wsum, Slots<P>& in) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const uint32_t i0 = lc * (uint32_t)kTile + (uint32_t)tid * (uint32_t)kPerThread;
  int32_t (&c)[4] = in.c;
  P (&off)[4] = in.off;
  P (&vx)[4] = in.vx;
  P (&vy)[4] = in.vy;
  P (&vz)[4] = in.vz;
  uint32_t (&id)[4] = in.id;
  const P* Ep = d.Ep;
  const int K = d.K;
  int ch[4];
  bool alive[4];
  uint32_t n_absl = 0, n_absr = 0, n_ovf = 0, n_push = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ch[j] = -1;
    alive[j] = (i0 + (uint32_t)j < n_main) && (c[j] >= 0);
    n_push += (uint32_t)__popcll(__ballot(alive[j]));
    if (alive[j]) {
      // leapfrog push, linear gather of E' = (-e/m_e) dt E
      const P e0 = Ep[c[j]];
      const P e1 = Ep[c[j] + 1];
      const P t1 = e1 - e0;
      const P g = e0 + off[j] * t1;
      vz[j] = vz[j] + g;
      const P s = off[j] + vz[j] * d.kdz;
      const P f = floor(s);
      if (!(f >= (P)(-c[j]))) {
        c[j] = -1;
        alive[j] = false;
        n_absl += 1;
      } else if (f >= (P)(d.nc - c[j])) {
        c[j] = -1;
        alive[j] = false;
        n_absr += 1;
      } else {
        int32_t cn = c[j] + (int32_t)f;
        P on = s - f;
        if (on == (P)1) {
          cn = cn + 1;
          on = (P)0;
        }
        c[j] = cn;
        off[j] = on;
      }
    }
    if (alive[j]) {
      // null-collision test with one Philox block of stream (tag 0, id, step)
      uint32_t w0, w1, w2, w3;
      philox4x32_10(id[j], step, 0u, kTagElectron, (uint32_t)d.seed, (uint32_t)(d.seed >> 32), w0,
                    w1, w2, w3);
      P u0;
      if constexpr (sizeof(P) == 4)
        u0 = (P)u01_f32(w0);
      else
        u0 = (P)u01_f64(w0, w1);
      if (u0 < d.Pmax) {
        const P v2 = (vx[j] * vx[j] + vy[j] * vy[j]) + vz[j] * vz[j];
        const P en = d.KE * v2;
        const P sx = en * d.inv_dE;
        int i;
        P t;
        if (sx >= (P)(d.ne - 1)) {
          i = d.ne - 2;
          t = (P)1;
          n_ovf += 1;
        } else {
          i = (int)sx;
          t = sx - (P)i;
        }
        const P* ra = tab + i * K;
        for (int k = 0; k < K; ++k) {
          const P pa = ra[k];
          const P pb = ra[K + k];
          const P pk = pa + t * (pb - pa);
          if (u0 < pk) {
            ch[j] = k;
            break;
          }
        }
      }
    }
  }
  // event counters (rare): one LDS atomic per thread with events
  if (n_absl) atomicAdd(&ctr[kCtrAbsL], n_absl);
  if (n_absr) atomicAdd(&ctr[kCtrAbsR], n_absr);
  if (n_ovf) atomicAdd(&ctr[kCtrOverflow], n_ovf);
  if (lane == 0 && n_push) atomicAdd(&ctr[kCtrPushed], n_push);

  // collision queue positions and child slots, in particle order
  bool col[4], ion[4];
  const uint64_t lt = lanemask_lt();
  uint32_t pc = 0, pi = 0, tc = 0, ti = 0, ncol = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    col[j] = ch[j] >= 0;
    ion[j] = col[j] && d.kind[ch[j]] == 2;
    ncol += col[j] ? 1u : 0u;
    const uint64_t mc = __ballot(col[j]);
    const uint64_t mi = __ballot(ion[j]);
    pc += (uint32_t)__popcll(mc & lt);
    pi += (uint32_t)__popcll(mi & lt);
    tc += (uint32_t)__popcll(mc);
    ti += (uint32_t)__popcll(mi);
  }
  if (lane == 0) wsum[wv] = tc | (ti << 16);
  __syncthreads();
  uint32_t TC = 0, TI = 0, qpos = pc, kpos = pi;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t v = wsum[w];
    const uint32_t a = v & 0xFFFFu, b = v >> 16;
    if (w < wv) {
      qpos += a;
      kpos += b;
    }
    TC += a;
    TI += b;
  }
  for (uint32_t r0 = 0; r0 < TC; r0 += (uint32_t)kQueue) {
    uint32_t qi = qpos, ki = kpos;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (col[j]) {
        if (qi >= r0 && qi < r0 + (uint32_t)kQueue) {
          QEntry<P>& e = q[qi - r0];
          e.vx = vx[j];
          e.vy = vy[j];
          e.vz = vz[j];
          e.off = off[j];
          e.id = id[j];
          e.c = c[j];
          e.ch = ch[j];
          e.kid = ion[j] ? (int32_t)ki : -1;
        }
        qi += 1;
        ki += ion[j] ? 1u : 0u;
      }
    }
    __syncthreads();
    const uint32_t nr = min((uint32_t)kQueue, TC - r0);
    for (uint32_t e = (uint32_t)tid; e < nr; e += (uint32_t)kThreads)
      handle<P>(d, q[e], lc, step, sample, bins, eedf, ctr);
    __syncthreads();
    qi = qpos;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (col[j]) {
        if (qi >= r0 && qi < r0 + (uint32_t)kQueue) {
          const QEntry<P>& e = q[qi - r0];
          vx[j] = e.vx;
          vy[j] = e.vy;
          vz[j] = e.vz;
        }
        qi += 1;
      }
    }
    __syncthreads();
  }
  // deposit at x^{n+1} (consecutive equal cells merged in registers), EEDF
  int rc = -1;
  uint64_t a0 = 0, a1 = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!alive[j]) continue;
    if (sample) atomicAdd(&eedf[eedf_bin<P>(vx[j], vy[j], vz[j], d)], 1u);
    const int64_t W1 = cic_w1<P>(off[j]);
    const int64_t W0 = ((int64_t)1 << 32) - W1;
    if (c[j] == rc) {
      a0 += (uint64_t)W0;
      a1 += (uint64_t)W1;
    } else {
      if (rc >= 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&bins[rc]), (unsigned long long)a0);
        atomicAdd(reinterpret_cast<unsigned long long*>(&bins[rc + 1]), (unsigned long long)a1);
      }
      rc = c[j];
      a0 = (uint64_t)W0;
      a1 = (uint64_t)W1;
    }
  }
  if (rc >= 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&bins[rc]), (unsigned long long)a0);
    atomicAdd(reinterpret_cast<unsigned long long*>(&bins[rc + 1]), (unsigned long long)a1);
  }
  // write back; vx, vy change only in collisions
  st4(d.cell[buf] + i0, c);
  st4(d.off[buf] + i0, off);
  st4(d.vz[buf] + i0, vz);
  if (ncol) {
    st4(d.vx[buf] + i0, vx);
    st4(d.vy[buf] + i0, vy);
  }
  if (tid == 0) d.chunk_kids[lc] = TI;
}

template <class P>
__device__ void segment(const Disch<P>& d, uint32_t lc0, uint32_t lc1, unsigned char* smem,
                        const Lds& L) {
  const int tid = threadIdx.x;
  P* tab = reinterpret_cast<P*>(smem + L.tab);
  int64_t* bins = reinterpret_cast<int64_t*>(smem + L.bins);
  QEntry<P>* q = reinterpret_cast<QEntry<P>*>(smem + L.q);
  uint32_t* eedf = reinterpret_cast<uint32_t*>(smem + L.eedf);
  uint32_t* ctr = reinterpret_cast<uint32_t*>(smem + L.ctr);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + L.wsum);
  const int tabN = d.ne * d.K;
  for (int i = tid; i < tabN; i += kThreads) tab[i] = d.tab[i];
  for (int i = tid; i < d.nn; i += kThreads) bins[i] = 0;
  for (int i = tid; i <= d.nbins; i += kThreads) eedf[i] = 0;
  if (tid < kCtrN) ctr[tid] = 0;
  State* st = d.st;
  const uint32_t step = (uint32_t)st->step;
  const bool sample = ((st->step + 1) % d.eedf_every) == 0;
  const uint32_t n_main = st->n_main;
  const int buf = st->buf;
  int64_t* cnt = d.cnt[st->cbuf ^ 1];
  __syncthreads();
  // the next chunk's slots are loaded before the current one is processed
  Slots<P> cur, nxt;
  load_slots<P>(d, buf, lc0, cur);
  for (uint32_t lc = lc0; lc < lc1; ++lc) {
    if (lc + 1 < lc1) load_slots<P>(d, buf, lc + 1, nxt);
    chunk<P>(d, lc, step, n_main, buf, sample, tab, bins, q, eedf, ctr, wsum, cur);
    cur = nxt;
  }
  __syncthreads();
  for (int i = tid; i < d.nn; i += kThreads) {
    const int64_t v = bins[i];
    if (v) atomic_add_i64(&cnt[i], v);
  }
  if (sample)
    for (int i = tid; i <= d.nbins; i += kThreads)
      if (eedf[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&d.eedf[i]),
                             (unsigned long long)eedf[i]);
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
  __syncthreads();
}

// ---- ion fluid -----------------------------------------------------------

__device__ __forceinline__ double dmin0(double e) { return (0.0 < e) ? 0.0 : e; }  // min(e, 0)
__device__ __forceinline__ double dmax0(double e) { return (e < 0.0) ? 0.0 : e; }  // max(e, 0)

template <class P>
__device__ __forceinline__ double ion_temperature(const Disch<P>& d, double mu, double E) {
  const double x = mu * fabs(E);
  return d.TN + d.kappa * (x * x);
}

// Drift-diffusion, explicit: Eq (2.5) with Eqs (2.7)-(2.8) and central
// differences, field-switched drift flux at the walls, then Eq (2.4) with
// half cells at the walls.
template <class P>
__device__ void fluid_dd(const Disch<P>& d) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn;
  double* ni = d.ni;
  double* gam = d.gam;
  const double* E = d.E;
  double* n0 = d.scratch;
  const double mu = d.mu;
  for (int j = tid; j < nn; j += kThreads) n0[j] = ni[j];
  __syncthreads();
  for (int j = tid; j < nn; j += kThreads) {
    double g;
    if (j == 0) {
      g = (mu * n0[0]) * dmin0(E[0]);
    } else if (j == nc) {
      g = (mu * n0[nc]) * dmax0(E[nc]);
    } else {
      const double T = ion_temperature(d, mu, E[j]);
      const double Dc = (mu * T) / kECharge;
      g = (mu * n0[j]) * E[j] - (Dc * (n0[j + 1] - n0[j - 1])) * d.inv_2dz;
    }
    gam[j] = g;
  }
  __syncthreads();
  for (int j = tid; j < nn; j += kThreads) {
    double v;
    if (j == 0)
      v = n0[0] - d.dt_dz * (gam[1] - gam[0]);
    else if (j == nc)
      v = n0[nc] - d.dt_dz * (gam[nc] - gam[nc - 1]);
    else
      v = n0[j] - d.dt_2dz * (gam[j + 1] - gam[j - 1]);
    ni[j] = v;
  }
  if (tid == 0) {
    d.st->wall[0] = gam[0];
    d.st->wall[1] = gam[nc];
  }
}

// Full fluid: Eq (2.3) for Gamma^{n+1/2} with lagged nu and semi-implicit
// advection (tridiagonal; Thomas method, one reciprocal per row), drift wall
// fluxes with mu = e/(M nu) (Eq 2.6), then Eq (2.4).
template <class P>
__device__ void fluid_full(const Disch<P>& d, double* lds) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn, m = nc - 1;
  double* ni = d.ni;
  double* gam = d.gam;
  const double* E = d.E;
  double* n0 = d.scratch;
  double* g0 = n0 + nn;
  double* u = g0 + nn;
  double* T = u + nn;
  const double nu = d.nu, mu = d.mu_full;
  for (int j = tid; j < nn; j += kThreads) {
    const double nj = ni[j], gj = gam[j];
    n0[j] = nj;
    g0[j] = gj;
    u[j] = (nj > d.nfloor) ? gj / nj : 0.0;
    T[j] = ion_temperature(d, mu, E[j]);
  }
  __syncthreads();
  // tridiagonal coefficients in LDS so that the serial elimination reads
  // its operands at LDS latency; c and r are overwritten by c' and d'
  double* La = lds;
  double* Lb = La + nn;
  double* Lc = Lb + nn;
  double* Lr = Lc + nn;
  for (int j = 1 + tid; j <= m; j += kThreads) {
    const int k = j - 1;
    La[k] = -d.dt_2dz * u[j - 1];
    Lb[k] = 1.0 + nu * d.hdt;
    Lc[k] = d.dt_2dz * u[j + 1];
    Lr[k] = (g0[j] * (1.0 - nu * d.hdt) + (d.e_M_dt * n0[j]) * E[j]) -
            d.dt_2dzM * (n0[j + 1] * T[j + 1] - n0[j - 1] * T[j - 1]);
  }
  __syncthreads();
  const double gl = (mu * n0[0]) * dmin0(E[0]);
  const double gr = (mu * n0[nc]) * dmax0(E[nc]);
  if (tid == 0) {
    Lr[0] = Lr[0] - La[0] * gl;
    Lr[m - 1] = Lr[m - 1] - Lc[m - 1] * gr;
    double rr = 1.0 / Lb[0];
    double cpp = Lc[0] * rr;
    double dpp = Lr[0] * rr;
    Lc[0] = cpp;
    Lr[0] = dpp;
    // operands of kB rows are loaded ahead of their dependent eliminations
    constexpr int kB = 8;
    int k = 1;
    for (; k + kB - 1 < m; k += kB) {
      double ak[kB], bk[kB], ck[kB], rk[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        ak[q] = La[k + q];
        bk[q] = Lb[k + q];
        ck[q] = Lc[k + q];
        rk[q] = Lr[k + q];
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const double den = bk[q] - ak[q] * cpp;
        const double num = rk[q] - ak[q] * dpp;
        rr = 1.0 / den;
        cpp = ck[q] * rr;
        dpp = num * rr;
        Lc[k + q] = cpp;
        Lr[k + q] = dpp;
      }
    }
    for (; k < m; ++k) {
      const double ak = La[k];
      const double den = Lb[k] - ak * cpp;
      const double num = Lr[k] - ak * dpp;
      rr = 1.0 / den;
      cpp = Lc[k] * rr;
      dpp = num * rr;
      Lc[k] = cpp;
      Lr[k] = dpp;
    }
    double x = dpp;
    La[m - 1] = x;
    k = m - 2;
    for (; k - kB + 1 >= 0; k -= kB) {
      double ck[kB], rk[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        ck[q] = Lc[k - q];
        rk[q] = Lr[k - q];
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        x = rk[q] - ck[q] * x;
        La[k - q] = x;
      }
    }
    for (; k >= 0; --k) {
      x = Lr[k] - Lc[k] * x;
      La[k] = x;
    }
    d.st->wall[0] = gl;
    d.st->wall[1] = gr;
  }
  __syncthreads();
  for (int j = tid; j < nn; j += kThreads) gam[j] = (j == 0) ? gl : (j == nc) ? gr : La[j - 1];
  __syncthreads();
  for (int j = tid; j < nn; j += kThreads) {
    double v;
    if (j == 0)
      v = n0[0] - d.dt_dz * (gam[1] - gam[0]);
    else if (j == nc)
      v = n0[nc] - d.dt_dz * (gam[nc] - gam[nc - 1]);
    else
      v = n0[j] - d.dt_2dz * (gam[j + 1] - gam[j - 1]);
    ni[j] = v;
  }
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_electron(const Disch<P>* __restrict__ ds, ElecArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int D = a.D;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < D) {
    const Disch<P>& d = ds[blockIdx.x];
    if (d.st->steps_left > 0) {
      if (d.ion_model == 0)
        fluid_dd<P>(d);
      else
        fluid_full<P>(d, reinterpret_cast<double*>(smem));
    }
    return;
  }
  const Lds L = lds_layout<P>(a);
  uint32_t* pre = reinterpret_cast<uint32_t*>(smem + L.pre);
  for (int i = tid; i < D; i += kThreads) {
    const State* st = ds[i].st;
    pre[i + 1] = (st->steps_left > 0) ? (st->n_main + (uint32_t)kTile - 1u) / (uint32_t)kTile : 0u;
  }
  if (tid == 0) pre[0] = 0;
  __syncthreads();
  if (tid == 0)
    for (int i = 0; i < D; ++i) pre[i + 1] += pre[i];
  __syncthreads();
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
    segment<P>(ds[di], g0 - pre[di], end - pre[di], smem, L);
    g0 = end;
    ++di;
  }
}

}  // namespace

template <class P>
size_t electron_lds_bytes(int D, int tab_max, int nn_max, int nb1_max, int fluid_nn) {
  ElecArgs a{D, tab_max, nn_max, nb1_max, fluid_nn};
  return lds_layout<P>(a).total;
}

template <class P>
hipError_t launch_electron_impl(const Disch<P>* d_dev, int D, int grid, int tab_max, int nn_max,
                                int nb1_max, int fluid_nn, hipStream_t s) {
  ElecArgs a{D, tab_max, nn_max, nb1_max, fluid_nn};
  const size_t lds = lds_layout<P>(a).total;
  hipLaunchKernelGGL(k_electron<P>, dim3(grid), dim3(kThreads), lds, s, d_dev, a);
  return hipGetLastError();
}

template <class P>
int electron_occupancy(int tab_max, int nn_max, int nb1_max, int fluid_nn, int D) {
  int nb = 0;
  const size_t lds = electron_lds_bytes<P>(D, tab_max, nn_max, nb1_max, fluid_nn);
  if (hipFuncSetAttribute((const void*)k_electron<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_electron<P>, kThreads, lds) != hipSuccess)
    return 0;
  return nb;
}

template size_t electron_lds_bytes<float>(int, int, int, int, int);
template size_t electron_lds_bytes<double>(int, int, int, int, int);
template hipError_t launch_electron_impl<float>(const Disch<float>*, int, int, int, int, int, int,
                                                hipStream_t);
template hipError_t launch_electron_impl<double>(const Disch<double>*, int, int, int, int, int,
                                                 int, hipStream_t);
template int electron_occupancy<float>(int, int, int, int, int);
template int electron_occupancy<double>(int, int, int, int, int);

}  // namespace hd
