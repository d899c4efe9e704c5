// End of a time step and field of the next one, one workgroup per discharge:
// offsets of the staged ionization children (exclusive scan over chunks),
// ion-induced secondary emission (Sec. II.D), ion sources of the step
// (G^n in Eq 2.4), run averages, append bookkeeping, then the Poisson solve
// of the coupling (Sec. II.D) for the next step.  A second kernel appends the
// children and secondaries to the particle arrays in canonical order.
#include "hd_device.h"

namespace hd {

namespace {

constexpr double kECharge = 1.602176634e-19;
constexpr int kWaves = kFinThreads / 64;

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *total.  sh must hold kWaves + 1 words.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t s = sh[w];
    if (w < wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Secondary electrons of one wall (side 0: z = 0, side 1: z = L) for ion
// flux F: int(X) + Bernoulli(X - int(X)) superparticles, X = gamma F dt / w;
// cosine law, uniform azimuth, partial first flight.  Written to the
// emission buffer and deposited.
template <class P>
__device__ void emit(const Disch<P>& d, int side, double F, uint32_t step, int64_t* cn,
                     uint32_t* n_out, uint64_t* emitted, uint64_t* absorbed, uint64_t* clamped) {
  Stream s(d.seed, kTagEmission, (uint32_t)side, step);
  const double X = ((d.gamma_see * F) * d.dt) / d.w;
  const double fl = floor(X);
  const double ub = Uni<double>::get(s);
  int64_t ns = (int64_t)fl + ((ub < X - fl) ? 1 : 0);
  if (ns > kSeeMax) {
    *clamped += (uint64_t)(ns - kSeeMax);
    ns = kSeeMax;
  }
  uint32_t m = 0;
  const double v = d.see_v;
  for (int64_t k = 0; k < ns; ++k) {
    const double uc = Uni<double>::get(s);
    const double cth = sqrt(uc);
    const double sth = sqrt(1.0 - uc);
    double a = 1.0, b = 0.0, qq = 1.0;
    for (int t = 0; t < kSphereTries; ++t) {
      const double ta = 2.0 * Uni<double>::get(s) - 1.0;
      const double tb = 2.0 * Uni<double>::get(s) - 1.0;
      const double tq = ta * ta + tb * tb;
      if (tq < 1.0 && tq > 0.0) {
        a = ta;
        b = tb;
        qq = tq;
        break;
      }
    }
    const double cph = (a * a - b * b) / qq;
    const double sph = (2.0 * a * b) / qq;
    const double vz = v * cth;
    const double vp = v * sth;
    const double upp = Uni<double>::get(s);
    const double flight = (vz * d.dt) * upp;
    const double z = side == 0 ? flight : d.L - flight;
    const double sc = z / d.dz;
    const double fc = floor(sc);
    *emitted += 1;
    if (!(fc > -2147483648.0 && fc < 2147483647.0)) {  // outside any cell index
      *absorbed += 1;
      continue;
    }
    int32_t c = (int32_t)fc;
    P off = (P)(sc - fc);
    if (off == (P)1) {
      c = c + 1;
      off = (P)0;
    }
    if (c < 0 || c >= d.nc) {
      *absorbed += 1;
      continue;
    }
    const int idx = side * kSeeMax + (int)m;
    d.sc[idx] = c;
    d.soff[idx] = off;
    d.svx[idx] = (P)(vp * cph);
    d.svy[idx] = (P)(vp * sph);
    d.svz[idx] = (P)(side == 0 ? vz : -vz);
    const int64_t W1 = cic_w1<P>(off);
    const int64_t W0 = ((int64_t)1 << 32) - W1;
    atomic_add_i64(&cn[c], W0);
    atomic_add_i64(&cn[c + 1], W1);
    m += 1;
  }
  *n_out = m;
}

template <class P>
__device__ __forceinline__ double scale_of(const Disch<P>& d, int j) {
  return (j == 0 || j == d.nc) ? d.scale_wall : d.scale_in;
}

// Poisson's equation with phi_0 = V(t), phi_N = 0 (Thomas elimination with
// the constant inverse pivots, one fused multiply-add per sweep step), E from
// centred differences inside and Gauss's law over the wall half cells, and
// E' = (-e/m_e) dt E rounded to the particle precision.
// The interior system (-1, 2, -1) is solved by the partitioned elimination;
// lds holds 4 * nn + 7 * kTriRed doubles.
template <class P>
__device__ void field(const Disch<P>& d, const int64_t* cn, double V, double* lds) {
  const int tid = threadIdx.x, nc = d.nc, nn = d.nn, m = nc - 1;
  double* rho = d.scratch;
  double* A = lds;        // rows r = j - 1 of the interior unknowns j = 1 .. m
  double* B = A + nn;     // receives phi_j at r = j - 1
  double* Cc = B + nn;
  double* Dd = Cc + nn;
  double* red = Dd + nn;
  for (int j = tid; j < nn; j += kFinThreads) {
    const double ne = (double)load_dev(&cn[j]) * scale_of(d, j);
    const double r = kECharge * (d.ni[j] - ne);
    rho[j] = r;
    if (j >= 1 && j <= m) {
      double dj = d.kp * r;
      if (j == 1) dj = dj + V;
      if (j == m) dj = dj + 0.0;
      A[j - 1] = -1.0;
      B[j - 1] = 2.0;
      Cc[j - 1] = -1.0;
      Dd[j - 1] = dj;
    }
  }
  solve_tridiag_block(m, A, B, Cc, Dd, red);
  auto phi = [&](int j) { return j == 0 ? V : (j == nc ? 0.0 : B[j - 1]); };
  for (int j = tid; j < nn; j += kFinThreads) {
    double e;
    if (j == 0)
      e = (phi(0) - phi(1)) * d.inv_dz - rho[0] * d.hdz_eps;
    else if (j == nc)
      e = (phi(nc - 1) - phi(nc)) * d.inv_dz + rho[nc] * d.hdz_eps;
    else
      e = (phi(j - 1) - phi(j + 1)) * d.inv_2dz;
    d.phi[j] = phi(j);
    d.E[j] = e;
    d.Ep[j] = (P)(d.qm_dt * e);
  }
}

template <class P>
__global__ __launch_bounds__(kFinThreads) void k_finalize(const Disch<P>* __restrict__ ds,
                                                          int field_only) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Disch<P>& d = ds[blockIdx.x];
  State* st = d.st;
  const int tid = threadIdx.x;
  __shared__ uint32_t sh[kWaves + 1];
  __shared__ uint32_t sh_see[2];
  if (!field_only) {
    if (st->steps_left <= 0) return;
    const int cb = st->cbuf ^ 1;  // deposit of this step
    int64_t* cn = d.cnt[cb];
    const uint32_t n_main = st->n_main;
    // sub-chunks the electron kernel wrote child counts for (whole chunks)
    const uint32_t nch = (n_main + (uint32_t)kTile - 1u) / (uint32_t)kTile * (uint32_t)(kTile / kSub);
    // offsets of the staged children: tiles of kFinThreads x 16 sub-chunks,
    // each thread reading and writing 16 consecutive counts as four 16-byte
    // vectors (nch is a multiple of 4)
    uint32_t n_kids = 0;
    for (uint32_t t0 = 0; t0 < nch; t0 += (uint32_t)kFinThreads * 16u) {
      const uint32_t k0 = t0 + (uint32_t)tid * 16u;
      uint4 v[4];
      uint32_t loc = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = make_uint4(0u, 0u, 0u, 0u);
        if (k0 + 4u * (uint32_t)q < nch)
          v[q] = *reinterpret_cast<const uint4*>(d.chunk_kids + k0 + 4u * (uint32_t)q);
        loc += (v[q].x + v[q].y) + (v[q].z + v[q].w);
      }
      uint32_t tot;
      uint32_t run = n_kids + block_scan(loc, sh, &tot);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint4 b;
        b.x = run;
        b.y = b.x + v[q].x;
        b.z = b.y + v[q].y;
        b.w = b.z + v[q].z;
        run = b.w + v[q].w;
        if (k0 + 4u * (uint32_t)q < nch)
          *reinterpret_cast<uint4*>(d.chunk_base + k0 + 4u * (uint32_t)q) = b;
      }
      n_kids += tot;
    }
    // emission from the wall fluxes of this step's fluid update
    if (tid < 2) {
      const double g = st->wall[tid];
      const double F = tid == 0 ? ((-g < 0.0) ? 0.0 : -g) : ((g < 0.0) ? 0.0 : g);
      uint64_t em = 0, ab = 0, cl = 0;
      uint32_t n = 0;
      emit<P>(d, tid, F, (uint32_t)st->step, cn, &n, &em, &ab, &cl);
      sh_see[tid] = n;
      if (em) atomicAdd(reinterpret_cast<unsigned long long*>(&st->emitted[tid]), (unsigned long long)em);
      if (ab) atomicAdd(reinterpret_cast<unsigned long long*>(&st->absorbed[tid]), (unsigned long long)ab);
      if (cl) atomicAdd(reinterpret_cast<unsigned long long*>(&st->see_clamped), (unsigned long long)cl);
    }
    __syncthreads();
    // ion sources of the step, run averages
    for (int j = tid; j < d.nn; j += kFinThreads) {
      const double nj = d.ni[j] + (double)d.ion_src[j] * scale_of(d, j);
      d.ni[j] = nj;
      d.ion_src[j] = 0;
      d.acc_cnt[j] += (uint64_t)load_dev(&cn[j]);
      d.acc_ni[j] += nj;
    }
    if (tid == 0) {
      const uint32_t ns0 = sh_see[0], ns1 = sh_see[1];
      const uint64_t n_app = (uint64_t)n_kids + ns0 + ns1;
      st->n_chunks = nch;
      st->n_kids = n_kids;
      st->n_see[0] = ns0;
      st->n_see[1] = ns1;
      if ((uint64_t)n_main + n_app > (uint64_t)d.capacity) {
        st->error = -4;  // capacity exceeded
        st->append_pending = 0;
        st->steps_left = 0;
      } else {
        st->append_base = n_main;
        st->id_base = st->next_id;
        st->n_main = n_main + (uint32_t)n_app;
        st->next_id = st->next_id + (uint32_t)n_app;
        st->append_pending = n_app > 0 ? 1 : 0;
        st->steps_left = st->steps_left - 1;
      }
      st->step = st->step + 1;
      st->n_acc = st->n_acc + 1;
      st->sort_due = (st->step % d.sort_every) == 0 ? 1 : 0;
      st->cbuf = cb;
    }
    __syncthreads();
  }
  // field of the (new) current step
  const int cur = st->cbuf;
  const int64_t step = st->step;
  const double V = (step < d.volt_len) ? d.volt[step] : 0.0;
  field<P>(d, d.cnt[cur], V, reinterpret_cast<double*>(smem));
  // clear the deposit target of the next step
  int64_t* nxt = d.cnt[cur ^ 1];
  for (int j = tid; j < d.nn; j += kFinThreads) nxt[j] = 0;
}

// Append this step's children (in sub-chunk order, i.e. parent order), then the
// left and right secondaries, with consecutive ids.
template <class P>
__global__ __launch_bounds__(kThreads) void k_append(const Disch<P>* __restrict__ ds, int D) {
  const int tid = threadIdx.x;
  for (int di = 0; di < D; ++di) {
    const Disch<P>& d = ds[di];
    const State* st = d.st;
    if (!st->append_pending) continue;
    const int buf = st->buf;
    const uint32_t nch = st->n_chunks, base = st->append_base, idb = st->id_base;
    for (uint32_t lc = blockIdx.x; lc < nch; lc += gridDim.x) {
      const uint32_t k = d.chunk_kids[lc];
      if (k == 0) continue;
      const uint32_t cb = d.chunk_base[lc];
      for (uint32_t t = (uint32_t)tid; t < k; t += (uint32_t)kThreads) {
        const uint32_t src = lc * (uint32_t)kSub + t;
        const uint32_t dst = base + cb + t;
        d.cell[buf][dst] = d.kc[src];
        d.off[buf][dst] = d.koff[src];
        d.vx[buf][dst] = d.kvx[src];
        d.vy[buf][dst] = d.kvy[src];
        d.vz[buf][dst] = d.kvz[src];
        d.id[buf][dst] = idb + cb + t;
      }
    }
    if ((int)blockIdx.x == di % (int)gridDim.x) {
      const uint32_t nk = st->n_kids, n0 = st->n_see[0], n1 = st->n_see[1];
      for (uint32_t t = (uint32_t)tid; t < n0 + n1; t += (uint32_t)kThreads) {
        const uint32_t src = t < n0 ? t : (uint32_t)kSeeMax + (t - n0);
        const uint32_t dst = base + nk + t;
        d.cell[buf][dst] = d.sc[src];
        d.off[buf][dst] = d.soff[src];
        d.vx[buf][dst] = d.svx[src];
        d.vy[buf][dst] = d.svy[src];
        d.vz[buf][dst] = d.svz[src];
        d.id[buf][dst] = idb + nk + t;
      }
    }
  }
}

// Arms every discharge of a batch for n more steps (discharges in an error
// state stay idle).
template <class P>
__global__ void k_set_steps(const Disch<P>* __restrict__ ds, int D, int64_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  State* st = ds[i].st;
  st->steps_left = st->error ? 0 : n;
}

template <class P>
__global__ void k_diag(int64_t n, const P* a, const P* b, P* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const P x = a[i], y = b[i];
  out[4 * i + 0] = sqrt(x);
  out[4 * i + 1] = x / y;
  out[4 * i + 2] = rint(x * (P)4294967296.0);
  out[4 * i + 3] = floor(x);
}

}  // namespace

template <class P>
hipError_t launch_finalize(const Disch<P>* d_dev, int D, int field_only, int nn_max,
                           hipStream_t s) {
  const size_t lds = ((size_t)4 * (size_t)nn_max + 7u * kTriRed) * 8u;
  hipLaunchKernelGGL(k_finalize<P>, dim3(D), dim3(kFinThreads), lds, s, d_dev, field_only);
  return hipGetLastError();
}

template <class P>
hipError_t finalize_set_lds(int nn_max) {
  return hipFuncSetAttribute((const void*)k_finalize<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (4 * nn_max + 7 * kTriRed) * 8);
}

template hipError_t finalize_set_lds<float>(int);
template hipError_t finalize_set_lds<double>(int);

template <class P>
hipError_t launch_append(const Disch<P>* d_dev, int D, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_append<P>, dim3(grid), dim3(kThreads), 0, s, d_dev, D);
  return hipGetLastError();
}

template <class P>
hipError_t launch_diag(int64_t n, const P* a, const P* b, P* out, hipStream_t s) {
  const int bs = 256;
  const int64_t g = (n + bs - 1) / bs;
  if (g > 0) hipLaunchKernelGGL(k_diag<P>, dim3((unsigned)g), dim3(bs), 0, s, n, a, b, out);
  return hipGetLastError();
}

template <class P>
hipError_t launch_set_steps(const Disch<P>* d_dev, int D, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_steps<P>, dim3((D + 63) / 64), dim3(64), 0, s, d_dev, D, n);
  return hipGetLastError();
}

template hipError_t launch_set_steps<float>(const Disch<float>*, int, int64_t, hipStream_t);
template hipError_t launch_set_steps<double>(const Disch<double>*, int, int64_t, hipStream_t);
template hipError_t launch_finalize<float>(const Disch<float>*, int, int, int, hipStream_t);
template hipError_t launch_finalize<double>(const Disch<double>*, int, int, int, hipStream_t);
template hipError_t launch_append<float>(const Disch<float>*, int, int, hipStream_t);
template hipError_t launch_append<double>(const Disch<double>*, int, int, hipStream_t);
template hipError_t launch_diag<float>(int64_t, const float*, const float*, float*, hipStream_t);
template hipError_t launch_diag<double>(int64_t, const double*, const double*, double*,
                                        hipStream_t);

}  // namespace hd
