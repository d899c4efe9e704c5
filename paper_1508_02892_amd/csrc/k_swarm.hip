// Auxiliary ion Monte Carlo (Sec. II.C) on gfx950: swarms of one ion species
// in prescribed uniform fields E0 and a Maxwellian background gas, giving the
// stationary drift u from which the mobility u/E0 and, by Eq (2.6), the
// momentum-exchange frequency follow.  The field is uniform and the domain
// periodic, so positions never enter and every ion is independent: one
// thread owns one ion for a whole launch of many steps, its velocity and
// running sums stay in registers, and HBM is touched only at the ends of the
// launch.  The null-collision rate table sits in LDS.
#include "hd_device.h"

namespace hd {
namespace {

// Two standard normal deviates by Marsaglia's polar method from FP64
// uniforms; (0, 0) after kSphereTries points outside the unit disk.
template <bool V>
__device__ __forceinline__ void normal_pair(StreamT<V>& st, double& g0, double& g1) {
  for (int t = 0; t < kSphereTries; ++t) {
    const double a = 2.0 * Uni<double>::get(st) - 1.0;
    const double b = 2.0 * Uni<double>::get(st) - 1.0;
    const double q = a * a + b * b;
    if (q < 1.0 && q > 0.0) {
      const double f = sqrt((-2.0 * fit_log(q)) / q);
      g0 = a * f;
      g1 = b * f;
      return;
    }
  }
  g0 = 0.0;
  g1 = 0.0;
}

// A Maxwellian velocity of thermal speed vth: three deviates of two polar
// pairs (the fourth is drawn and dropped), rounded to P.
template <class P, bool V>
__device__ __forceinline__ void maxwellian(StreamT<V>& st, double vth, P& x, P& y, P& z) {
  double g0, g1, g2, g3;
  normal_pair(st, g0, g1);
  normal_pair(st, g2, g3);
  x = (P)(vth * g0);
  y = (P)(vth * g1);
  z = (P)(vth * g2);
}

template <class P>
__global__ __launch_bounds__(kSwarmThreads) void k_swarm_init(SwarmDev<P> w) {
  const int64_t gid = (int64_t)blockIdx.x * kSwarmThreads + threadIdx.x;
  if (gid >= (int64_t)w.n_fields * w.n_ions) return;
  const int f = (int)(gid / w.n_ions);
  const uint32_t i = (uint32_t)(gid - (int64_t)f * w.n_ions);
  Stream st(w.seed, kTagSwarmLoad + 16u * (uint32_t)f, i, 0u);
  P x, y, z;
  maxwellian<P>(st, w.vth_i0, x, y, z);
  w.vx[gid] = x;
  w.vy[gid] = y;
  w.vz[gid] = z;
  w.avz[gid] = 0.0;
  w.av2[gid] = 0.0;
}

// n_steps steps of every ion, starting at step index step0.  Each step:
// v_z += e E0 dt / M; the stream (kTagSwarm + 16 f, ion, step) gives u0;
// for u0 < P_max a gas atom's velocity is drawn, and the collision is real
// when u0 < P_max nu(eps)/nu_max at the pair's relative energy
// eps = M_r g^2/(2e) (table interpolated linearly, last interval beyond
// its end); a real collision keeps the centre-of-mass velocity and turns
// the relative velocity g to a random direction: v' = (m1 v + m2 v_t) +
// m2 |g| n.  With accumulate, the step's v_z and |v|^2 join the ion's sums.
template <class P>
__global__ __launch_bounds__(kSwarmThreads) void k_swarm_step(SwarmDev<P> w, uint32_t step0,
                                                               int n_steps, int accumulate) {
  extern __shared__ __align__(16) unsigned char smem[];
  P* tab = reinterpret_cast<P*>(smem);
  __shared__ uint32_t cnt[2];
  const int tid = threadIdx.x;
  for (int k = tid; k < w.ne; k += kSwarmThreads) tab[k] = w.tab[k];
  if (tid < 2) cnt[tid] = 0u;
  __syncthreads();
  const int64_t bpf = (w.n_ions + kSwarmThreads - 1) / kSwarmThreads;  // blocks per swarm
  const int f = (int)((int64_t)blockIdx.x / bpf);
  const int64_t i = ((int64_t)blockIdx.x - (int64_t)f * bpf) * kSwarmThreads + tid;
  uint32_t n_coll = 0, n_over = 0;
  if (i < w.n_ions) {
    const int64_t k = (int64_t)f * w.n_ions + i;
    P vx = w.vx[k], vy = w.vy[k], vz = w.vz[k];
    double az = w.avz[k], a2 = w.av2[k];
    const P acc = w.a[f];
    const P Pmax = w.Pmax, KEr = w.KEr, inv_dE = w.inv_dE, m1 = w.m1, m2 = w.m2;
    const P top = (P)(w.ne - 1);
    const uint32_t tag = kTagSwarm + 16u * (uint32_t)f;
    for (int s = 0; s < n_steps; ++s) {
      StreamT<true> st(w.seed, tag, (uint32_t)i, step0 + (uint32_t)s);  // one ion per lane
      vz = vz + acc;
      const P u0 = Uni<P>::get(st);
      if (u0 < Pmax) {
        P tx, ty, tz;
        maxwellian<P>(st, w.vth_n, tx, ty, tz);
        const P gx = vx - tx, gy = vy - ty, gz = vz - tz;
        const P g2 = (gx * gx + gy * gy) + gz * gz;
        const P sc = (KEr * g2) * inv_dE;
        int j;
        P t;
        if (!(sc < top)) {  // beyond the table (or not a number)
          j = w.ne - 2;
          t = (P)1;
          n_over += 1u;
        } else {
          j = (int)sc;
          t = sc - (P)j;
        }
        const P pc = tab[j] + t * (tab[j + 1] - tab[j]);
        if (u0 < pc) {
          P nx, ny, nz;
          sphere<P>(st, nx, ny, nz);
          const P r = m2 * sqrt(g2);
          vx = (m1 * vx + m2 * tx) + r * nx;
          vy = (m1 * vy + m2 * ty) + r * ny;
          vz = (m1 * vz + m2 * tz) + r * nz;
          n_coll += 1u;
        }
      }
      if (accumulate) {
        const double x = (double)vx, y = (double)vy, z = (double)vz;
        az = az + z;
        a2 = a2 + ((x * x + y * y) + z * z);
      }
    }
    w.vx[k] = vx;
    w.vy[k] = vy;
    w.vz[k] = vz;
    w.avz[k] = az;
    w.av2[k] = a2;
  }
  if (n_coll) atomicAdd(&cnt[0], n_coll);
  if (n_over) atomicAdd(&cnt[1], n_over);
  __syncthreads();
  if (tid == 0 && cnt[0])
    atomicAdd(reinterpret_cast<unsigned long long*>(&w.coll[f]), (unsigned long long)cnt[0]);
  if (tid == 1 && cnt[1])
    atomicAdd(reinterpret_cast<unsigned long long*>(&w.over[f]), (unsigned long long)cnt[1]);
}

// Clears the per-swarm counters and sums (a fill kernel rather than a
// memset, so that the launch may be captured into a graph).
template <class P>
__global__ void k_swarm_clear(SwarmDev<P> w) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= w.n_fields) return;
  w.coll[f] = 0;
  w.over[f] = 0;
  w.sums[2 * f] = 0.0;
  w.sums[2 * f + 1] = 0.0;
}

// Sums over the ions of one swarm (block f) in a fixed order: strided
// per-thread sums, then a pairwise tree in LDS.
constexpr int kRedThreads = 1024;
template <class P>
__global__ __launch_bounds__(kRedThreads) void k_swarm_reduce(SwarmDev<P> w) {
  __shared__ double r1[kRedThreads], r2[kRedThreads];
  const int f = blockIdx.x, tid = threadIdx.x;
  const double* az = w.avz + (int64_t)f * w.n_ions;
  const double* a2 = w.av2 + (int64_t)f * w.n_ions;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = tid; i < w.n_ions; i += kRedThreads) {
    s1 = s1 + az[i];
    s2 = s2 + a2[i];
  }
  r1[tid] = s1;
  r2[tid] = s2;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      r1[tid] = r1[tid] + r1[tid + h];
      r2[tid] = r2[tid] + r2[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    w.sums[2 * f] = r1[0];
    w.sums[2 * f + 1] = r2[0];
  }
}

}  // namespace

template <class P>
hipError_t launch_swarm_init(const SwarmDev<P>& w, hipStream_t s) {
  const int64_t total = (int64_t)w.n_fields * w.n_ions;
  const unsigned grid = (unsigned)((total + kSwarmThreads - 1) / kSwarmThreads);
  hipLaunchKernelGGL(k_swarm_init<P>, dim3(grid), dim3(kSwarmThreads), 0, s, w);
  return hipGetLastError();
}

template <class P>
hipError_t launch_swarm_step(const SwarmDev<P>& w, uint32_t step0, int n_steps, int accumulate,
                             hipStream_t s) {
  const int64_t bpf = (w.n_ions + kSwarmThreads - 1) / kSwarmThreads;
  const unsigned grid = (unsigned)(bpf * w.n_fields);
  const size_t lds = (size_t)w.ne * sizeof(P);
  hipLaunchKernelGGL(k_swarm_step<P>, dim3(grid), dim3(kSwarmThreads), lds, s, w, step0, n_steps,
                     accumulate);
  return hipGetLastError();
}

template <class P>
hipError_t launch_swarm_clear(const SwarmDev<P>& w, hipStream_t s) {
  hipLaunchKernelGGL(k_swarm_clear<P>, dim3((w.n_fields + 255) / 256), dim3(256), 0, s, w);
  return hipGetLastError();
}

template <class P>
hipError_t launch_swarm_reduce(const SwarmDev<P>& w, hipStream_t s) {
  hipLaunchKernelGGL(k_swarm_reduce<P>, dim3(w.n_fields), dim3(kRedThreads), 0, s, w);
  return hipGetLastError();
}

template hipError_t launch_swarm_init<float>(const SwarmDev<float>&, hipStream_t);
template hipError_t launch_swarm_init<double>(const SwarmDev<double>&, hipStream_t);
template hipError_t launch_swarm_step<float>(const SwarmDev<float>&, uint32_t, int, int,
                                             hipStream_t);
template hipError_t launch_swarm_step<double>(const SwarmDev<double>&, uint32_t, int, int,
                                              hipStream_t);
template hipError_t launch_swarm_reduce<float>(const SwarmDev<float>&, hipStream_t);
template hipError_t launch_swarm_clear<float>(const SwarmDev<float>&, hipStream_t);
template hipError_t launch_swarm_clear<double>(const SwarmDev<double>&, hipStream_t);
template hipError_t launch_swarm_reduce<double>(const SwarmDev<double>&, hipStream_t);

}  // namespace hd
