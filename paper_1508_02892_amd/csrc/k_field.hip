// End of a time step and field of the next one, one workgroup per discharge:
// offsets of the staged ionization children (exclusive scan over the electron
// launch's per-workgroup totals),
// ion-induced secondary emission (Sec. II.D), ion sources of the step
// (G^n in Eq 2.4), run averages, append bookkeeping, then the Poisson solve
// of the coupling (Sec. II.D) for the next step.  Further workgroups of the
// same launch append the children and secondaries to the particle arrays in
// canonical order while the field is solved.
#include "hd.h"
#include "hd_device.h"

namespace hd {

namespace {

constexpr double kECharge = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;

// Windows of 64 x kScanWin workgroup totals scanned by one wave per pass.
constexpr int kScanWin = 16;

// Secondary electrons of one wall (side 0: z = 0, side 1: z = L) for ion
// flux F: int(X) + Bernoulli(X - int(X)) superparticles, X = gamma F dt / w;
// cosine law, uniform azimuth, partial first flight.  Written to the
// emission buffer and deposited.
template <class P>
__device__ void emit(const Disch<P>& d, int side, double F, uint32_t step, int64_t* cn_lds,
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
    atomicAdd(reinterpret_cast<unsigned long long*>(&cn_lds[c]), (unsigned long long)W0);
    atomicAdd(reinterpret_cast<unsigned long long*>(&cn_lds[c + 1]), (unsigned long long)W1);
    m += 1;
  }
  *n_out = m;
}

template <class P>
__device__ __forceinline__ double scale_of(const Disch<P>& d, int j) {
  return (j == 0 || j == d.nc) ? d.scale_wall : d.scale_in;
}

// ---- Poisson solve with precomputed elimination factors --------------------
// The n interior rows split into P partitions (P = min(64, n/8), plain
// Thomas below 16 rows); each partition's interior rows are eliminated
// forward and backward, which leaves a reduced system of the partitions'
// first and last rows (2P rows).  That system is solved by parallel cyclic
// reduction: at stride s = 1, 2, 4, ... every row is combined with rows
// i - s and i + s (multipliers alpha_i = -a_i / b_{i-s}, gamma_i =
// -c_i / b_{i+s}, a missing neighbour entering with 0), and after
// ceil(log2 2P) steps x_i = d_i (1 / b_i).  The interior unknowns then
// follow from the partitions' end values.  The matrix is the constant
// (-1, 2, -1), so every factor is constant in time: the partitions' pivot
// reciprocals and eliminated coefficients depend only on a row's place in
// its partition and on the partition's length (n / P rounded down or up),
// and the reduction's multipliers only on the row and the step.  They are
// computed once, by the same operations in the same order as the general
// method, and each step runs only the right-hand-side recurrences (same
// results bit for bit, no division on the serial path).
constexpr double kPa = -1.0, kPb = 2.0, kPc = -1.0;
constexpr int kPcrSteps = 7;  // ceil(log2 128): the reduced system has at most 2 x 64 rows
constexpr int kFacMax = 6 * 64 + (2 * kPcrSteps + 1) * kTriRed;  // doubles of factor tables
constexpr int kPoisRed = 6 * kTriRed;  // doubles of LDS: reduced system (matrix scratch at set-up)

__host__ __device__ inline int field_partitions(int n) { return n < 16 ? 0 : (n / 8 < 64 ? n / 8 : 64); }

// Offsets (in doubles) of the factor tables for n unknowns: forward
// reciprocal pivot and eliminated c at local row k (fr, fc), final A and C
// for both partition lengths (xa, xc); the reduction's multipliers alpha and
// gamma of step k, row i at pal + k m2 + i and pga + k m2 + i, and 1 / b_i
// of the last step at prb (m2 = 2P rows, ns steps).  For P = 0 the plain
// Thomas factors of all n rows at fr and fc.
struct PoisFac {
  int n, P, L0, Lmax, size;
  float inv_n, inv_P;  // 1 / n, 1 / P rounded to FP32 (partition of a row, its start)
  int fr, fc, xa, xc;
  int m2, ns, pal, pga, prb;
};

__device__ inline PoisFac pois_fac(int n) {
  PoisFac f;
  f.n = n;
  f.inv_n = 1.0f / (float)n;
  f.P = field_partitions(n);
  f.inv_P = f.P ? 1.0f / (float)f.P : 0.0f;
  f.m2 = 2 * f.P;
  f.ns = 0;
  for (int s = 1; s < f.m2; s *= 2) ++f.ns;
  if (f.P == 0) {
    f.L0 = f.Lmax = 0;
    f.fr = 0;
    f.fc = n;
    f.xa = f.xc = f.pal = f.pga = f.prb = 2 * n;
    f.size = 2 * n;
    return f;
  }
  f.L0 = n / f.P;
  f.Lmax = f.L0 + 1;
  f.fr = 0;
  f.fc = f.Lmax;
  f.xa = 2 * f.Lmax;
  f.xc = 4 * f.Lmax;
  f.pal = 6 * f.Lmax;
  f.pga = f.pal + f.ns * f.m2;
  f.prb = f.pga + f.ns * f.m2;
  f.size = f.prb + f.m2;
  return f;
}

// One thread: all factors for n unknowns into t; scr: 6 * kTriRed doubles
// of LDS for the reduced matrix.
__device__ void pois_factor(const PoisFac& f, double* t, double* scr) {
  const double a = kPa, b = kPb, c = kPc;
  if (f.P == 0) {
    double rr = 1.0 / b;
    double cp = c * rr;
    t[f.fr] = rr;
    t[f.fc] = cp;
    for (int j = 1; j < f.n; ++j) {
      const double den = b - a * cp;
      rr = 1.0 / den;
      cp = c * rr;
      t[f.fr + j] = rr;
      t[f.fc + j] = cp;
    }
    return;
  }
  const int Lm = f.Lmax;
  // forward elimination of the interior rows k = 1 .. Lmax - 2 (identical in
  // every partition); forward A and C to both length classes
  double r = 1.0 / b, ap = a * r, cp = c * r;
  for (int k = 1; k <= Lm - 2; ++k) {
    if (k > 1) {
      r = 1.0 / (b - a * cp);
      ap = -(a * ap) * r;
      cp = c * r;
    }
    t[f.fr + k] = r;
    t[f.fc + k] = cp;
    t[f.xa + k] = ap;
    t[f.xa + Lm + k] = ap;
    t[f.xc + k] = cp;
    t[f.xc + Lm + k] = cp;
  }
  // backward elimination for partitions of length L0 and L0 + 1
  for (int cls = 0; cls < 2; ++cls) {
    const int L = f.L0 + cls;
    double* xa = t + f.xa + cls * Lm;
    double* xc = t + f.xc + cls * Lm;
    double bap = xa[L - 2], bcp = xc[L - 2];
    for (int k = L - 3; k >= 1; --k) {
      const double ci = t[f.fc + k];
      bap = xa[k] - ci * bap;
      bcp = -(ci * bcp);
      xa[k] = bap;
      xc[k] = bcp;
    }
  }
  // the reduced system's matrix: the first and last rows of every partition
  const int m = f.m2;
  double* A = scr;
  double* B = scr + kTriRed;
  double* C = scr + 2 * kTriRed;
  double* A2 = scr + 3 * kTriRed;
  double* B2 = scr + 4 * kTriRed;
  double* C2 = scr + 5 * kTriRed;
  for (int j = 0; j < m; ++j) {
    const int p = j >> 1;
    const int s = (int)((int64_t)p * f.n / f.P);
    const int e = (int)((int64_t)(p + 1) * f.n / f.P) - 1;
    const int L = e - s + 1;
    const double* xa = t + f.xa + (L - f.L0) * Lm;
    const double* xc = t + f.xc + (L - f.L0) * Lm;
    if ((j & 1) == 0) {
      A[j] = a;
      B[j] = b - c * xa[1];
      C[j] = -(c * xc[1]);
    } else {
      A[j] = -(a * xa[L - 2]);
      B[j] = b - a * xc[L - 2];
      C[j] = c;
    }
  }
  A[0] = 0.0;
  C[m - 1] = 0.0;
  // the reduction's multipliers, step by step
  int k = 0;
  for (int s = 1; s < m; s *= 2, ++k) {
    for (int i = 0; i < m; ++i) {
      const bool lo = i - s >= 0, hi = i + s < m;
      const double al = lo ? -A[i] / B[i - s] : 0.0;
      const double ga = hi ? -C[i] / B[i + s] : 0.0;
      A2[i] = lo ? al * A[i - s] : 0.0;
      C2[i] = hi ? ga * C[i + s] : 0.0;
      B2[i] = (B[i] + (lo ? al * C[i - s] : 0.0)) + (hi ? ga * A[i + s] : 0.0);
      t[f.pal + k * m + i] = al;
      t[f.pga + k * m + i] = ga;
    }
    for (int i = 0; i < m; ++i) {
      A[i] = A2[i];
      B[i] = B2[i];
      C[i] = C2[i];
    }
  }
  for (int i = 0; i < m; ++i) t[f.prb + i] = 1.0 / B[i];
}

// Partition of interior row i, floor(((i + 1) P - 1) / n), evaluated as
// floor(((i + 1) P - 1/2) / n) in FP32: the half keeps the quotient at least
// 1/(2n) >= 2^-13 from an integer while the two roundings move it by at most
// P 2^-23 <= 2^-17 (n <= 4095, P <= 64), so the floor is exact.
__device__ __forceinline__ int pois_part(const PoisFac& f, int i) {
  return (int)(((float)((i + 1) * f.P) - 0.5f) * f.inv_n);
}

// First row of partition p, floor(p n / P), evaluated as
// floor((p n + 1/2) / P) in FP32 (the same argument: the quotient stays at
// least 1/(2P) >= 2^-7 from an integer).
__device__ __forceinline__ int pois_start(const PoisFac& f, int p) {
  return (int)(((float)(p * f.n) + 0.5f) * f.inv_P);
}

// Place of interior row i in the solver's array: partition p sits
// p doubles higher (the 64 lanes of a sweep, one partition each, then fall
// in different LDS banks).  Holds the right-hand side, then the solution.
__device__ __forceinline__ int pois_slot(const PoisFac& f, int i) {
  return f.P ? i + pois_part(f, i) : i;
}

// Right-hand-side sweeps of one partition: D[k] is row s + k (L
// rows, lane-dependent); forward v_1 = v_1 r_1, v_k = fma(m_k, v_{k-1},
// v_k r_k) for k = 2 .. L - 2; backward v_k = fma(f_k, v_{k+1}, v_k) for
// k = L - 3 .. 1 (f_k = -c'_k); D swept in place.  Rows go in batches of 8
// whose loads are issued together, so LDS latency is paid per batch, not per
// row; the batch at a sweep's end may reach past the partition: its extra
// rows are loaded (the arrays are padded for it) but neither computed into
// the chain (selects) nor stored.  Returns the forward value of row L - 2.
constexpr int kB = 8;
template <class FR, class FM, class FF>
__device__ __forceinline__ double part_sweep(double* D, int L, FR r, FM m, FF fneg) {
  double dp = D[1] * r(1);
  D[1] = dp;
  int k = 2;
  for (; k + kB - 1 <= L - 2; k += kB) {
    double dv[kB], mv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = D[k + u] * r(k + u);
      mv[u] = m(k + u);
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dp = fma(mv[u], dp, dv[u]);
      dv[u] = dp;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) D[k + u] = dv[u];
  }
  if (k <= L - 2) {  // rows k .. L - 2 (fewer than kB)
    double dv[kB], mv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = D[k + u] * r(k + u);
      mv[u] = m(k + u);
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const double nv = fma(mv[u], dp, dv[u]);
      dp = (k + u <= L - 2) ? nv : dp;
      dv[u] = nv;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (k + u <= L - 2) D[k + u] = dv[u];
  }
  const double vf = dp;
  // backward in batches [1 + kB j, kB + kB j]; the top one holds row L - 3
  int j = (L - 4) / kB;
  {
    const int b = 1 + kB * j;
    double dv[kB], cv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = D[b + u];
      cv[u] = fneg(b + u);
    }
#pragma unroll
    for (int u = kB - 1; u >= 0; --u) {
      const double nv = fma(cv[u], dp, dv[u]);
      const bool ok = b + u <= L - 3;
      dp = ok ? nv : dp;
      dv[u] = nv;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (b + u <= L - 3) D[b + u] = dv[u];
  }
  for (--j; j >= 0; --j) {
    const int b = 1 + kB * j;
    double dv[kB], cv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = D[b + u];
      cv[u] = fneg(b + u);
    }
#pragma unroll
    for (int u = kB - 1; u >= 0; --u) {
      dp = fma(cv[u], dp, dv[u]);
      dv[u] = dp;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) D[b + u] = dv[u];
  }
  return vf;
}

// Thomas sweeps of m rows (the same on every lane), in place: x_0 = d_0 r_0,
// x_j = fma(m_j, x_{j-1}, d_j r_j), then x_j = fma(-cp_j, x_{j+1}, x_j);
// batches of 8 as above.
template <class FR, class FM, class FC>
__device__ __forceinline__ void thomas_sweep(double* X, int m, FR r, FM mm, FC cp) {
  double dp = X[0] * r(0);
  X[0] = dp;
  for (int k = 1; k <= m - 1; k += kB) {
    double dv[kB], mv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = X[k + u] * r(k + u);
      mv[u] = mm(k + u);
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const double nv = fma(mv[u], dp, dv[u]);
      dp = (k + u <= m - 1) ? nv : dp;
      dv[u] = nv;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (k + u <= m - 1) X[k + u] = dv[u];
  }
  for (int b = ((m - 2) / kB) * kB; b >= 0; b -= kB) {  // batches [b, b + kB) from the top
    double dv[kB], cv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      dv[u] = X[b + u];
      cv[u] = -cp(b + u);
    }
#pragma unroll
    for (int u = kB - 1; u >= 0; --u) {
      const double nv = fma(cv[u], dp, dv[u]);
      const bool ok = b + u <= m - 2;
      dp = ok ? nv : dp;
      dv[u] = nv;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (b + u <= m - 2) X[b + u] = dv[u];
  }
}

// The partition of lane p (rows s .. s + L - 1 at dd[0 ..]): swept in
// place, the reduced right-hand side to Dn.
__device__ __forceinline__ void partition_sweep(const PoisFac& f, const double* t, double* dd, int L,
                                             double* Dn, int p) {
  const double a = kPa, c = kPc;
  const double* fr = t + f.fr;
  const double* fc = t + f.fc;
  const double d0 = dd[0], de = dd[L - 1];
  const double vf = part_sweep(
      dd, L, [&](int k) { return fr[k]; }, [&](int k) { return -(a * fr[k]); },
      [&](int k) { return -fc[k]; });
  Dn[2 * p] = fma(-c, dd[1], d0);
  Dn[2 * p + 1] = fma(-a, vf, de);
}

// Orders the calling wave's LDS writes before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Solve of the (-1, 2, -1) system, in two parts around a workgroup barrier:
// pois_sweeps (wave 0) and pois_recover (every thread).  The right-hand side
// is in d (row i at pois_slot(i)) and is swept in place; the recovery writes
// the solution in natural order; t: factor tables (LDS); red: kPoisRed
// doubles of LDS (the reduced
// system's right-hand side at [0, 2P), its solution at kTriRed, the
// reduction's exchange buffer at 2 kTriRed).  The partitions' sweeps run one
// partition per lane, the reduction runs rows i and i + 64 on lane i, and
// the interior unknowns are recovered by every thread.  The right-hand side
// is carried by fused multiply-adds, one rounding per row of a sweep:
// forward d'_i = fma(-(a r_i), d'_{i-1}, d_i r_i), backward d'_i =
// fma(-c'_i, d'_{i+1}, d'_i), reduction d'_i = fma(gamma_i, d_{i+s},
// fma(alpha_i, d_{i-s}, d_i)).
__device__ void pois_sweeps(const PoisFac& f, const double* t, double* d, double* red) {
  const int lane = threadIdx.x, n = f.n, P = f.P;
  const double a = kPa;
  if (P == 0) {  // n < 16: plain Thomas, on all of wave 0 (the same values)
    const int zo = (int)(threadIdx.x / blockDim.x);
    thomas_sweep(
        d + zo, n, [&](int j) { return t[f.fr + zo + j]; },
        [&](int j) { return -(a * t[f.fr + zo + j]); }, [&](int j) { return t[f.fc + zo + j]; });
    return;
  }
  if (lane < P) {  // one partition per lane
    const int s = pois_start(f, lane);
    const int L = pois_start(f, lane + 1) - s;
    partition_sweep(f, t, d + s + lane, L, red, lane);
  }
  wave_sync();
  // parallel cyclic reduction of the 2P rows: rows r0 = lane, r1 = lane + 64
  const int m = f.m2, r0 = lane, r1 = lane + 64;
  const bool v0 = r0 < m, v1 = r1 < m;
  const int i0 = v0 ? r0 : 0, i1 = v1 ? r1 : 0;  // table rows (clamped)
  double* ex = red + 2 * kTriRed;
  double d0 = red[i0], d1 = red[i1];
  for (int k = 0, s = 1; k < f.ns; ++k, s *= 2) {
    ex[r0] = d0;
    ex[r1] = d1;
    const double al0 = t[f.pal + k * m + i0], ga0 = t[f.pga + k * m + i0];
    const double al1 = t[f.pal + k * m + i1], ga1 = t[f.pga + k * m + i1];
    wave_sync();
    const double dm0 = r0 - s >= 0 ? ex[v0 && r0 - s >= 0 ? r0 - s : 0] : 0.0;
    const double dp0 = r0 + s < m ? ex[r0 + s < m ? r0 + s : 0] : 0.0;
    const double dm1 = r1 - s >= 0 && v1 ? ex[v1 ? r1 - s : 0] : 0.0;
    const double dp1 = r1 + s < m ? ex[r1 + s < m ? r1 + s : 0] : 0.0;
    d0 = fma(ga0, dp0, fma(al0, dm0, d0));
    d1 = fma(ga1, dp1, fma(al1, dm1, d1));
    wave_sync();
  }
  double* xr = red + kTriRed;
  if (v0) xr[r0] = d0 * t[f.prb + r0];
  if (v1) xr[r1] = d1 * t[f.prb + r1];
}

// The interior unknowns from their partition's end values, written in
// natural order to x (row i at x[i]; x may not overlap d or red).
__device__ void pois_recover(const PoisFac& f, const double* t, const double* d, const double* red,
                             double* x) {
  const int n = f.n;
  if (f.P == 0) {  // the plain Thomas solve left the solution in d
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = d[i];
    return;
  }
  const double* rx = red + kTriRed;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int p = pois_part(f, i);
    const int s = pois_start(f, p);
    const int e = pois_start(f, p + 1) - 1;
    const double xs = rx[2 * p], xe = rx[2 * p + 1];
    double xi;
    if (i == s) {
      xi = xs;
    } else if (i == e) {
      xi = xe;
    } else {
      const int o = (e - s + 1 - f.L0) * f.Lmax + (i - s);
      xi = fma(-t[f.xc + o], xe, fma(-t[f.xa + o], xs, d[i + p]));
    }
    x[i] = xi;
  }
}

// LDS of the finalize kernel (doubles): the solution, this step's deposit
// and its emission part, the reduced system and the factor tables.
__host__ __device__ constexpr size_t finalize_lds_doubles(int nn_max) {
  return 3u * (size_t)nn_max + 64u + (size_t)kPoisRed + kFacMax;
}

// Grid nodes belong to the threads of waves 1 .. 15 of the end-of-step
// workgroup (wave 0 keeps the serial work: emission, sweeps); node j of
// thread t >= 64 is j = (t - 64) + u kNodeThreads; nodes per thread for at
// most 4097 nodes.
constexpr int kNodeThreads = kFinThreads - 64;
constexpr int kNodeSlots = (kMaxNodes + kNodeThreads - 1) / kNodeThreads;

// End of a step (field_only == 0) and the field of the next one.  Global
// inputs are loaded together up front so that the kernel pays few memory
// round trips: the state, this step's deposit, n_i and the ion sources,
// the first tile of child counts, the factor tables and V(t).
// ---- append, in the workgroups of the end-of-step launch after the first D
// Append this step's children (in sub-chunk order, i.e. parent order), then the
// left and right secondaries, with consecutive ids.  A sub-chunk's children
// start at its workgroup's offset (from the end-of-step scan) plus its own
// offset inside the workgroup (from the electron launch).  Each wave takes 64
// consecutive sub-chunks and copies the children of each non-empty one with
// all of its lanes.  The workgroups wait (bounded) for the discharge's
// end-of-step workgroup to publish its offsets; the last one to finish
// re-arms the flag for the next launch.
constexpr int kSpinMax = 1 << 17;  // ~0.2 s: a backstop, never reached in a correct run

__device__ __forceinline__ void publish_ready(State* st) {
  __hip_atomic_store(&st->fin_ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class P>
__device__ __forceinline__ void append_one(const Disch<P>& d, int buf, uint32_t src_c, uint32_t dst,
                                           uint32_t id, const Gp<int32_t>* sc, const Gp<P>* so,
                                           const Gp<P>* sx, const Gp<P>* sy, const Gp<P>* sz) {
  gptr(d.cell[buf])[dst] = sc[src_c];
  gptr(d.off[buf])[dst] = so[src_c];
  gptr(d.vx[buf])[dst] = sx[src_c];
  gptr(d.vy[buf])[dst] = sy[src_c];
  gptr(d.vz[buf])[dst] = sz[src_c];
  gptr(d.id[buf])[dst] = id;
}

template <class P>
__device__ void append_blocks(const Disch<P>* __restrict__ ds, int D) {
  __shared__ int ok;
  __shared__ int gave_up;  // a wait timed out: wait for no further discharge
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  if (tid == 0) gave_up = 0;
  // The append workgroups form groups of G, each group serving every
  // groups-th discharge: all of them on one discharge when it is alone, one
  // per discharge when the batch has as many discharges as workgroups, so
  // that a batch's discharges are appended side by side, not one by one.
  const uint32_t ab = blockIdx.x - (uint32_t)D, nab = gridDim.x - (uint32_t)D;
  const uint32_t G = max(1u, nab / (uint32_t)D), groups = nab / G, gi = ab / G, gr = ab % G;
  if (gi >= groups) return;  // the remainder of nab / G: no group
  const uint32_t wave = (gr * (uint32_t)kFinThreads + tid) >> 6;
  const uint32_t nwaves = G * (uint32_t)(kFinThreads / 64);
  const uint32_t gid = gr * (uint32_t)kFinThreads + tid, gsz = G * (uint32_t)kFinThreads;
  for (int di = (int)gi; di < D; di += (int)groups) {
    const Disch<P>& d = ds[di];
    State* st = d.st;
    if (tid == 0) {
      // relaxed polling (an acquire per poll would invalidate the caches of
      // the whole XCD each time), then one acquire for the workgroup
      int it = gave_up ? kSpinMax : 0;
      while (it < kSpinMax &&
             __hip_atomic_load(&st->fin_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        __builtin_amdgcn_s_sleep(2);
        ++it;
      }
      ok = it < kSpinMax;
      if (!ok) gave_up = 1;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!ok) {
      if (tid == 0) st->error = HD_ESYNC;  // the end-of-step workgroup never published
    } else if (st->append_pending) {
      const int buf = st->buf;
      const uint32_t nch = st->n_chunks, base = st->append_base, idb = st->id_base;
      const uint32_t nk = st->n_kids, n0 = st->n_see[0], n1 = st->n_see[1];
      const uint32_t soff = st->seg_off, sper = st->seg_per;
      const Gp<uint32_t>* kids = gptr(d.chunk_kids);
      const Gp<uint32_t>* cbase = gptr(d.chunk_base);
      const Gp<uint32_t>* sbase = gptr(d.seg);
      for (uint32_t k0 = wave * 64u; k0 < nch; k0 += nwaves * 64u) {
        const uint32_t k = k0 + lane;
        const uint32_t cnt = k < nch ? kids[k] : 0u;
        uint64_t live = __ballot(cnt != 0u);
        if (live == 0) continue;
        // offset = the workgroup's among all children + the sub-chunk's in it
        const uint32_t cb =
            cnt ? sbase[(soff + k / (uint32_t)(kTile / kSub)) / sper] + cbase[k] : 0u;
        while (live) {
          const int l = __ffsll((unsigned long long)live) - 1;
          live &= live - 1;
          const uint32_t n = (uint32_t)__shfl((int)cnt, l, 64);
          const uint32_t b = (uint32_t)__shfl((int)cb, l, 64);
          const uint32_t src0 = (k0 + (uint32_t)l) * (uint32_t)kSub;
          for (uint32_t t = lane; t < n; t += 64u)
            append_one<P>(d, buf, src0 + t, base + b + t, idb + b + t, gptr(d.kc), gptr(d.koff),
                          gptr(d.kvx), gptr(d.kvy), gptr(d.kvz));
        }
      }
      for (uint32_t t = gid; t < n0 + n1; t += gsz) {
        const uint32_t src = t < n0 ? t : (uint32_t)kSeeMax + (t - n0);
        append_one<P>(d, buf, src, base + nk + t, idb + nk + t, gptr(d.sc), gptr(d.soff),
                      gptr(d.svx), gptr(d.svy), gptr(d.svz));
      }
    }
    __syncthreads();
    if (tid == 0) {
      if (atomicAdd(&st->app_done, 1u) == G - 1u) {  // the group's last: re-arm for the next launch
        st->app_done = 0u;
        __hip_atomic_store(&st->fin_ready, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

template <class P>
__global__ __launch_bounds__(kFinThreads) void k_finalize(const Disch<P>* __restrict__ ds, int D,
                                                          int field_only) {
  extern __shared__ __align__(16) unsigned char smem[];
  if ((int)blockIdx.x >= D) {
    append_blocks<P>(ds, D);
    return;
  }
  const Disch<P>& d = ds[blockIdx.x];
  Gp<State>* st = gptr(d.st);
  const int tid = threadIdx.x, nn = d.nn, nc = d.nc, m = nc - 1;
  // the wave index as a uniform value, so that branches on it stay branches
  // (registers live in one wave's path are not kept through another's)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int kLastWave = kFinThreads / 64 - 1;
  const bool node = wave > 0;     // owns grid nodes
  const int nt = tid - 64;        // its index among the node threads
  double* X = reinterpret_cast<double*>(smem);         // interior rows (pois_slot), right-hand side then solution
  int64_t* CN = reinterpret_cast<int64_t*>(X + nn + 64);  // deposit of the step
  int64_t* EN = CN + nn;                                   // its emission part
  double* red = reinterpret_cast<double*>(EN + nn);
  double* T = red + kPoisRed;
  __shared__ uint32_t sh_see[2];
  __shared__ double sh_pw[4];  // power bookkeeping of the step (thread 0)
  __shared__ int64_t sh_per;
  // Global inputs are requested before any of them is used: the state, both
  // deposit buffers (the state says which is this step's), n_i, the ion
  // sources, the run sums of n_i and the Poisson factor tables.
  const int64_t steps_left = st->steps_left;
  const int64_t step0 = st->step;
  const int cbuf0 = st->cbuf;
  const uint32_t n_main = st->n_main;
  const uint32_t next_id = st->next_id;
  const uint32_t seg_off = st->seg_off, seg_per = st->seg_per;
  const double wall_g = tid < 2 ? st->wall[tid] : 0.0;
  const double amp = st->volt_amp;
  const Gp<int64_t>* gc0 = gptr(d.cnt[0]);
  const Gp<int64_t>* gc1 = gptr(d.cnt[1]);
  const Gp<double>* gni = gptr(d.ni);
  const Gp<int64_t>* gsrc = gptr(d.ion_src);
  Gp<double>* acc_ni = gptr(d.acc_ni);
  int64_t c0v[kNodeSlots], c1v[kNodeSlots], srcv[kNodeSlots];
  double n0v[kNodeSlots], accv[kNodeSlots];
#pragma unroll
  for (int u = 0; u < kNodeSlots; ++u) {
    const int j = nt + u * kNodeThreads;
    c0v[u] = c1v[u] = srcv[u] = 0;
    n0v[u] = accv[u] = 0.0;
    if (node && j < nn) {
      c0v[u] = gc0[j];
      c1v[u] = gc1[j];
      n0v[u] = gni[j];
      if (!field_only) {
        srcv[u] = gsrc[j];
        accv[u] = acc_ni[j];
      }
    }
  }
  const PoisFac f = pois_fac(m);
  Gp<double>* gtab = gptr(d.scratch);
  constexpr int kTabSlots = (kFacMax + kFinThreads - 1) / kFinThreads;
  double tv[kTabSlots];
  if (!field_only) {
#pragma unroll
    for (int u = 0; u < kTabSlots; ++u) {
      const int i = tid + u * kFinThreads;
      tv[u] = i < f.size ? gtab[i] : 0.0;
    }
  }
  if (!field_only && steps_left <= 0) {
    if (tid == 0) {  // nothing completed: nothing to append
      st->append_pending = 0;
      publish_ready(d.st);
    }
    return;
  }
  const int64_t step1 = field_only ? step0 : step0 + 1;
  const int cur = field_only ? cbuf0 : (cbuf0 ^ 1);
  Gp<int64_t>* cn = gptr(d.cnt[cur]);
  const Gp<double>* volt = gptr(d.volt);
  const double V = amp * ((step1 < d.volt_len) ? volt[step1] : 0.0);
  // absorbed-power bookkeeping inputs (thread 0): the field and voltage of
  // the level this step started from and the electron counts at z = 0
  double e0_old = 0.0, v_old = 0.0, pw_sum = 0.0;
  uint64_t abs0 = 0, emi0 = 0, abs_prev = 0, emi_prev = 0;
  int64_t periods = 0;
  if (!field_only && tid == 0) {
    e0_old = gptr(d.E)[0];
    v_old = gptr(d.phi)[0];
    abs0 = st->absorbed[0];
    emi0 = st->emitted[0];
    abs_prev = st->pw_abs0;
    emi_prev = st->pw_emi0;
    pw_sum = st->pw_sum;
    periods = st->rf_periods;
  }
  // the electron launch's per-workgroup child totals of this discharge
  const uint32_t nchunk = field_only ? 0u : (n_main + (uint32_t)kTile - 1u) / (uint32_t)kTile;
  const uint32_t nch = nchunk * (uint32_t)(kTile / kSub);  // sub-chunks
  const uint32_t pb0 = nchunk ? seg_off / seg_per : 0u;
  const uint32_t pb1 = nchunk ? (seg_off + nchunk - 1u) / seg_per + 1u : 0u;  // exclusive
  Gp<uint32_t>* gseg = gptr(d.seg);
  // Emission deposits into a grid of its own (EN, zeroed here), so that it
  // can run beside the deposit's other updates; this step's final deposit
  // is CN + EN.

  // this step's deposit to LDS; n_i with this step's ion sources; with
  // several species the others are updated here too and netv is the ion
  // charge density sum_s Z_s n_s (species in order)
  double niv[kNodeSlots], netv[kNodeSlots];
#pragma unroll
  for (int u = 0; u < kNodeSlots; ++u) {
    const int j = nt + u * kNodeThreads;
    niv[u] = 0.0;
    netv[u] = 0.0;
    if (node && j < nn) {
      CN[j] = cur ? c1v[u] : c0v[u];
      niv[u] = field_only ? n0v[u] : n0v[u] + (double)srcv[u] * scale_of(d, j);
      netv[u] = niv[u];
      if (d.S > 1) {
        double net = (double)d.Z[0] * niv[u];
        for (int q = 1; q < d.S; ++q) {
          const size_t k = (size_t)q * (size_t)nn + (size_t)j;
          double nq = gni[k];
          if (!field_only) {
            nq = nq + (double)gsrc[k] * scale_of(d, j);
            gptr(d.ni)[k] = nq;
            gptr(d.ion_src)[k] = 0;
          }
          net = net + (double)d.Z[q] * nq;
        }
        netv[u] = net;
      }
      accv[u] = accv[u] + netv[u];  // the run sum after this step
    }
  }
  if (field_only) {
    if (tid == 0) pois_factor(f, T, red);
  } else {
#pragma unroll
    for (int u = 0; u < kTabSlots; ++u) {
      const int i = tid + u * kFinThreads;
      if (i < f.size) T[i] = tv[u];
    }
  }
  // emission from the wall fluxes of this step's fluid update (wave 0,
  // which zeroes the emission grid first and owns no nodes, so it starts as
  // soon as the state has arrived)
  if (!field_only && wave == 0) {
    for (int j = tid; j < nn; j += 64) EN[j] = 0;
    wave_sync();
  }
  if (!field_only && tid < 2) {
    double F = tid == 0 ? ((-wall_g < 0.0) ? 0.0 : -wall_g) : ((wall_g < 0.0) ? 0.0 : wall_g);
    if (d.ion_model == HD_ION_DD_SPECIES) F = st->see_flux[tid];  // positive ions only
    uint64_t em = 0, ab = 0, cl = 0;
    uint32_t n = 0;
    emit<P>(d, tid, F, (uint32_t)step0, EN, &n, &em, &ab, &cl);
    sh_see[tid] = n;
    if (tid == 0) {
      // Power delivered at the driven electrode over [t_n, t_n+1] (Eq 2.9's
      // integrand): conduction current e (Gamma_i - Gamma_e) from the ion
      // wall flux and the electrons that left / entered through z = 0 this
      // step, plus the displacement current eps0 dE/dt (finished once E is
      // known), times the mean voltage.
      abs0 += ab;  // totals at z = 0 after this step
      emi0 += em;
      const double dn = (double)(emi0 - emi_prev) - (double)(abs0 - abs_prev);
      const double ge = (d.w * dn) / d.dt;
      sh_pw[0] = pw_sum;
      sh_pw[1] = 0.5 * (v_old + V);
      sh_pw[2] = kECharge * (wall_g - ge);
      sh_pw[3] = e0_old;
      sh_per = periods;
      st->pw_abs0 = abs0;
      st->pw_emi0 = emi0;
    }
    if (em) atomicAdd(reinterpret_cast<unsigned long long*>(&d.st->emitted[tid]), (unsigned long long)em);
    if (ab) atomicAdd(reinterpret_cast<unsigned long long*>(&d.st->absorbed[tid]), (unsigned long long)ab);
    if (cl) atomicAdd(reinterpret_cast<unsigned long long*>(&d.st->see_clamped), (unsigned long long)cl);
  }
  __syncthreads();
  // ion sources of the step, the final deposit, run averages: written by
  // the node waves while wave 0 sweeps
  auto grid_out = [&]() {
    Gp<double>* wni = gptr(d.ni);
    Gp<int64_t>* wsrc = gptr(d.ion_src);
#pragma unroll
    for (int u = 0; u < kNodeSlots; ++u) {
      const int j = nt + u * kNodeThreads;
      if (node && j < nn) {
        const int64_t c = CN[j] + EN[j];
        wni[j] = niv[u];
        wsrc[j] = 0;
        cn[j] = c;
        atomicAdd(reinterpret_cast<unsigned long long*>(&d.acc_cnt[j]), (unsigned long long)c);
        acc_ni[j] = accv[u];
      }
    }
  };
  // Poisson's equation with phi_0 = V(t), phi_N = 0 for the interior nodes
  double rho_0 = 0.0, rho_n = 0.0;  // charge density at the walls (nodes 0 and nc)
#pragma unroll
  for (int u = 0; u < kNodeSlots; ++u) {
    const int j = nt + u * kNodeThreads;
    if (node && j < nn) {
      const int64_t c = field_only ? CN[j] : CN[j] + EN[j];
      const double ne = (double)c * scale_of(d, j);
      const double r = kECharge * (netv[u] - ne);
      if (j == 0) rho_0 = r;
      if (j == nc) rho_n = r;
      if (j >= 1 && j <= m) {
        double dj = d.kp * r;
        if (j == 1) dj = dj + V;
        if (j == m) dj = dj + 0.0;
        X[pois_slot(f, j - 1)] = dj;
      }
    }
  }
  // offsets of the staged children: exclusive scan of the electron launch's
  // per-workgroup totals, by the last wave alone while wave 0 sweeps; then
  // the append bookkeeping
  auto children = [&]() {
    const uint32_t lane = (uint32_t)tid & 63u;
    uint32_t n_kids = 0;
    // windows of 64 kScanWin totals; lane l takes kScanWin consecutive ones
    // (a serial scan in registers), then one wave scan of the lane sums
    for (uint32_t t0 = pb0; t0 < pb1; t0 += 64u * kScanWin) {
      const uint32_t k0 = t0 + lane * (uint32_t)kScanWin;
      uint32_t v[kScanWin];
#pragma unroll
      for (int w = 0; w < kScanWin; ++w) v[w] = k0 + (uint32_t)w < pb1 ? gseg[k0 + (uint32_t)w] : 0u;
      uint32_t sum = 0;
#pragma unroll
      for (int w = 0; w < kScanWin; ++w) sum += v[w];
      uint32_t x = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
      }
      uint32_t run = n_kids + x - sum;  // exclusive prefix of this lane's first total
#pragma unroll
      for (int w = 0; w < kScanWin; ++w) {
        if (k0 + (uint32_t)w < pb1) gseg[k0 + (uint32_t)w] = run;
        run += v[w];
      }
      n_kids += (uint32_t)__shfl((int)x, 63, 64);
    }
    if (lane != 0) return;
    const uint32_t ns0 = sh_see[0], ns1 = sh_see[1];
    const uint64_t n_app = (uint64_t)n_kids + ns0 + ns1;
    st->n_chunks = nch;
    st->n_kids = n_kids;
    st->n_see[0] = ns0;
    st->n_see[1] = ns1;
    const bool over = (uint64_t)n_main + n_app > (uint64_t)d.capacity;
    if (over) {
      // capacity exceeded: nothing is appended and no sort follows, so that
      // the other particle buffer still holds the interval's checkpoint
      st->error = HD_ECAPACITY;
      st->error_step = step0;
      st->append_pending = 0;
      st->steps_left = 0;
    } else {
      st->append_base = n_main;
      st->id_base = next_id;
      st->n_main = n_main + (uint32_t)n_app;
      st->next_id = next_id + (uint32_t)n_app;
      st->append_pending = n_app > 0 ? 1 : 0;
      st->steps_left = steps_left - 1;
    }
    st->step = step1;
    atomicAdd(reinterpret_cast<unsigned long long*>(&d.st->n_acc), 1ull);
    st->sort_due = (!over && (step1 % d.sort_every) == 0) ? 1 : 0;
    st->cbuf = cur;
    // the append workgroups of this launch may start (they run beside the
    // field solve)
    publish_ready(d.st);
  };
  __syncthreads();
  if (wave == 0) {
    pois_sweeps(f, T, X, red);
  } else if (!field_only) {
    if (wave == kLastWave) children();
    grid_out();
  }
  __syncthreads();
  // the solution in natural order, over this step's deposit grid (no longer
  // needed: the node waves stored it during the sweeps)
  double* Phi = reinterpret_cast<double*>(CN);
  pois_recover(f, T, X, red, Phi);
  __syncthreads();
  if (field_only)
    for (int i = tid; i < f.size; i += kFinThreads) gtab[i] = T[i];
  // E from centred differences inside and Gauss's law over the wall half
  // cells; E' = (-e/m_e) dt E rounded to the particle precision
  auto phi = [&](int j) { return j == 0 ? V : (j == nc ? 0.0 : Phi[j - 1]); };
  Gp<double>* gphi = gptr(d.phi);
  Gp<double>* gE = gptr(d.E);
  Gp<P>* gEp = gptr(d.Ep);
  Gp<int64_t>* nxt = gptr(d.cnt[cur ^ 1]);
  double e0_new = 0.0;
  bool finite = true;
#pragma unroll
  for (int u = 0; u < kNodeSlots; ++u) {
    const int j = nt + u * kNodeThreads;
    if (node && j < nn) {
      double e;
      if (j == 0)
        e = (phi(0) - phi(1)) * d.inv_dz - rho_0 * d.hdz_eps;
      else if (j == nc)
        e = (phi(nc - 1) - phi(nc)) * d.inv_dz + rho_n * d.hdz_eps;
      else
        e = (phi(j - 1) - phi(j + 1)) * d.inv_2dz;
      finite = finite && (fabs(e) <= 1.7976931348623157e308);  // false for inf and NaN
      gphi[j] = phi(j);
      gE[j] = e;
      gEp[j] = (P)(d.qm_dt * e);
      nxt[j] = 0;  // deposit target of the next step
      if (j == 0) e0_new = e;
    }
  }
  if (!field_only && tid == 64) {  // the owner of node 0
    // The interval belongs to the period that contains t_n+1; when that
    // level ends a period, the period's mean sets the next amplitude.
    const double jd = kEps0 * ((e0_new - sh_pw[3]) / d.dt);
    double sum = sh_pw[0] + sh_pw[1] * (sh_pw[2] + jd);
    if (d.rf_steps > 0 && step1 % d.rf_steps == 0) {
      const double pa = sum / (double)d.rf_steps;
      st->p_abs = pa;
      st->rf_periods = sh_per + 1;
      if (d.power_P0 > 0.0) st->volt_amp = amp * (1.0 - d.power_alpha * ((pa - d.power_P0) / d.power_P0));
      sum = 0.0;
    }
    st->pw_sum = sum;
  }
  // a field that is not finite stops the discharge: its next steps idle
  if (__syncthreads_or(finite ? 0 : 1) && tid == 0) {
    st->error = HD_ENUMERIC;
    st->error_step = step0;
    st->steps_left = 0;
    st->sort_due = 0;
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

// field_only: the field of the current state (at set-up), no step ends and
// no append workgroups.  Otherwise app_blocks (>= 1) workgroups append.
template <class P>
hipError_t launch_finalize(const Disch<P>* d_dev, int D, int field_only, int nn_max,
                           int app_blocks, hipStream_t s) {
  const size_t lds = finalize_lds_doubles(nn_max) * 8u;
  const int grid = D + (field_only ? 0 : app_blocks);
  hipLaunchKernelGGL(k_finalize<P>, dim3(grid), dim3(kFinThreads), lds, s, d_dev, D, field_only);
  return hipGetLastError();
}

template <class P>
hipError_t finalize_set_lds(int nn_max) {
  return hipFuncSetAttribute((const void*)k_finalize<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(finalize_lds_doubles(nn_max) * 8u));
}

template hipError_t finalize_set_lds<float>(int);
template hipError_t finalize_set_lds<double>(int);

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
template hipError_t launch_finalize<float>(const Disch<float>*, int, int, int, int, hipStream_t);
template hipError_t launch_finalize<double>(const Disch<double>*, int, int, int, int, hipStream_t);
template hipError_t launch_diag<float>(int64_t, const float*, const float*, float*, hipStream_t);
template hipError_t launch_diag<double>(int64_t, const double*, const double*, double*,
                                        hipStream_t);

}  // namespace hd
