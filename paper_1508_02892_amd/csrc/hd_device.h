// Device-side helpers: the counter-based Philox4x32-10 stream, uniform maps,
// vector memory access and wave-level utilities for gfx950 (wave64).
#pragma once

#include "hd_internal.h"

namespace hd {

enum : uint32_t {
  kTagElectron = 0,
  kTagLoad = 1,
  kTagEmission = 2,
  kTagSwarm = 3,     // swarm steps; + 16 x field index
  kTagSwarmLoad = 4  // swarm initial velocities; + 16 x field index
};

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products with the published multipliers; the key advances
// by the published Weyl increments between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                              uint32_t k0, uint32_t k1, uint32_t& o0,
                                              uint32_t& o1, uint32_t& o2, uint32_t& o3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
  }
  o0 = x0;
  o1 = x1;
  o2 = x2;
  o3 = x3;
}

// The same block for code that runs it on every lane of full waves: from
// the third round on, hi(M*x) ^ x' ^ key is one three-input bitwise op
// (truth table 0x96) instead of two xors.  The first two rounds keep plain
// xors, where wave-uniform counter words and keys fold into scalar ops; so
// does the plain version above, for code where most operands are uniform.
__device__ __forceinline__ void philox4x32_10_v(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                uint32_t k0, uint32_t k1, uint32_t& o0,
                                                uint32_t& o1, uint32_t& o2, uint32_t& o3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0, y2;
    if (r < 2) {
      y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
      y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    } else {
      y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x1, k0, 0x96);
      y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x3, k1, 0x96);
    }
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
  }
  o0 = x0;
  o1 = x1;
  o2 = x2;
  o3 = x3;
}

// Stream S(tag, id, step): Philox blocks with counter {id, step, b, tag} and
// key {seed_lo, seed_hi}, words consumed in order.  The four words of the
// current block are kept in registers as a shift queue (no dynamic indexing).
// V selects the per-lane form of the block (for full waves of distinct ids).
template <bool V = false>
struct StreamT {
  uint32_t k0, k1, id, step, tag, blk;
  uint32_t w0, w1, w2, w3;
  int left;
  __device__ __forceinline__ StreamT(uint64_t seed, uint32_t tag_, uint32_t id_, uint32_t step_)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), id(id_), step(step_), tag(tag_), blk(0),
        w0(0), w1(0), w2(0), w3(0), left(0) {}
  __device__ __forceinline__ uint32_t word() {
    if (left == 0) {
      if constexpr (V)
        philox4x32_10_v(id, step, blk, tag, k0, k1, w0, w1, w2, w3);
      else
        philox4x32_10(id, step, blk, tag, k0, k1, w0, w1, w2, w3);
      blk += 1;
      left = 4;
    }
    const uint32_t r = w0;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    left -= 1;
    return r;
  }
};
using Stream = StreamT<false>;

__device__ __forceinline__ float u01_f32(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ double u01_f64(uint32_t hi, uint32_t lo) {
  return (double)((((uint64_t)hi << 32) | (uint64_t)lo) >> 11) * 0x1p-53;
}

template <class P>
struct Uni;
template <>
struct Uni<float> {
  static constexpr int kWords = 1;
  template <bool V>
  __device__ __forceinline__ static float get(StreamT<V>& s) { return u01_f32(s.word()); }
};
template <>
struct Uni<double> {
  static constexpr int kWords = 2;
  template <bool V>
  __device__ __forceinline__ static double get(StreamT<V>& s) {
    const uint32_t hi = s.word();
    const uint32_t lo = s.word();
    return u01_f64(hi, lo);
  }
};

// ---- 4-wide contiguous loads / stores (16-byte aligned for float, int) ----
__device__ __forceinline__ void ld4(const float* p, float (&o)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  o[0] = t.x;
  o[1] = t.y;
  o[2] = t.z;
  o[3] = t.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&o)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}
__device__ __forceinline__ void ld4(const int32_t* p, int32_t (&o)[4]) {
  const int4 t = *reinterpret_cast<const int4*>(p);
  o[0] = t.x;
  o[1] = t.y;
  o[2] = t.z;
  o[3] = t.w;
}
__device__ __forceinline__ void ld4(const uint32_t* p, uint32_t (&o)[4]) {
  const uint4 t = *reinterpret_cast<const uint4*>(p);
  o[0] = t.x;
  o[1] = t.y;
  o[2] = t.z;
  o[3] = t.w;
}
__device__ __forceinline__ void st4(float* p, const float (&o)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
}
__device__ __forceinline__ void st4(double* p, const double (&o)[4]) {
  *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
  *reinterpret_cast<double2*>(p + 2) = make_double2(o[2], o[3]);
}
__device__ __forceinline__ void st4(int32_t* p, const int32_t (&o)[4]) {
  *reinterpret_cast<int4*>(p) = make_int4(o[0], o[1], o[2], o[3]);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Global-memory pointers: particle arrays are reached through the discharge
// descriptor, so the compiler cannot infer their address space by itself;
// typed pointers give plain global loads and stores instead of flat ones.
template <class T>
using Gp = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ Gp<T>* gptr(T* p) {
  return (Gp<T>*)p;
}
// ---- wave reductions without LDS ------------------------------------------
// DPP row shifts by 1, 2, 4 and 8 leave each 16-lane row's reduction in its
// last lane (whose chain reads only lanes inside the row, so the value other
// lanes get from outside the row never reaches it), and the four row results
// are read out and combined as scalars.  A shuffle would be one LDS permute
// per step.  Results are wave-uniform.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#define HD_ROW_STEP(C)                                                   \
  {                                                                      \
    const uint64_t y = ((uint64_t)dpp_shr<C>(hi) << 32) | dpp_shr<C>(lo); \
    const uint64_t z = (((uint64_t)hi << 32) | lo) + y;                  \
    lo = (uint32_t)z;                                                    \
    hi = (uint32_t)(z >> 32);                                            \
  }
  HD_ROW_STEP(0x111)  // row_shr:1
  HD_ROW_STEP(0x112)  // row_shr:2
  HD_ROW_STEP(0x114)  // row_shr:4
  HD_ROW_STEP(0x118)  // row_shr:8
#undef HD_ROW_STEP
  uint64_t t = 0;
#pragma unroll
  for (int r = 15; r < 64; r += 16)
    t += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, r) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)lo, r);
  return t;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x += dpp_shr<0x111>(x);
  x += dpp_shr<0x112>(x);
  x += dpp_shr<0x114>(x);
  x += dpp_shr<0x118>(x);
  uint32_t t = 0;
#pragma unroll
  for (int r = 15; r < 64; r += 16) t += (uint32_t)__builtin_amdgcn_readlane((int)x, r);
  return t;
}

__device__ __forceinline__ int wave_min_i32(int x) {
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x111, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x112, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x114, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x118, 0xf, 0xf, false));
  int t = __builtin_amdgcn_readlane(x, 15);
  t = min(t, __builtin_amdgcn_readlane(x, 31));
  t = min(t, __builtin_amdgcn_readlane(x, 47));
  return min(t, __builtin_amdgcn_readlane(x, 63));
}

__device__ __forceinline__ int wave_max_i32(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x111, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x112, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x114, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x118, 0xf, 0xf, false));
  int t = __builtin_amdgcn_readlane(x, 15);
  t = max(t, __builtin_amdgcn_readlane(x, 31));
  t = max(t, __builtin_amdgcn_readlane(x, 47));
  return max(t, __builtin_amdgcn_readlane(x, 63));
}

// Vector load / store of global memory, with the nontemporal hint when NT:
// data streamed once per launch then bypass the caches' normal retention,
// which pays when the arrays are far larger than the MALL and costs when
// they would have stayed in it.
template <bool NT, class V>
__device__ __forceinline__ V vld(const Gp<V>* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, class V>
__device__ __forceinline__ void vst(Gp<V>* p, const V& v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Four consecutive elements as 16-byte vectors (two for 8-byte elements).
template <bool NT = false, class T>
__device__ __forceinline__ void gld4(const Gp<T>* p, T (&o)[4]) {
  if constexpr (sizeof(T) == 4) {
    typedef __attribute__((ext_vector_type(4))) T v4;
    const v4 t = vld<NT>(reinterpret_cast<const Gp<v4>*>(p));
    o[0] = t[0];
    o[1] = t[1];
    o[2] = t[2];
    o[3] = t[3];
  } else {
    typedef __attribute__((ext_vector_type(2))) T v2;
    const v2 a = vld<NT>(reinterpret_cast<const Gp<v2>*>(p));
    const v2 b = vld<NT>(reinterpret_cast<const Gp<v2>*>(p + 2));
    o[0] = a[0];
    o[1] = a[1];
    o[2] = b[0];
    o[3] = b[1];
  }
}
template <bool NT = false, class T>
__device__ __forceinline__ void gst4(Gp<T>* p, const T (&o)[4]) {
  if constexpr (sizeof(T) == 4) {
    typedef __attribute__((ext_vector_type(4))) T v4;
    v4 t;
    t[0] = o[0];
    t[1] = o[1];
    t[2] = o[2];
    t[3] = o[3];
    vst<NT>(reinterpret_cast<Gp<v4>*>(p), t);
  } else {
    typedef __attribute__((ext_vector_type(2))) T v2;
    v2 a, b;
    a[0] = o[0];
    a[1] = o[1];
    b[0] = o[2];
    b[1] = o[3];
    vst<NT>(reinterpret_cast<Gp<v2>*>(p), a);
    vst<NT>(reinterpret_cast<Gp<v2>*>(p + 2), b);
  }
}

// Fixed-point cloud-in-cell weight on node c+1: rint(off * 2^32).
template <class P>
__device__ __forceinline__ int64_t cic_w1(P off) {
  return (int64_t)rint(off * (P)4294967296.0);
}

// The same weight as an unsigned value: below 2^32 for FP32 (off < 1 has at
// most 24 significant bits, so rint(off 2^32) <= 2^32 - 2^8) and at most
// 2^32 for FP64.
__device__ __forceinline__ uint64_t cic_w1u_f32(float off) {
  return (uint64_t)(uint32_t)rintf(off * 4294967296.0f);
}
template <class P>
__device__ __forceinline__ uint64_t cic_w1u(P off) {
  if constexpr (sizeof(P) == 4)
    return cic_w1u_f32(off);
  else
    return (uint64_t)rint(off * (P)4294967296.0);
}

// Relaxed device-scope add to a 64-bit word in global memory, issued as a
// global (not flat) atomic: a flat operation counts on both the vector-memory
// and the LDS counters, and while one is outstanding every wait for a load
// has to be a wait for all of them.
__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) {
  __hip_atomic_fetch_add((Gp<unsigned long long>*)p, (unsigned long long)v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- tridiagonal systems --------------------------------------------------

// Partitions of the exact partitioned tridiagonal solve for n unknowns: the
// largest P <= 64 with 2 P^2 <= n, 0 (plain Thomas) below 8 unknowns.
__host__ __device__ inline int tri_partitions(int n) {
  if (n < 8) return 0;
  int P = 1;
  while (P + 1 <= 64 && 2 * (P + 1) * (P + 1) <= n) ++P;
  return P;
}
constexpr int kTriRed = 128;  // max rows of the reduced system (2 x 64 partitions)

// Thomas method for rows [0, n) of a x_{j-1} + b x_j + c x_{j+1} = d, one
// reciprocal of the pivot per row; cp, dp are work arrays.  Rows are read
// and written in full batches of B (LDS latency off the dependent chain).
// Every lane that calls it computes the same values (callers run it on a
// whole wave so that the running values stay in vector registers).
template <int B>
__device__ inline void thomas_serial(int n, const double* a, const double* b, const double* c,
                                     const double* d, double* cp, double* dp, double* x) {
  double rr = 1.0 / b[0];
  double cpp = c[0] * rr, dpp = d[0] * rr;
  cp[0] = cpp;
  dp[0] = dpp;
  int j = 1;
  for (; j + B <= n; j += B) {
    double av[B], bv[B], cv[B], dv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      av[u] = a[j + u];
      bv[u] = b[j + u];
      cv[u] = c[j + u];
      dv[u] = d[j + u];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const double den = bv[u] - av[u] * cpp;
      const double num = dv[u] - av[u] * dpp;
      rr = 1.0 / den;
      cpp = cv[u] * rr;
      dpp = num * rr;
      cv[u] = cpp;
      dv[u] = dpp;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      cp[j + u] = cv[u];
      dp[j + u] = dv[u];
    }
  }
  for (; j < n; ++j) {
    const double aj = a[j];
    const double den = b[j] - aj * cpp;
    const double num = d[j] - aj * dpp;
    rr = 1.0 / den;
    cpp = c[j] * rr;
    dpp = num * rr;
    cp[j] = cpp;
    dp[j] = dpp;
  }
  double xv = dpp;
  x[n - 1] = xv;
  j = n - 2;
  for (; j - B >= -1; j -= B) {
    double cv[B], dv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      cv[u] = cp[j - u];
      dv[u] = dp[j - u];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      xv = dv[u] - cv[u] * xv;
      dv[u] = xv;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) x[j - u] = dv[u];
  }
  for (; j >= 0; --j) {
    xv = dp[j] - cp[j] * xv;
    x[j] = xv;
  }
}

// Exact partitioned solve of a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i,
// i < n, called by every thread of the workgroup (it synchronises inside).
// Partition p = rows [p n / P, (p+1) n / P): lane p of wave 0 eliminates its
// interior rows forward and backward so that each is x_i = D_i - A_i x_s -
// C_i x_e in terms of the partition's first and last unknowns; the first and
// last rows of all partitions form a 2P-row tridiagonal system solved by
// wave 0; then every thread recovers interior unknowns.  a, c, d (LDS) are
// overwritten with A, C, D; b receives the solution x.  red: 7 * kTriRed
// doubles of LDS.  B: rows per batch of the serial sweeps.
template <int B = 4>
__device__ inline void solve_tridiag_block(int n, double* a, double* b, double* c, double* d,
                                           double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // 0, but not known to be: keeps wave-0 serial values in vector registers
  const int zo = (int)(threadIdx.x / blockDim.x);
  const int P = tri_partitions(n);
  double* ra = red;
  double* rb = ra + kTriRed;
  double* rc = rb + kTriRed;
  double* rd = rc + kTriRed;
  double* rx = rd + kTriRed;
  double* rcp = rx + kTriRed;
  double* rdp = rcp + kTriRed;
  __syncthreads();
  if (P == 0) {
    if (tid < 64) {
      if (tid == 0)
        for (int i = 0; i < n; ++i) rd[i] = d[i];
      thomas_serial<B>(n, a + zo, b + zo, c + zo, rd + zo, rcp + zo, rdp + zo, b + zo);
    }
    __syncthreads();
    return;
  }
  if (tid < P) {
    const int p = tid;
    const int s = p * n / P;
    const int e = (p + 1) * n / P - 1;
    // forward over the interior rows s+1 .. e-1
    int i = s + 1;
    double rr = 1.0 / b[i];
    double ap = a[i] * rr, cp = c[i] * rr, dp = d[i] * rr;
    a[i] = ap;
    c[i] = cp;
    d[i] = dp;
    for (i = s + 2; i + B <= e; i += B) {
      double av[B], bv[B], cv[B], dv[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        av[u] = a[i + u];
        bv[u] = b[i + u];
        cv[u] = c[i + u];
        dv[u] = d[i + u];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const double ai = av[u];
        rr = 1.0 / (bv[u] - ai * cp);
        ap = -(ai * ap) * rr;
        cp = cv[u] * rr;
        dp = (dv[u] - ai * dp) * rr;
        av[u] = ap;
        cv[u] = cp;
        dv[u] = dp;
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        a[i + u] = av[u];
        c[i + u] = cv[u];
        d[i + u] = dv[u];
      }
    }
    for (; i <= e - 1; ++i) {
      const double ai = a[i], bi = b[i], ci = c[i], di = d[i];
      rr = 1.0 / (bi - ai * cp);
      ap = -(ai * ap) * rr;
      cp = ci * rr;
      dp = (di - ai * dp) * rr;
      a[i] = ap;
      c[i] = cp;
      d[i] = dp;
    }
    // backward: x_i = D_i - A_i x_s - C_i x_e
    for (i = e - 2; i - B >= s; i -= B) {
      double av[B], cv[B], dv[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        av[u] = a[i - u];
        cv[u] = c[i - u];
        dv[u] = d[i - u];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const double ci = cv[u];
        dp = dv[u] - ci * dp;
        ap = av[u] - ci * ap;
        cp = -(ci * cp);
        dv[u] = dp;
        av[u] = ap;
        cv[u] = cp;
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        d[i - u] = dv[u];
        a[i - u] = av[u];
        c[i - u] = cv[u];
      }
    }
    for (; i >= s + 1; --i) {
      const double ci = c[i];
      dp = d[i] - ci * dp;
      ap = a[i] - ci * ap;
      cp = -(ci * cp);
      d[i] = dp;
      a[i] = ap;
      c[i] = cp;
    }
    // first and last rows with x_{s+1}, x_{e-1} substituted
    ra[2 * p] = a[s];
    rb[2 * p] = b[s] - c[s] * a[s + 1];
    rc[2 * p] = -(c[s] * c[s + 1]);
    rd[2 * p] = d[s] - c[s] * d[s + 1];
    ra[2 * p + 1] = -(a[e] * a[e - 1]);
    rb[2 * p + 1] = b[e] - a[e] * c[e - 1];
    rc[2 * p + 1] = c[e];
    rd[2 * p + 1] = d[e] - a[e] * d[e - 1];
  }
  __syncthreads();
  if (tid < 64)
    thomas_serial<B>(2 * P, ra + zo, rb + zo, rc + zo, rd + zo, rcp + zo, rdp + zo, rx + zo);
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    const int p = ((i + 1) * P - 1) / n;
    const int s = p * n / P;
    const int e = (p + 1) * n / P - 1;
    const double xs = rx[2 * p], xe = rx[2 * p + 1];
    double xi;
    if (i == s)
      xi = xs;
    else if (i == e)
      xi = xe;
    else
      xi = (d[i] - a[i] * xs) - c[i] * xe;
    b[i] = xi;
  }
  __syncthreads();
}

// Relaxed device-scope load (bypasses a possibly stale per-CU cache line).
template <class T>
__device__ __forceinline__ T load_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- isotropic directions and elementary functions ----------------------

// Marsaglia (1972): a uniformly random unit vector (2a sqrt(1-q),
// 2b sqrt(1-q), 1-2q) from a uniform point (a, b) of the unit disk,
// q = a^2 + b^2; (0, 0, 1) after kSphereTries misses.
template <class P, bool V>
__device__ __forceinline__ void sphere(StreamT<V>& s, P& nx, P& ny, P& nz) {
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

// Logarithm and exponential in FP64 whose steps are fixed so that any
// implementation of the same steps rounds identically (the fitted ion
// transport and the swarm's normal deviates use them): ln x by
// binary-exponent reduction of x to m in [sqrt(1/2), sqrt(2)) and the atanh
// series of s = (m - 1)/(m + 1) through s^21; exp y by Cody-Waite reduction
// y = k ln2 + r (ln2 split into a head exact in k ln2 and a tail) and the
// Taylor series of e^r through r^14, scaled by 2^k.
__device__ __forceinline__ double fit_log(double x) {
  int e;
  double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double acc = 1.0 / 21.0;
#pragma unroll
  for (int odd = 19; odd >= 1; odd -= 2) acc = acc * s2 + 1.0 / (double)odd;
  return (double)e * 0.69314718055994530942 + (2.0 * s) * acc;
}

__device__ __forceinline__ double fit_exp(double y) {
  const double k = rint(y * 1.44269504088896340736);
  const double r = (y - k * 6.93147180369123816490e-01) - k * 1.90821492927058770002e-10;
  double fact[15];  // n! for n = 0..14, exact in double
  fact[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= 14; ++n) fact[n] = fact[n - 1] * (double)n;
  double acc = 1.0 / fact[14];
#pragma unroll
  for (int n = 13; n >= 0; --n) acc = acc * r + 1.0 / fact[n];
  return ldexp(acc, (int)k);
}

}  // namespace hd
