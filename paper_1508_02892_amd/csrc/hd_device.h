// Device-side helpers: the counter-based Philox4x32-10 stream, uniform maps,
// vector memory access and wave-level utilities for gfx950 (wave64).
#pragma once

#include "hd_internal.h"

namespace hd {

enum : uint32_t { kTagElectron = 0, kTagLoad = 1, kTagEmission = 2 };

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

// Stream S(tag, id, step): Philox blocks with counter {id, step, b, tag} and
// key {seed_lo, seed_hi}, words consumed in order.  The four words of the
// current block are kept in registers as a shift queue (no dynamic indexing).
struct Stream {
  uint32_t k0, k1, id, step, tag, blk;
  uint32_t w0, w1, w2, w3;
  int left;
  __device__ __forceinline__ Stream(uint64_t seed, uint32_t tag_, uint32_t id_, uint32_t step_)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), id(id_), step(step_), tag(tag_), blk(0),
        w0(0), w1(0), w2(0), w3(0), left(0) {}
  __device__ __forceinline__ uint32_t word() {
    if (left == 0) {
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

__device__ __forceinline__ float u01_f32(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ double u01_f64(uint32_t hi, uint32_t lo) {
  return (double)((((uint64_t)hi << 32) | (uint64_t)lo) >> 11) * 0x1p-53;
}

template <class P>
struct Uni;
template <>
struct Uni<float> {
  static constexpr int kWords = 1;
  __device__ __forceinline__ static float get(Stream& s) { return u01_f32(s.word()); }
};
template <>
struct Uni<double> {
  static constexpr int kWords = 2;
  __device__ __forceinline__ static double get(Stream& s) {
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

// Fixed-point cloud-in-cell weight on node c+1: rint(off * 2^32).
template <class P>
__device__ __forceinline__ int64_t cic_w1(P off) {
  return (int64_t)rint(off * (P)4294967296.0);
}

__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

// Relaxed device-scope load (bypasses a possibly stale per-CU cache line).
template <class T>
__device__ __forceinline__ T load_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace hd
