// Exact 32-bit-word modular arithmetic for gfx950 (moduli q < 2^30).
//
// On gfx950 v_mul_lo_u32 / v_mul_hi_u32 / v_mad_u64_u32 issue at close to
// full VALU rate, so the products below are plain 32-bit integer multiplies.
// Lazy ranges: values may live in [0, 2q) or [0, 4q) between steps; 4q < 2^32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

// x in [0, 2m) -> [0, m): if x >= m then x - m wraps below x, else it wraps above.
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) { return min(x, x - m); }

// Shoup product y * w mod q, result in [0, 2q), for any y < 2^32, w < q and
// wp = floor(w * 2^32 / q).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t y, uint32_t w, uint32_t wp, uint32_t q) {
  const uint32_t qt = __umulhi(y, wp);
  return y * w - qt * q;
}

// Cooley-Tukey butterfly (x, y) <- (x + w y, x - w y), Harvey's lazy form:
// inputs and outputs in [0, 4q).
__device__ __forceinline__ void bfly_ct(uint32_t& x, uint32_t& y, uint32_t w, uint32_t wp,
                                        uint32_t q, uint32_t q2) {
  const uint32_t xx = csub(x, q2);
  const uint32_t t = mul_shoup(y, w, wp, q);
  x = xx + t;
  y = xx + q2 - t;
}

// Gentleman-Sande butterfly (x, y) <- (x + y, w (x - y)): inputs and outputs in [0, 2q).
__device__ __forceinline__ void bfly_gs(uint32_t& x, uint32_t& y, uint32_t w, uint32_t wp,
                                        uint32_t q, uint32_t q2) {
  const uint32_t s = csub(x + y, q2);
  const uint32_t d = x + q2 - y;
  x = s;
  y = mul_shoup(d, w, wp, q);
}

// Exact x mod q for any 64-bit x, q < 2^30, mu = floor(2^64 / q) split as
// (mu_hi, mu_lo).  The Barrett quotient floor(x mu / 2^64) is either Q or
// Q - 1 (Q = floor(x / q)), so x - qh q lies in [0, 2q) and is computed in
// 32 bits; only the low word of qh is needed, which is why the 64-bit
// partial sum may wrap.
__device__ __forceinline__ uint32_t reduce64(uint64_t x, uint32_t q, uint32_t mu_hi,
                                             uint32_t mu_lo) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  uint64_t s = (uint64_t)x1 * mu_lo + __umulhi(x0, mu_lo);
  s += (uint64_t)x0 * mu_hi;
  const uint32_t qh = x1 * mu_hi + (uint32_t)(s >> 32);
  return csub(x0 - qh * q, q);
}

// x mod q for x < 2^32 with mu32 = floor(2^32 / q): remainder in [0, 2q), one correction.
__device__ __forceinline__ uint32_t reduce32(uint32_t x, uint32_t q, uint32_t mu32) {
  return csub(x - __umulhi(x, mu32) * q, q);
}

// Load through the constant address space: for a work-group-uniform address
// this becomes a scalar (s_load) read.  Only for tables that no kernel writes.
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized tables only");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  cword* s = (cword*)p;
  T v;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = s[i];
  return v;
}


// Global-memory accesses through the global address space.  Data pointers
// that come from job tables are generic (flat) pointers, which the compiler
// must assume may alias LDS: each flat load would then wait for the LDS
// stores before it.  Accessing them as global memory lets loads be issued
// back to back.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld4(const uint32_t* p) {
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
// Streaming load: the non-temporal hint marks the line for early eviction
// (data read once, such as evaluation-key words).
__device__ __forceinline__ uint4 ld4nt(const uint32_t* p) {
  const u32x4 v = __builtin_nontemporal_load((const __attribute__((address_space(1))) u32x4*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(uint32_t* p, uint4 v) {
  const u32x4 w = {v.x, v.y, v.z, v.w};
  *(__attribute__((address_space(1))) u32x4*)p = w;
}
__device__ __forceinline__ uint32_t ld1(const uint32_t* p) {
  return *(const __attribute__((address_space(1))) uint32_t*)p;
}
__device__ __forceinline__ void st1(uint32_t* p, uint32_t v) {
  *(__attribute__((address_space(1))) uint32_t*)p = v;
}

}  // namespace ckks
