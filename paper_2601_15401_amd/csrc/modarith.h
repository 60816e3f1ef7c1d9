// Device modular arithmetic for moduli m < 2^31 (32-bit residues).
//
// Three forms are used:
//  * Shoup multiplication by a constant w < m with companion
//    w' = floor(w 2^32 / m): y w - floor(y w' / 2^32) m is congruent to y w and
//    lies in [0, 2m) for any 32-bit y.  Used for twiddles and table constants.
//  * Montgomery multiplication of two variables with R = 2^32: for T = a b
//    < m 2^32, REDC(T) = T R^-1 mod m in [0, m).  Used where both operands
//    vary (tensor product); the accumulated R^-1 factors are removed once.
//  * 64-bit multiply-accumulate followed by one reduction of the 64-bit sum
//    (basis conversion, key inner product, rescale sums).
// All values stay below 2^32 because 2m < 2^32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mick {

// [0, 2m) -> [0, m): x - m wraps above x exactly when x < m.
__device__ __forceinline__ uint32_t red1(uint32_t x, uint32_t m) { return min(x, x - m); }

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t m) { return red1(a + b, m); }

__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t m) { return red1(a - b + m, m); }

// Result in [0, 2m), congruent to y * w.
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t y, uint32_t w, uint32_t wsh, uint32_t m) {
  return y * w - __umulhi(y, wsh) * m;
}

__device__ __forceinline__ uint32_t shoup(uint32_t y, uint32_t w, uint32_t wsh, uint32_t m) {
  return red1(shoup_lazy(y, w, wsh, m), m);
}

// a * b * 2^-32 mod m in [0, m), for a * b < m * 2^32.  minv = m^-1 mod 2^32.
// With lo = a b mod 2^32, a b - (lo minv mod 2^32) m is a multiple of 2^32
// whose quotient r = hi - mh lies in (-m, m); min(r + m, r) (unsigned)
// selects r + m exactly when r wrapped below zero.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t m, uint32_t minv) {
  const uint32_t lo = a * b, hi = __umulhi(a, b);
  const uint32_t r = hi - __umulhi(lo * minv, m);
  return min(r + m, r);
}

// Montgomery reduction of T < m 2^32: T 2^-32 mod m in [0, m).  As in
// mont_mul, the quotient lies in (-m, m) and min(r + m, r) corrects it.
__device__ __forceinline__ uint32_t redc(uint64_t T, uint32_t m, uint32_t minv) {
  const uint32_t lo = (uint32_t)T, hi = (uint32_t)(T >> 32);
  const uint32_t r = hi - __umulhi(lo * minv, m);
  return min(r + m, r);
}

// Montgomery reduction of T < 2m 2^32: T 2^-32 mod m in [0, m).  The
// quotient hi - mh lies in (-m, 2m) here; r + m would overflow 32 bits for
// m near 2^31, so the negative case is detected by comparing hi and mh.
__device__ __forceinline__ uint32_t redc_2m(uint64_t T, uint32_t m, uint32_t minv) {
  const uint32_t lo = (uint32_t)T, hi = (uint32_t)(T >> 32);
  const uint32_t mh = __umulhi(lo * minv, m);
  const uint32_t r = hi - mh;
  return hi < mh ? r + m : red1(r, m);
}

// Montgomery reduction of T < 2m 2^32 left lazy: T 2^-32 mod m as a value in
// (0, 3m), below 2^32 for m < 2^30.  With u = lo m^-1 mod 2^32 the low word
// of u m equals lo, so (T - u m) / 2^32 = hi - mh lies in (-m, 2m).
__device__ __forceinline__ uint32_t redc_lazy(uint64_t T, uint32_t m, uint32_t minv) {
  const uint32_t lo = (uint32_t)T, hi = (uint32_t)(T >> 32);
  return hi + m - __umulhi(lo * minv, m);
}

// Four independent (hi, lo) += a * b on 96-bit accumulators: each is one
// 32x32+64-bit multiply-add whose carry-out goes to a lane mask and one add
// of that carry into hi.  The four carries take four lane-mask pairs, so
// the multiply-adds issue back to back and each carry add comes four
// instructions after its multiply-add.  (One product per statement gave
// every statement the same scalar pair, chaining all products of a tile
// through it with a wait state between statements.)
__device__ __forceinline__ void mac96x4(uint64_t& l0, uint32_t& h0, uint64_t& l1, uint32_t& h1, uint64_t& l2,
                                        uint32_t& h2, uint64_t& l3, uint32_t& h3, uint32_t a0, uint32_t b0,
                                        uint32_t a1, uint32_t b1, uint32_t a2, uint32_t b2, uint32_t a3,
                                        uint32_t b3) {
  uint64_t c0, c1, c2, c3;
  asm("v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
      "v_mad_u64_u32 %2, %9, %14, %15, %2\n\t"
      "v_mad_u64_u32 %4, %10, %16, %17, %4\n\t"
      "v_mad_u64_u32 %6, %11, %18, %19, %6\n\t"
      "v_addc_co_u32_e64 %1, %8, 0, %1, %8\n\t"
      "v_addc_co_u32_e64 %3, %9, 0, %3, %9\n\t"
      "v_addc_co_u32_e64 %5, %10, 0, %5, %10\n\t"
      "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
      : "+v"(l0), "+v"(h0), "+v"(l1), "+v"(h1), "+v"(l2), "+v"(h2), "+v"(l3), "+v"(h3), "=&s"(c0), "=&s"(c1),
        "=&s"(c2), "=&s"(c3)
      : "v"(a0), "v"(b0), "v"(a1), "v"(b1), "v"(a2), "v"(b2), "v"(a3), "v"(b3));
}

// lo32(a b + c d): two chained 32 x 32 + 64-bit multiply-adds, the first
// product's 64-bit result feeding the second as its addend; only the low
// word is kept.  The low word of a 64-bit sum depends only on the low words
// of its terms, so this is (a b + c d) mod 2^32 exactly.  One instruction
// per product, where a 32-bit multiply and a separate add would take two
// for the second.  d is uniform across the wave (a modulus or its negation).
__device__ __forceinline__ uint32_t mad2_lo(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  uint64_t p, cy;  // cy: carry-out lane mask, unused
  asm("v_mad_u64_u32 %0, %1, %2, %3, 0\n\t"
      "v_mad_u64_u32 %0, %1, %4, %5, %0"
      : "=&v"(p), "=&s"(cy)
      : "v"(a), "v"(b), "v"(c), "s"(d));
  return (uint32_t)p;
}

// lo32(a b + c d + e) with d and e uniform: as mad2_lo, with e as the first
// multiply-add's 64-bit addend.
__device__ __forceinline__ uint32_t mad2_lo_add(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
  uint64_t p, cy;  // cy: carry-out lane mask, unused
  const uint64_t e64 = e;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %6\n\t"
      "v_mad_u64_u32 %0, %1, %4, %5, %0"
      : "=&v"(p), "=&s"(cy)
      : "v"(a), "v"(b), "v"(c), "s"(d), "s"(e64));
  return (uint32_t)p;
}

// Shoup product in [0, 2m) with negm = 2^32 - m: y w + floor(y w' / 2^32)
// (2^32 - m) mod 2^32 = y w - floor(y w' / 2^32) m, the value of shoup_lazy
// in three instructions.
__device__ __forceinline__ uint32_t shoup_lazy_neg(uint32_t y, uint32_t w, uint32_t wsh, uint32_t negm) {
  return mad2_lo(y, w, __umulhi(y, wsh), negm);
}

// Per-modulus constants for reducing a full 64-bit value.
struct Red64 {
  uint32_t m;
  uint32_t r32;    // 2^32 mod m
  uint32_t r32sh;  // floor(r32 2^32 / m)
  uint32_t onesh;  // floor(2^32 / m)
};

// x mod m for any 64-bit x: x = hi 2^32 + lo, both halves reduced by Shoup.
__device__ __forceinline__ uint32_t reduce64(uint64_t x, const Red64& c) {
  uint32_t hi = (uint32_t)(x >> 32), lo = (uint32_t)x;
  uint32_t a = shoup(hi, c.r32, c.r32sh, c.m);
  uint32_t b = red1(lo - __umulhi(lo, c.onesh) * c.m, c.m);
  return red1(a + b, c.m);
}

}  // namespace mick
