// Device modular arithmetic for gfx950 (section 2 of the paper, re-designed for a
// 64-lane wavefront: one residue per lane, no lane splitting).
//
// Word model: T = uint32_t for p < 2^31, T = uint64_t for p < 2^62 (section 2: U of
// n bits, p of at most m bits).  Measured on gfx950, v_mul_lo_u32, v_mul_hi_u32 and
// v_mad_u64_u32 issue at the same rate as v_min_u32, so the fixed-multiplicand
// product costs three multiplies and one subtraction, with no special-form tricks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace nttgpu {

template <typename T>
struct TwPair {
  T w;   // twiddle value, canonical
  T ws;  // floor(w * 2^bits(T) / p): the precomputed multiplicand of Function 8
};

// Global-address-space views of device pointers.  Loads through them are
// global_load (not flat) instructions: the compiler knows they cannot alias LDS, so
// it can issue them early and wait for them separately from LDS traffic.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gcptr<T> gconst(const void* p) {
  return (gcptr<T>)(const T*)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> gmut(void* p) {
  return (gptr<T>)(T*)p;
}
// Value known to be equal in every lane, moved to scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t uni(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
__device__ __forceinline__ const void* uni(const void* x) { return (const void*)uni((uint64_t)(uintptr_t)x); }
__device__ __forceinline__ void* uni(void* x) { return (void*)uni((uint64_t)(uintptr_t)x); }
__device__ __forceinline__ double uni(double x) {
  return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(x)));
}
template <typename T>
__device__ __forceinline__ TwPair<T> uni(const TwPair<T>& t) {
  TwPair<T> r;
  r.w = uni(t.w);
  r.ws = uni(t.ws);
  return r;
}

template <typename T>
__device__ __forceinline__ TwPair<T> ldtw(gcptr<TwPair<T>> p) {
  TwPair<T> t;
  t.w = p->w;
  t.ws = p->ws;
  return t;
}
// The same from an address that is the same in every lane, read through the constant
// address space: a scalar load into scalar registers.  Its wait is on the LDS/scalar
// counter, not on the vector-memory counter, so it does not wait for the operand
// loads issued before it.  Only for tables that no kernel writes.
template <typename T>
using kcptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ TwPair<T> ldtw_s(gcptr<TwPair<T>> p) {
  const kcptr<TwPair<T>> q = (kcptr<TwPair<T>>)(uintptr_t)(const TwPair<T>*)p;
  TwPair<T> t;
  t.w = q->w;
  t.ws = q->ws;
  return t;
}

template <typename T>
struct Arith;

// 32-bit residues, p < 2^31.
template <>
struct Arith<uint32_t> {
  uint32_t p, p2, pinv;  // p, 2p, p^-1 mod 2^32

  // Function 8 (fixed multiplicand y = w, psi = ws) with the final correction left
  // out: for ANY x < 2^32 the result x w - floor(x ws / 2^32) p lies in [0, 2p)
  // (Proposition 4's bound with x not reduced), computed modulo 2^32 since 2p < 2^32.
  // The low word x w + q (2^32 - p) comes from two v_mad_u64_u32 (x w, then + q (2^32
  // - p)): three instructions with the v_mul_hi_u32, one fewer than mul_lo, mul_lo
  // and a subtraction.  Only the low words are used; the carry-out goes to vcc.
  __device__ __forceinline__ uint32_t shoup(uint32_t x, uint32_t w, uint32_t ws) const {
    const uint32_t q = __umulhi(x, ws);
    uint64_t d1, d2;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(d1) : "v"(x), "v"(w) : "vcc");
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(d2) : "v"(q), "s"(0u - p), "v"(d1) : "vcc");
    return (uint32_t)d2;
  }
  // The same for a multiplicand that is the same in every lane of the wave (held in
  // a scalar register; callers pass only values that went through uni()).
  __device__ __forceinline__ uint32_t shoup_u(uint32_t x, uint32_t w, uint32_t ws) const {
    const uint32_t q = __umulhi(x, ws);
    uint64_t d1, d2;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(d1) : "v"(x), "s"(w) : "vcc");
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(d2) : "v"(q), "s"(0u - p), "v"(d1) : "vcc");
    return (uint32_t)d2;
  }
  // Function 2's min trick: [0, 2p) -> [0, p) and [0, 4p) -> [0, 2p).
  __device__ __forceinline__ uint32_t red1(uint32_t x) const { return min(x, x - p); }
  __device__ __forceinline__ uint32_t red2(uint32_t x) const { return min(x, x - p2); }
  // Function 13 (Montgomery, m = n = 32) on a = x y < 2^32 p, with the sign
  // convention chi' = p^-1: returns x y 2^-32 mod p in (0, 2p).
  __device__ __forceinline__ uint32_t mont(uint32_t x, uint32_t y) const {
    uint64_t t = (uint64_t)x * y;
    uint32_t m = (uint32_t)t * pinv;
    return (uint32_t)(t >> 32) - __umulhi(m, p) + p;
  }
};

// 64-bit residues, p < 2^62 (so 4p < 2^64 and every lazy range fits).
template <>
struct Arith<uint64_t> {
  uint64_t p, p2, pinv;

  __device__ __forceinline__ uint64_t shoup(uint64_t x, uint64_t w, uint64_t ws) const {
    uint64_t q = __umul64hi(x, ws);
    return x * w - q * p;
  }
  __device__ __forceinline__ uint64_t shoup_u(uint64_t x, uint64_t w, uint64_t ws) const { return shoup(x, w, ws); }
  __device__ __forceinline__ uint64_t red1(uint64_t x) const {
    uint64_t y = x - p;
    return x < p ? x : y;
  }
  __device__ __forceinline__ uint64_t red2(uint64_t x) const {
    uint64_t y = x - p2;
    return x < p2 ? x : y;
  }
  __device__ __forceinline__ uint64_t mont(uint64_t x, uint64_t y) const {
    uint64_t lo = x * y;
    uint64_t hi = __umul64hi(x, y);
    uint64_t m = lo * pinv;
    return hi - __umul64hi(m, p) + p;
  }
};

// Residues held in doubles (section 3, numeric types: 52 explicit mantissa bits),
// p < 2^50.  Sums of residues below 2^53 are exact, so the integer butterflies' add,
// subtract and compare-and-subtract (Function 17) carry over unchanged.  The product
// is Function 16: h = x y rounded, l = x y - h exactly (one FMA), c = floor(h u) with
// u = 1/p rounded, d = h - c p exactly (one FMA), e = d + l = x y - c p.  For
// x y < 2^50 p (Proposition 13 with 52 mantissa bits), c is floor(x y / p) up to one,
// so e lies in [-p, 2p); one correction gives [0, 2p), the range the integer
// fixed-multiplicand product leaves.  Operands stay below 4p between butterflies when
// p < 2^48 (lazy), so x w < 2^50 p; otherwise the butterflies reduce the multiplicand
// to [0, p) first (mul_operand), so x w < p^2 < 2^50 p for every p < 2^50.
// Explicit _rn operations keep the compiler from contracting h into another FMA.
template <>
struct Arith<double> {
  double p, p2, pinv;  // p, 2p, u = 1/p (rounded to nearest)

  __device__ __forceinline__ double shoup(double x, double w, double) const {
    const double h = __dmul_rn(x, w);
    const double l = __fma_rn(x, w, -h);
    const double c = floor(__dmul_rn(h, pinv));
    const double d = __fma_rn(-c, p, h);
    const double e = __dadd_rn(d, l);
    return e < 0.0 ? __dadd_rn(e, p) : e;
  }
  __device__ __forceinline__ double shoup_u(double x, double w, double ws) const { return shoup(x, w, ws); }
  __device__ __forceinline__ double red1(double x) const { return x >= p ? __dsub_rn(x, p) : x; }
  __device__ __forceinline__ double red2(double x) const { return x >= p2 ? __dsub_rn(x, p2) : x; }
  // Product of two residues: the integer path's Montgomery scale 2^bits / N is 1 / N
  // here, carried by the same table entries.
  __device__ __forceinline__ double mont(double x, double y) const { return shoup(x, y, 0.0); }
};

// ----------------------------------------------------------------------------
// Arithmetic modes: the LAZY template argument of the butterflies and of every kernel
// body above them, read from the plan's constants at run time.
//   kLazy (4p < 2^bits; p < 2^48 for doubles): Harvey-style ranges.
//   kSafe (the 31-bit primes; 2^48 <= p < 2^49 for doubles): every sum is formed from
//         operands reduced to [0, p), values stay below 2p.
//   kBand (doubles, 2^49 <= p < 2^50): as kSafe, and each multiplicand is reduced to
//         [0, p) before its product: Function 16 needs x y < 2^50 p, which x < 2p no
//         longer guarantees.
constexpr int kSafe = 0;
constexpr int kLazy = 1;
constexpr int kBand = 2;

// Calls f with the plan's arithmetic mode as a compile-time constant
// (std::integral_constant<int, mode>); kBand is instantiated for doubles only.
template <typename T, typename F>
__device__ __forceinline__ void with_mode(int mode, F&& f) {
  if (mode == kLazy) {
    f(std::integral_constant<int, kLazy>());
    return;
  }
  if constexpr (std::is_same<T, double>::value) {
    if (mode == kBand) {
      f(std::integral_constant<int, kBand>());
      return;
    }
  }
  f(std::integral_constant<int, kSafe>());
}

// Butterflies.
//
// Forward, Cooley-Tukey form (X, Y) -> (X + w Y, X - w Y):
//   LAZY: X in [0,4p), Y < 2^bits  ->  both outputs in [0,4p)
//   SAFE: X in [0,2p), Y < 2^bits  ->  both outputs in [0,2p)
// UNI: the twiddle is the same in every lane (it went through uni()).
// kBand follows kSafe's ranges with the multiplicand reduced first (mul_operand).
template <int LAZY, typename T>
__device__ __forceinline__ T mul_operand(const Arith<T>& ar, T x) {
  if constexpr (LAZY == kBand) return ar.red1(x);
  else return x;
}

template <int LAZY, bool UNI = false, typename T>
__device__ __forceinline__ void ct_bfly(const Arith<T>& ar, T& X, T& Y, const TwPair<T>& tw) {
  const T Ym = mul_operand<LAZY>(ar, Y);
  T t = UNI ? ar.shoup_u(Ym, tw.w, tw.ws) : ar.shoup(Ym, tw.w, tw.ws);
  if constexpr (LAZY == kLazy) {
    T x = ar.red2(X);
    X = x + t;
    Y = x - t + ar.p2;
  } else {
    T x = ar.red1(X);
    t = ar.red1(t);
    X = x + t;
    Y = x - t + ar.p;
  }
}

// Inverse, Gentleman-Sande form (X, Y) -> (X + Y, (X - Y) w):
//   LAZY: inputs in [0,2p) -> outputs in [0,2p)
//   SAFE: inputs in [0,p)  -> outputs in [0,p)
template <int LAZY, bool UNI = false, typename T>
__device__ __forceinline__ void gs_bfly(const Arith<T>& ar, T& X, T& Y, const TwPair<T>& tw) {
  if constexpr (LAZY == kLazy) {
    T s = ar.red2(X + Y);
    const T d = X - Y + ar.p2;
    Y = UNI ? ar.shoup_u(d, tw.w, tw.ws) : ar.shoup(d, tw.w, tw.ws);
    X = s;
  } else {
    T s = ar.red1(X + Y);
    const T d = mul_operand<LAZY>(ar, X - Y + ar.p);
    Y = ar.red1(UNI ? ar.shoup_u(d, tw.w, tw.ws) : ar.shoup(d, tw.w, tw.ws));
    X = s;
  }
}

// Canonical representative from the range a butterfly left behind.
template <int LAZY, typename T>
__device__ __forceinline__ T canon_from_fwd(const Arith<T>& ar, T x) {
  if constexpr (LAZY == kLazy) return ar.red1(ar.red2(x));
  else return ar.red1(x);
}
template <int LAZY, typename T>
__device__ __forceinline__ T canon_from_inv(const Arith<T>& ar, T x) {
  if constexpr (LAZY == kLazy) return ar.red1(x);
  else return x;
}

}  // namespace nttgpu
