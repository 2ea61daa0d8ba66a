// Device modular arithmetic for gfx950.
//
// The paper (Section 3.1) reviews the ways to multiply modulo a word-size
// p without a divide (floating-point quotient, Barrett, Montgomery,
// Moller-Granlund) and builds on the FP64 FMA product of van der Hoeven,
// Lecerf and Quintin (Alg. 2), which needs p <= 50 bits.  On gfx950 the
// 32-bit integer multiplies (mul_lo, mul_hi, mad_u64_u32) issue at the
// same rate as FP64 FMA, so an integer product on 32-bit limbs is exact for
// any p < 2^63 and cheaper than Alg. 2 even for 31-bit p.
//
// The evaluation kernel multiplies every running value by a multiplier
// that stays fixed for a whole run (m_i, or Gamma_i = m_i^C), which is the
// setting of Shoup's precomputed-quotient product (V. Shoup, NTL; also
// Harvey, "Faster arithmetic for number-theoretic transforms", 2014):
// with w' = floor(w * 2^64 / p), q = floor(x * w' / 2^64) and
// r = x*w - q*p (mod 2^64) lies in [0, 2p) for every x < 2^64.  So the
// running values may stay in [0, 2p) ("lazy") and are only made canonical
// when a coefficient is output.
//
// w' itself is obtained without a 128-by-64 division: r = w*2^64 mod p is a
// Shoup product of w by the fixed constant (2^64 mod p), and since
// w*2^64 - r is divisible by p and the quotient is below 2^64,
// w' = (-r) * p^{-1} mod 2^64 (exact division by multiplication with the
// inverse of p modulo 2^64; Jebelean 1993).
//
// The integer code is plain 32/64-bit C, for which hipcc selects
// v_mad_u64_u32 / v_mul_hi_u32 / v_mul_lo_u32, except short
// arithmetic-only sequences written in assembly (the high word and the
// remainder of the 64-bit product, and the per-thread sum of 64-bit
// values), whose C forms the compiler expands into longer code.  The paper's FP64 product (Alg. 2,
// p < 2^50) is kept as a second policy so that both can be measured on the
// same kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace peval {

// Per-modulus constants, computed on the host.
struct Mod64 {
  uint64_t p;     // odd modulus, p < 2^63
  uint64_t pinv;  // p^{-1} mod 2^64
  uint64_t R;     // 2^64 mod p
  uint64_t Rq;    // floor(R * 2^64 / p)
  uint64_t oneq;  // floor(2^64 / p)       (Shoup quotient of w = 1)
};

struct Mod32 {
  uint32_t p;     // odd modulus, p < 2^31
  uint32_t pinv;  // p^{-1} mod 2^32
  uint32_t R;     // 2^32 mod p
  uint32_t Rq;    // floor(R * 2^32 / p)
  uint32_t oneq;  // floor(2^32 / p)
};

__device__ __forceinline__ uint64_t mad_wide(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * b + c;
}

// floor(a * b / 2^64) from four 32x32 products.  With t = a0 b1 + hi(a0 b0)
// (below 2^64), u = a1 b0 + t is at most 65 bits and floor(u / 2^32) =
// hi(a1 b0 + lo(t)) + hi(t), so the high word is a1 b1 + floor(u / 2^32).
// One multiply-add forms u modulo 2^64 and writes its 65th bit to the carry
// mask it always produces; the addend (hi(u), carry) of the last
// multiply-add is then one copy and one select.  That is 6 instructions
// against 8 for adding hi(t) and hi(u) separately, each of which needs an
// (x, 0) register pair built by a copy.  Assembly (arithmetic only) keeps
// the carry mask, with the two wait states gfx950 needs between a vector
// write of a mask and its read, which the compiler does not see.
__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t t = mad_wide(a0, b1, __umulhi(a0, b0));
  uint64_t u, carry, unused, q;
  uint32_t cbit;
  asm("v_mad_u64_u32 %0, %1, %3, %4, %5\n\t"   // u = a1 b0 + t (mod 2^64), carry = bit 64
      "s_nop 1\n\t"
      "v_cndmask_b32 %2, 0, 1, %1"               // cbit = carry
      : "=&v"(u), "=&s"(carry), "=v"(cbit) : "v"(a1), "v"(b0), "v"(t));
  const uint64_t s = ((uint64_t)cbit << 32) | (uint32_t)(u >> 32);  // floor(u / 2^32)
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(q), "=s"(unused) : "v"(a1), "v"(b1), "v"(s));
  return q;
}

// ---------------------------------------------------------------------------
// 64-bit residues (3 <= p < 2^63)
// ---------------------------------------------------------------------------

// x * w mod p in [0, 2p), for any x < 2^64, w < p, wq = floor(w 2^64 / p).
// q = floor(x wq / 2^64) as in mulhi64, and the remainder x w - q p
// (mod 2^64) formed as x w + q n with n = 2^64 - p, by multiply-adds only:
// the four 32x32 cross products that reach the high word are accumulated in
// one 64-bit pair (only its low 32 bits count), shifted up by 32 and used as
// the addend of x0 w0, then q0 n0 is added; every step wraps modulo 2^64,
// which is what is wanted.  The remainder takes 7 instructions, written
// into x's own registers (10 for the two 64-bit low products and the
// subtraction); the two cross products that do not involve q fill the two
// wait states between the carry mask of the quotient's middle multiply-add
// and its read.  Written in assembly (arithmetic only) because the compiler
// turns the same steps in C back into 64x64-bit multiply expansions.  The
// words of 2^64 - p are read from scalar registers (p is the same for every
// lane of a wave in every caller; each multiply-add reads one of them), so
// they are not copied into vector registers on every product.
__device__ __forceinline__ uint64_t shoup_mul(uint64_t x, uint64_t w, uint64_t wq, uint64_t p) {
  const uint64_t n = 0 - p;
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32), w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32);
  const uint32_t y0 = (uint32_t)wq, y1 = (uint32_t)(wq >> 32), n0 = (uint32_t)n, n1 = (uint32_t)(n >> 32);
  const uint64_t t = mad_wide(x0, y1, __umulhi(x0, y0));
  uint64_t u, h, carry, unused, q;
  uint32_t cbit;
  asm("v_mad_u64_u32 %[u], %[c], %[x1], %[y0], %[t]\n\t"  // u = x1 y0 + t (mod 2^64), c = bit 64
      "v_mad_u64_u32 %[h], %[z], %[x1], %[w0], 0\n\t"     // h = x1 w0
      "v_mad_u64_u32 %[h], %[z], %[x0], %[w1], %[h]\n\t"  // h += x0 w1
      "v_cndmask_b32 %[cb], 0, 1, %[c]"                     // cbit = c
      : [u] "=&v"(u), [h] "=&v"(h), [c] "=&s"(carry), [cb] "=v"(cbit), [z] "=&s"(unused)
      : [x1] "v"(x1), [y0] "v"(y0), [t] "v"(t), [w0] "v"(w0), [x0] "v"(x0), [w1] "v"(w1));
  const uint64_t s = ((uint64_t)cbit << 32) | (uint32_t)(u >> 32);  // floor((x1 y0 + t) / 2^32)
  asm("v_mad_u64_u32 %[q], %[z], %[x1], %[y1], %[s]"                // q = x1 y1 + s
      : [q] "=v"(q), [z] "=s"(unused) : [x1] "v"(x1), [y1] "v"(y1), [s] "v"(s));
  const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
  asm("v_mad_u64_u32 %[h], %[z], %[q1], %[n0], %[h]\n\t"  // h += q1 n0
      "v_mad_u64_u32 %[h], %[z], %[q0], %[n1], %[h]\n\t"  // h += q0 n1
      "v_lshlrev_b64 %[h], 32, %[h]\n\t"                  // h <<= 32
      "v_mad_u64_u32 %[x], %[z], %[x0], %[w0], %[h]\n\t"  // x = x0 w0 + h
      "v_mad_u64_u32 %[x], %[z], %[q0], %[n0], %[x]"        // x += q0 n0
      : [x] "+v"(x), [h] "+v"(h), [z] "=&s"(unused)
      : [q1] "v"(q1), [n0] "s"(n0), [q0] "v"(q0), [n1] "s"(n1), [x0] "v"(x0), [w0] "v"(w0));
  return x;
}

__device__ __forceinline__ uint64_t canon(uint64_t x, uint64_t p) {  // [0, 2p) -> [0, p)
  return x >= p ? x - p : x;
}

// Shoup quotient floor(w 2^64 / p) of a canonical w.
__device__ __forceinline__ uint64_t shoup_quot(uint64_t w, const Mod64 &m) {
  uint64_t r = canon(shoup_mul(w, m.R, m.Rq, m.p), m.p);  // w 2^64 mod p
  return (0 - r) * m.pinv;
}

// General product of canonical x, y; canonical result.
__device__ __forceinline__ uint64_t mul_mod(uint64_t x, uint64_t y, const Mod64 &m) {
  return canon(shoup_mul(x, y, shoup_quot(y, m), m.p), m.p);
}

__device__ __forceinline__ uint64_t add_mod(uint64_t x, uint64_t y, uint64_t p) {  // canonical in/out
  uint64_t s = x + y;  // < 2p < 2^64
  return s >= p ? s - p : s;
}

// Any x < 2^64 -> canonical.
__device__ __forceinline__ uint64_t reduce64(uint64_t x, const Mod64 &m) {
  return canon(shoup_mul(x, 1, m.oneq, m.p), m.p);
}

// hi * 2^64 + lo -> canonical (hi < 2^32).
__device__ __forceinline__ uint64_t reduce96(uint64_t lo, uint32_t hi, const Mod64 &m) {
  uint64_t a = canon(shoup_mul(hi, m.R, m.Rq, m.p), m.p);
  return add_mod(a, reduce64(lo, m), m.p);
}

// hi * 2^64 + lo -> some 64-bit word congruent to it mod p (hi < 2^32), with
// one product where reduce96 takes two: y = hi R lazily (R = 2^64 mod p,
// y < 2p), then lo + y; if that sum carries out of 64 bits, the carry's 2^64
// is replaced by R.  The wrapped sum is below y < 2p, and R = 2^64 - k p with
// k = floor(2^64 / p) >= 2 for p < 2^63, so adding R cannot carry again.
__device__ __forceinline__ uint64_t fold96(uint64_t lo, uint32_t hi, const Mod64 &m) {
  const uint64_t y = shoup_mul(hi, m.R, m.Rq, m.p);
  const uint64_t s = lo + y;
  return s < y ? s + m.R : s;
}

// base^e mod p by square-and-multiply, canonical base, e >= 0.
__device__ __forceinline__ uint64_t pow_mod(uint64_t base, uint64_t e, const Mod64 &m) {
  uint64_t r = 1 % m.p;
  while (e) {
    if (e & 1) r = mul_mod(r, base, m);
    e >>= 1;
    if (e) base = mul_mod(base, base, m);
  }
  return r;
}

// ---------------------------------------------------------------------------
// 32-bit residues (3 <= p < 2^31)
// ---------------------------------------------------------------------------

// x * w mod p in [0, 2p) for p < 2^31, any x < 2^32, wq = floor(w 2^32 / p):
// the remainder x w - q p (mod 2^32) as the low word of x w + q (2^32 - p),
// two multiply-adds (against two multiplies and a subtraction); each in an
// assembly statement of its own (arithmetic only), so that the result may
// take the registers of x and the compiler cannot fold them back into
// 32-bit multiplies.
__device__ __forceinline__ uint32_t shoup_mul(uint32_t x, uint32_t w, uint32_t wq, uint32_t p) {
  const uint32_t q = __umulhi(x, wq);
  const uint32_t n = 0u - p;
  uint64_t t, r, carry;  // carry: the unused carry-out mask of each v_mad_u64_u32
  asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(t), "=s"(carry) : "v"(x), "v"(w));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(q), "v"(n), "v"(t));
  return (uint32_t)r;
}

__device__ __forceinline__ uint32_t canon(uint32_t x, uint32_t p) {
  return x >= p ? x - p : x;
}

__device__ __forceinline__ uint32_t shoup_quot(uint32_t w, const Mod32 &m) {
  uint32_t r = canon(shoup_mul(w, m.R, m.Rq, m.p), m.p);
  return (0u - r) * m.pinv;
}

__device__ __forceinline__ uint32_t mul_mod(uint32_t x, uint32_t y, const Mod32 &m) {
  return canon(shoup_mul(x, y, shoup_quot(y, m), m.p), m.p);
}

__device__ __forceinline__ uint32_t add_mod(uint32_t x, uint32_t y, uint32_t p) {
  uint32_t s = x + y;  // < 2p < 2^32
  return s >= p ? s - p : s;
}

__device__ __forceinline__ uint32_t reduce32(uint32_t x, const Mod32 &m) {
  return canon(shoup_mul(x, 1u, m.oneq, m.p), m.p);
}

// hi * 2^32 + lo -> canonical.
__device__ __forceinline__ uint32_t reduce64(uint64_t v, const Mod32 &m) {
  uint32_t a = canon(shoup_mul((uint32_t)(v >> 32), m.R, m.Rq, m.p), m.p);
  return add_mod(a, reduce32((uint32_t)v, m), m.p);
}

__device__ __forceinline__ uint32_t pow_mod(uint32_t base, uint64_t e, const Mod32 &m) {
  uint32_t r = 1u % m.p;
  while (e) {
    if (e & 1) r = mul_mod(r, base, m);
    e >>= 1;
    if (e) base = mul_mod(base, base, m);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Width policies used to template the kernels
// ---------------------------------------------------------------------------

// 64-bit residues; lazy sums of up to 2^32 values below 2^64 in 96 bits.
struct W64 {
  using T = uint64_t;
  using PT = uint64_t;  // partial sums and output
  using M = Mod64;
  struct Acc {
    uint32_t w0, w1, w2;
  };
  static constexpr int bytes = 8;
  __device__ static __forceinline__ Acc zero() { return Acc{0u, 0u, 0u}; }
  __device__ static __forceinline__ void add(Acc &a, T x) {
    unsigned c0, c1;
    a.w0 = __builtin_addc(a.w0, (uint32_t)x, 0u, &c0);
    a.w1 = __builtin_addc(a.w1, (uint32_t)(x >> 32), c0, &c1);
    a.w2 += c1;
  }
  __device__ static __forceinline__ void add(Acc &a, const Acc &b) {
    unsigned c0, c1;
    a.w0 = __builtin_addc(a.w0, b.w0, 0u, &c0);
    a.w1 = __builtin_addc(a.w1, b.w1, c0, &c1);
    a.w2 = a.w2 + b.w2 + c1;
  }
  __device__ static __forceinline__ T reduce(const Acc &a, const M &m) {
    return reduce96(((uint64_t)a.w1 << 32) | a.w0, a.w2, m);
  }
  // A partial coefficient (segment sum) as any 64-bit representative: the
  // combine makes it canonical after the walk, where the VALUs are idle.
  __device__ static __forceinline__ T reduce_partial(const Acc &a, const M &m) {
    return fold96(((uint64_t)a.w1 << 32) | a.w0, a.w2, m);
  }
  __device__ static __forceinline__ T canon_partial(T v, const M &m) { return reduce64(v, m); }
  // A thread's sum over its terms: the low and high 32-bit halves of the
  // values are summed separately in 64 bits (value = lo + hi 2^32), one
  // multiply-add by 1 each and no carry chain; exact for up to 2^32 values.
  // It becomes a 96-bit Acc once per row (stage).
  struct Sum {
    uint64_t lo, hi;
  };
  __device__ static __forceinline__ Sum sum_zero() { return Sum{0, 0}; }
  // a sum started from its first value: each half by one multiply-add by 1
  // (the zero-extended half in a fresh pair, no clearing of the pair first)
  __device__ static __forceinline__ Sum sum_first(T x) {
    Sum s;
    uint64_t carry;
    asm("v_mad_u64_u32 %0, %2, %3, 1, 0\n\t"
        "v_mad_u64_u32 %1, %2, %4, 1, 0"
        : "=&v"(s.lo), "=&v"(s.hi), "=&s"(carry)
        : "v"((uint32_t)x), "v"((uint32_t)(x >> 32)));
    return s;
  }
  __device__ static __forceinline__ void sum_add(Sum &s, T x) {
    uint64_t carry;
    asm("v_mad_u64_u32 %0, %2, %3, 1, %0\n\t"
        "v_mad_u64_u32 %1, %2, %4, 1, %1"
        : "+v"(s.lo), "+v"(s.hi), "=&s"(carry)
        : "v"((uint32_t)x), "v"((uint32_t)(x >> 32)));
  }
  // value = lo + hi 2^32 = w0 + w1 2^32 + w2 2^64: the middle word with one
  // add-with-carry, the carry into the top word with a second
  __device__ static __forceinline__ Acc stage(const Sum &s, const M &) {
    unsigned c;
    const uint32_t w1 = __builtin_addc((uint32_t)(s.lo >> 32), (uint32_t)s.hi, 0u, &c);
    return Acc{(uint32_t)s.lo, w1, (uint32_t)(s.hi >> 32) + c};
  }
  __device__ static __forceinline__ void add_walk(Acc &a, const Acc &b, const M &) { add(a, b); }
  __device__ static __forceinline__ T mul_lazy(T x, T w, T wq, const M &m) {
    return shoup_mul(x, w, wq, m.p);
  }
};

// 32-bit residues; lazy sums in 64 bits.
struct W32 {
  using T = uint32_t;
  using PT = uint32_t;
  using M = Mod32;
  struct Acc {
    uint64_t v;
  };
  static constexpr int bytes = 4;
  __device__ static __forceinline__ Acc zero() { return Acc{0}; }
  __device__ static __forceinline__ void add(Acc &a, T x) { a.v += x; }
  __device__ static __forceinline__ void add(Acc &a, const Acc &b) { a.v += b.v; }
  __device__ static __forceinline__ T reduce(const Acc &a, const M &m) { return reduce64(a.v, m); }
  __device__ static __forceinline__ T reduce_partial(const Acc &a, const M &m) { return reduce64(a.v, m); }
  __device__ static __forceinline__ T canon_partial(T v, const M &) { return v; }
  using Sum = Acc;  // a thread's sum over its terms
  __device__ static __forceinline__ Sum sum_zero() { return zero(); }
  __device__ static __forceinline__ Sum sum_first(T x) {
    Sum s;
    uint64_t carry;
    asm("v_mad_u64_u32 %0, %1, %2, 1, 0" : "=v"(s.v), "=s"(carry) : "v"(x));
    return s;
  }
  // one multiply-add by 1 into the 64-bit sum (no carry chain)
  __device__ static __forceinline__ void sum_add(Sum &s, T x) {
    uint64_t carry;
    asm("v_mad_u64_u32 %0, %1, %2, 1, %0" : "+v"(s.v), "=s"(carry) : "v"(x));
  }
  __device__ static __forceinline__ Acc stage(const Acc &a, const M &) { return a; }
  __device__ static __forceinline__ void add_walk(Acc &a, const Acc &b, const M &) { add(a, b); }
  __device__ static __forceinline__ T mul_lazy(T x, T w, T wq, const M &m) {
    return shoup_mul(x, w, wq, m.p);
  }
};

// ---------------------------------------------------------------------------
// Pseudo-Mersenne moduli p = 2^k - c with small c (both 2^31 - 1 and
// 2^63 - 25 have this form): the full product x w = H 2^k + L is folded
// twice with 2^k = c (mod p), r = L + c H, which needs no precomputed
// quotient.  Kept as a third product so that it can be measured against
// Shoup's on the same kernel; the running value stays lazy in [0, 2p).
// ---------------------------------------------------------------------------
struct ModPM64 {
  uint64_t p;  // 2^63 - c
  uint64_t c;  // 1 <= c < 2^20
  Mod64 m;     // for the sums and the output reduction
};

__device__ __forceinline__ uint64_t pm63_mul_lazy(uint64_t x, uint64_t w, uint64_t c) {
  const uint64_t M63 = 0x7fffffffffffffffull;
  const uint64_t lo = x * w, hi = mulhi64(x, w);  // x < 2^64, w < 2^63: product < 2^127
  const uint64_t H = (hi << 1) | (lo >> 63);      // product >> 63, < 2^64
  const uint64_t L = lo & M63;
  // r1 = L + c H < 2^63 + 2^84, as (r1h, r1l)
  const uint64_t chl = c * H, chh = mulhi64(c, H);
  const uint64_t r1l = L + chl;
  const uint64_t r1h = chh + (r1l < L ? 1u : 0u);
  // second fold: r1 >> 63 < 2^22, so the result is below 2^63 + 2^42 < 2p
  const uint64_t h2 = (r1h << 1) | (r1l >> 63);
  return (r1l & M63) + c * h2;
}

struct W64PM {
  using T = uint64_t;
  using PT = uint64_t;
  using M = ModPM64;
  using Acc = W64::Acc;
  static constexpr int bytes = 8;
  __device__ static __forceinline__ Acc zero() { return W64::zero(); }
  __device__ static __forceinline__ void add(Acc &a, T x) { W64::add(a, x); }
  __device__ static __forceinline__ T reduce(const Acc &a, const M &m) { return W64::reduce(a, m.m); }
  __device__ static __forceinline__ T reduce_partial(const Acc &a, const M &m) { return W64::reduce_partial(a, m.m); }
  using Sum = W64::Sum;
  __device__ static __forceinline__ Sum sum_zero() { return W64::sum_zero(); }
  __device__ static __forceinline__ Sum sum_first(T x) { return W64::sum_first(x); }
  __device__ static __forceinline__ void sum_add(Sum &s, T x) { W64::sum_add(s, x); }
  __device__ static __forceinline__ Acc stage(const Sum &s, const M &m) { return W64::stage(s, m.m); }
  __device__ static __forceinline__ void add_walk(Acc &a, const Acc &b, const M &) { W64::add(a, b); }
  __device__ static __forceinline__ T mul_lazy(T x, T w, T, const M &m) { return pm63_mul_lazy(x, w, m.c); }
};

struct ModPM32 {
  uint32_t p;  // 2^31 - c
  uint32_t c;  // 1 <= c < 2^12
  Mod32 m;
};

__device__ __forceinline__ uint32_t pm31_mul_lazy(uint32_t x, uint32_t w, uint32_t c) {
  const uint64_t prod = (uint64_t)x * w;                     // < 2^63
  const uint64_t r1 = (prod & 0x7fffffffu) + (uint64_t)c * (uint32_t)(prod >> 31);  // < 2^31 + 2^44
  return (uint32_t)(r1 & 0x7fffffffu) + c * (uint32_t)(r1 >> 31);                 // < 2^31 + 2^25
}

struct W32PM {
  using T = uint32_t;
  using PT = uint32_t;
  using M = ModPM32;
  using Acc = W32::Acc;
  static constexpr int bytes = 4;
  __device__ static __forceinline__ Acc zero() { return W32::zero(); }
  __device__ static __forceinline__ void add(Acc &a, T x) { W32::add(a, x); }
  __device__ static __forceinline__ T reduce(const Acc &a, const M &m) { return W32::reduce(a, m.m); }
  __device__ static __forceinline__ T reduce_partial(const Acc &a, const M &m) { return W32::reduce(a, m.m); }
  using Sum = Acc;
  __device__ static __forceinline__ Sum sum_zero() { return zero(); }
  __device__ static __forceinline__ Sum sum_first(T x) { return W32::sum_first(x); }
  __device__ static __forceinline__ void sum_add(Sum &s, T x) { W32::sum_add(s, x); }
  __device__ static __forceinline__ Acc stage(const Acc &a, const M &) { return a; }
  __device__ static __forceinline__ void add_walk(Acc &a, const Acc &b, const M &) { W32::add(a, b); }
  __device__ static __forceinline__ T mul_lazy(T x, T w, T, const M &m) { return pm31_mul_lazy(x, w, m.c); }
};

// ---------------------------------------------------------------------------
// FP64 residues (p < 2^50): the paper's product, Alg. 2 (van der Hoeven,
// Lecerf and Quintin).  Values are exact integers held in doubles.
// ---------------------------------------------------------------------------
struct ModF64 {
  double p;   // the modulus
  double u;   // 1 / p, rounded to nearest
  Mod64 m;    // integer constants, for the output conversion
};

// Alg. 2 (p < 2^50): h + l = x*y exactly (FMA error-free product), c a
// quotient estimate from the precomputed 1/p, g = x y - c p the remainder.
// As printed, the algorithm takes x, y in [0, p), rounds the estimate down
// and applies two corrections (g >= p, g < 0) to land in [0, p).  Here x
// may be negative, |x| < p, with 0 <= y < p, and the estimate is rounded to
// nearest: h u differs from x y / p by at most 3/8 (relative errors of
// 2^-53 in h, in 1/p and in the product, on a quotient below 2^50), so
// |x y / p - c| <= 7/8 and g lies in (-7p/8, 7p/8) -- again a valid x, with
// no correction step.  g is exact: d = h - c p is an integer below 2^53 and
// d + l = x y - c p.  Running values thus stay signed; sums of them are
// folded (fp_fold) and made canonical only when a partial coefficient
// leaves the kernel.
__device__ __forceinline__ double alg2_mul_signed(double x, double y, double p, double u) {
#pragma clang fp contract(off)
  const double h = x * y;
  const double l = __builtin_fma(x, y, -h);
  const double c = __builtin_rint(h * u);
  const double d = __builtin_fma(-c, p, h);
  return d + l;
}

// An exact integer s with |s| < 2^53 folded to s - rint(s / p) p: congruent
// to s and within p/2 + 2^-30 p of zero (for p >= 2^31 the quotient
// estimate from 1/p is off by less than 2^-30), so |result| < p; exact,
// since the result is an integer below 2^53.  Rounding the quotient to
// nearest instead of down (as Alg. 2 does) leaves no correction step.  The
// sums of the FP64 policy (a thread's terms, the walks between threads) use
// it in place of Alg. 3's conditional subtraction, and stay signed.
__device__ __forceinline__ double fp_fold(double s, double p, double u) {
#pragma clang fp contract(off)
  const double c = __builtin_rint(s * u);
  return __builtin_fma(-c, p, s);
}

// Exact integer in [0, 2^53) held in a double -> uint64.
__device__ __forceinline__ uint64_t fp_to_u64(double v) {
#pragma clang fp contract(off)
  double hi = __builtin_floor(v * 0x1p-32);
  double lo = __builtin_fma(-hi, 0x1p32, v);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Running values in (-p, p) as doubles (alg2_mul_signed); a thread sums at
// most 8 of them (|sum| < 2^53, exact) and folds the sum into (-p, p); the
// walks add two folded values (|sum| < 2p) and fold again; partial sums
// leave as canonical uint64 residues (shared with the 64-bit integer path).
struct WF64 {
  using T = double;
  using PT = uint64_t;
  using M = ModF64;
  struct Acc {
    double s;
  };
  static constexpr int bytes = 8;
  __device__ static __forceinline__ Acc zero() { return Acc{0.0}; }
  __device__ static __forceinline__ void add(Acc &a, T x) { a.s += x; }
  using Sum = Acc;  // a thread's sum over its terms (at most 8, exact)
  __device__ static __forceinline__ Sum sum_zero() { return zero(); }
  __device__ static __forceinline__ Sum sum_first(T x) { return Sum{x}; }
  __device__ static __forceinline__ void sum_add(Sum &s, T x) { add(s, x); }
  // staged values and walk sums: folded, in (-p, p)
  __device__ static __forceinline__ void add_walk(Acc &a, const Acc &b, const M &m) {
    a.s = fp_fold(a.s + b.s, m.p, m.u);
  }
  __device__ static __forceinline__ PT reduce(const Acc &a, const M &m) {
    return fp_to_u64(a.s < 0.0 ? a.s + m.p : a.s);
  }
  __device__ static __forceinline__ PT reduce_partial(const Acc &a, const M &m) { return reduce(a, m); }
  __device__ static __forceinline__ Acc stage(const Acc &a, const M &m) { return Acc{fp_fold(a.s, m.p, m.u)}; }
  __device__ static __forceinline__ T mul_lazy(T x, T w, T, const M &m) { return alg2_mul_signed(x, w, m.p, m.u); }
};

}  // namespace peval
