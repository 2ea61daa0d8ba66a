// Images at T arbitrary points (x_{t,3}, ..., x_{t,n}) instead of the powers
// beta^t: the random evaluation points of Zippel's original method (paper,
// Section 2.1), whose cost the paper puts at O(nT(d+s)) (Section 2.3).
//
// With no common ratio between points there is no recurrence m_i^t; every
// term-evaluation forms its monomial afresh.  To keep that to a few products,
// the tail variables are grouped into at most four "factors": a factor's table
// holds, for one point, the products x_a^{e_a} x_b^{e_b} ... over every
// exponent combination of its variables (a variable of large degree is first
// split into two base-256 digits).  A term's monomial is then the product of
// one entry per factor, and its contribution a_i * M_i(x_t) takes NF Shoup
// products: every table entry carries its precomputed quotient, and so does
// the coefficient (which is fixed per term).
//
//   points_table_kernel  factor tables for every point of the launch (HBM);
//                        32-bit residues keep 4-byte entries, the factors
//                        after the first in Montgomery form (their product
//                        needs no quotient), 64-bit ones (value, quotient)
//   points_prep_kernel   per thread slot: a_i, its quotient, packed entry
//                        indices (once per polynomial and thread layout);
//                        a group's terms are dealt to its slots sorted by
//                        their table entries, k-major, so that neighbouring
//                        lanes read neighbouring entries
//   points_eval_kernel   per point: the block stages the point's tables in
//                        LDS (the next point's already on their way in
//                        registers), every thread sums its K terms; then the
//                        segmented walk of the power path, without the
//                        merge of sub-tiles (a pass holds only 8 points, too
//                        few to pay for the merge)
//
// The thread layout, partial-sum layout and combine are those of the power
// path, so the images come out in the same dense T x G form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace peval {

constexpr int kPointsP = 8;          // points per pass of the segmented walk
constexpr int kMaxFactors = 4;
constexpr int kMaxDigits = 2 * kMaxTail;
constexpr uint32_t kPointsTableBytes = 32768;  // LDS for one point's tables
// Bytes of one table entry: the value alone for 32-bit residues; the value
// and its Shoup quotient for 64-bit ones (for the FP64 product, the value as
// a double and an unused word).
template <class T>
constexpr uint32_t points_entry_bytes() { return sizeof(T) == 4 ? 4u : 16u; }
// 16-byte pieces per thread of the next point's tables prefetched into
// registers: four for 64-bit residues (tables up to 16 KiB; measured 10%
// faster on the 1e6-term workload), one for 32-bit ones (4-byte entries:
// tables up to 4 KiB in one piece per thread; four pieces cost those
// kernels a wave per SIMD)
template <class T>
constexpr int points_prefetch() { return sizeof(T) == 8 ? 4 : 1; }

// How a term's tail monomial is split into factor-table lookups.
struct FactorPlan {
  uint32_t ndig;                     // digit variables
  uint32_t nf;                       // factors, 1..kMaxFactors
  uint32_t E;                        // table entries per point, all factors (even)
  uint32_t f_off[kMaxFactors + 1];   // factor f owns entries f_off[f] .. f_off[f+1]-1
  uint8_t var[kMaxDigits];           // tail variable of the digit (0 = x3)
  uint8_t fac[kMaxDigits];           // factor holding the digit
  uint8_t shift[kMaxDigits];         // digit = (e >> shift) & mask
  uint16_t mask[kMaxDigits];
  uint16_t radix[kMaxDigits];        // digit values 0 .. radix-1
  uint32_t stride[kMaxDigits];       // place value of the digit in its factor's index
};

// One (value, quotient) table entry at byte offset off, read with a single
// 8- or 16-byte LDS load.
__device__ __forceinline__ void load_entry(const uint32_t *tab, uint32_t off, uint32_t &v, uint32_t &q) {
  const uint2 x = *reinterpret_cast<const uint2 *>(reinterpret_cast<const unsigned char *>(tab) + off);
  v = x.x;
  q = x.y;
}
__device__ __forceinline__ void load_entry(const uint64_t *tab, uint32_t off, uint64_t &v, uint64_t &q) {
  const uint4 x = *reinterpret_cast<const uint4 *>(reinterpret_cast<const unsigned char *>(tab) + off);
  v = ((uint64_t)x.y << 32) | x.x;
  q = ((uint64_t)x.w << 32) | x.z;
}
// FP64 product: the entry's value as a double (its second half is unused)
__device__ __forceinline__ void load_entry(const double *tab, uint32_t off, double &v, double &q) {
  v = *reinterpret_cast<const double *>(reinterpret_cast<const unsigned char *>(tab) + off);
  q = 0.0;
}
template <class T>
__device__ __forceinline__ T load_value(const T *tab, uint32_t off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const unsigned char *>(tab) + off);
}

// Montgomery's product for 32-bit residues (R = 2^32): x y / R mod p, lazy
// in [0, 2p), for x < 2p, y < p (so x y + m p < 2^64) and np = -p^{-1} mod
// 2^32.  Three instructions (the 64-bit product, m = lo(x y) np, then
// x y + m p, whose high word is the result) and no precomputed quotient of
// y, whose Montgomery form y R mod p is stored instead of y.
__device__ __forceinline__ uint32_t mont_mul32(uint32_t x, uint32_t y, uint32_t p, uint32_t np) {
  const uint64_t t = (uint64_t)x * y;
  const uint32_t mm = (uint32_t)t * np;
  return (uint32_t)(((uint64_t)mm * p + t) >> 32);
}

// -p^{-1} mod 2^32 for Montgomery's product (32-bit residues; unused otherwise)
template <class M>
__device__ __forceinline__ uint32_t mont_np(const M &) { return 0u; }
// (opaque to the compiler, which would otherwise move the negation after
// the multiply, one more instruction per product)
__device__ __forceinline__ uint32_t mont_np(const Mod32 &m) {
  uint32_t r = 0u - m.pinv;
  asm("" : "+s"(r));
  return r;
}

template <class A>
struct PointsArgs {
  const typename A::T *pa;     // [K][NT] coefficients (0 for padding)
  const typename A::T *paq;    // [K][NT] their Shoup quotients
  const uint64_t *pidx;        // [K][NT] byte offset of each factor's entry, 16 bits per factor
  const typename A::T *tables; // [T][E] entries of points_entry_bytes
  const uint64_t *endmask;
  const uint32_t *slot_base;
  typename A::PT *partial;     // [nslots][C][Lmax]
  uint64_t NT, NW;
  uint32_t C, T, Lmax, E;
  typename A::M m;
};

// One table entry for launch-local point t: the product over the factor's
// digits of x_var^(digit << shift), with its Shoup quotient; or, for the
// FP64 product (as_double), the value as a double and 0.
template <class A>
__global__ void points_table_kernel(const uint64_t *points, uint32_t ntail, uint32_t T, FactorPlan fp,
                                    typename A::T *tables, typename A::M m, uint32_t as_double) {
  using T_ = typename A::T;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)T * fp.E) return;
  const uint32_t t = (uint32_t)(idx / fp.E);
  const uint32_t e = (uint32_t)(idx - (uint64_t)t * fp.E);
  T_ v = (T_)(1 % m.p);
  if (e < fp.f_off[fp.nf]) {
    uint32_t f = 0;
    while (f + 1 < fp.nf && e >= fp.f_off[f + 1]) ++f;
    const uint32_t local = e - fp.f_off[f];
    for (uint32_t d = 0; d < fp.ndig; ++d) {
      if (fp.fac[d] != f) continue;
      const uint32_t digit = (local / fp.stride[d]) % fp.radix[d];
      if (!digit) continue;
      const T_ x = reduce64(points[(uint64_t)t * ntail + fp.var[d]], m);
      v = mul_mod(v, pow_mod(x, (uint64_t)digit << fp.shift[d], m), m);
    }
  }  // entries past the last factor (padding to an even count) hold 1
  if constexpr (sizeof(T_) == 4) {  // Montgomery form v 2^32 mod p past the first factor
    const bool mont = fp.nf > 1 && e >= fp.f_off[1] && e < fp.f_off[fp.nf];
    tables[idx] = mont ? canon(shoup_mul(v, m.R, m.Rq, m.p), m.p) : v;
    return;
  } else {
    if (as_double) {
      tables[2 * idx] = (T_)__double_as_longlong((double)v);
      tables[2 * idx + 1] = 0;
      return;
    }
    tables[2 * idx] = v;
    tables[2 * idx + 1] = shoup_quot(v, m);
  }
}

// Per thread slot (k, j): coefficient, quotient and the entry index of each
// factor.  slot_term[k * NT + j] names the term of the slot (a term of the
// thread's own group, in any order: the group's sum does not depend on it),
// or 0xffffffff for padding, which gets a zero coefficient and in-range
// indices.
// as_double: the coefficient as a double and no quotient (FP64 product).
template <class A>
__global__ void points_prep_kernel(const typename A::T *coeff, const uint16_t *exps, const uint32_t *slot_term,
                                   uint64_t s, uint64_t NT, uint32_t K, FactorPlan fp, typename A::T *pa,
                                   typename A::T *paq, uint64_t *pidx, typename A::M m, uint32_t as_double) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)K * NT) return;
  const uint32_t term = slot_term[idx];
  uint32_t local[kMaxFactors] = {0, 0, 0, 0};
  typename A::T a = 0, aq = 0;
  if (term != 0xffffffffu) {
    const uint64_t i = term;
    a = coeff[i];
    aq = shoup_quot(a, m);
    if constexpr (sizeof(a) == 8) {
      if (as_double) {
        a = (typename A::T)__double_as_longlong((double)a);
        aq = 0;
      }
    }
    for (uint32_t d = 0; d < fp.ndig; ++d) {
      const uint32_t e = exps[(uint64_t)fp.var[d] * s + i];
      const uint32_t digit = (e >> fp.shift[d]) & fp.mask[d];
      const uint32_t add = digit * fp.stride[d];
#pragma unroll
      for (int f = 0; f < kMaxFactors; ++f)
        if (fp.fac[d] == f) local[f] += add;
    }
  }
  // byte offsets of the entries in one point's tables (every offset is
  // below 32 KiB)
  uint64_t packed = 0;
#pragma unroll
  for (int f = 0; f < kMaxFactors; ++f)
    if ((uint32_t)f < fp.nf)
      packed |= (uint64_t)((fp.f_off[f] + local[f]) * points_entry_bytes<typename A::T>()) << (16 * f);
  pa[idx] = a;
  paq[idx] = aq;
  pidx[idx] = packed;
}



// Three waves per SIMD where the registers allow it without more than a
// couple of spills (every variant but K = 16 with three or four factor
// tables): the table gathers from LDS need the latency hiding, and the
// K = 16, NF = 2 variant would otherwise take a few registers more than
// three waves allow (two waves: 15% slower on 1e6 terms x 1024 points).
template <class A, int K, int NF>
__global__ __launch_bounds__(kEvalBlock, ((K == 16 && NF > 2) ? 2 : 3)) void points_eval_kernel(PointsArgs<A> a) {
  using T = typename A::T;
  constexpr int P = kPointsP;
  extern __shared__ __align__(16) unsigned char smem[];
  auto *stage = reinterpret_cast<Stage<A, P> *>(smem);
  T *tab = reinterpret_cast<T *>(smem + (kEvalBlock / 64) * sizeof(Stage<A, P>));
  const int lane = threadIdx.x & 63;
  const int warp = threadIdx.x >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * (kEvalBlock / 64) + warp;
  const uint32_t c = blockIdx.y;
  const bool active = wave < a.NW;  // idle waves still take part in the block barriers
  const uint64_t j = wave * 64 + lane;

  T av[K], aq[K];
  uint64_t ix[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    av[k] = active ? a.pa[(uint64_t)k * a.NT + j] : 0;
    aq[k] = active ? a.paq[(uint64_t)k * a.NT + j] : 0;
    ix[k] = active ? a.pidx[(uint64_t)k * a.NT + j] : 0;
  }
  const uint64_t emask = active ? a.endmask[wave] : 0;
  const uint32_t sbase = active ? a.slot_base[wave] : 0;
  // points of chain c, the same for the whole wave (the division is done
  // in vector registers; read back into a scalar one)
  const uint32_t L = __builtin_amdgcn_readfirstlane((c < a.T) ? (a.T - 1 - c) / a.C + 1 : 0);
  constexpr uint32_t EB = points_entry_bytes<T>();
  const uint32_t nvec = a.E * EB / 16;  // 16-byte pieces of one point's tables (E EB is a multiple of 16)
  const uint32_t pneg = mont_np(a.m);  // 32-bit residues: -p^{-1} mod 2^32

  // The first PRE x 256 pieces of the next point's tables are loaded into
  // registers while the current point is evaluated, so the HBM/L2 latency of
  // the copy overlaps the arithmetic; pieces beyond that are copied after the
  // barrier as they come.  Loads are unconditional at clamped indices
  // (nvec >= 1); the pieces past nvec are never stored.  (Held in named
  // variables: an indexed array here was kept in scratch memory.)
  constexpr int PRE = points_prefetch<T>();
  uint4 p0 = make_uint4(0, 0, 0, 0), p1 = p0, p2 = p0, p3 = p0;
  const uint32_t last = nvec - 1;
  const uint32_t u0 = min(threadIdx.x, last), u1 = min(threadIdx.x + kEvalBlock, last);
  const uint32_t u2 = min(threadIdx.x + 2 * kEvalBlock, last), u3 = min(threadIdx.x + 3 * kEvalBlock, last);
  static_assert(PRE == 0 || PRE == 1 || PRE == 4, "prefetch of 0, 1 or 4 pieces per thread");
  auto prefetch = [&](const uint4 *src) {
    if constexpr (PRE >= 1) p0 = src[u0];
    if constexpr (PRE == 4) {
      p1 = src[u1];
      p2 = src[u2];
      p3 = src[u3];
    }
  };
  const uint64_t pt_words = (uint64_t)a.E * EB / sizeof(T);  // words of one point's tables
  if (L) prefetch(reinterpret_cast<const uint4 *>(a.tables + (uint64_t)c * pt_words));

  for (uint32_t i0 = 0; i0 < L; i0 += P) {
    // (kept in a scalar register: the compiler forms the clamp with a vector
    // instruction, and the row loop would count in vector registers)
    const int np = __builtin_amdgcn_readfirstlane((L - i0 < (uint32_t)P) ? (int)(L - i0) : P);
#pragma unroll 1
    for (int q = 0; q < np; ++q) {
      const uint64_t t = (uint64_t)c + (uint64_t)(i0 + q) * a.C;
      const uint4 *src = reinterpret_cast<const uint4 *>(a.tables + t * pt_words);
      __syncthreads();  // the previous point's tables are no longer read
      {
        uint4 *t4 = reinterpret_cast<uint4 *>(tab);
        const uint32_t u = threadIdx.x;
        if constexpr (PRE >= 1) {
          if (u < nvec) t4[u] = p0;
        }
        if constexpr (PRE == 4) {
          if (u + kEvalBlock < nvec) t4[u + kEvalBlock] = p1;
          if (u + 2 * kEvalBlock < nvec) t4[u + 2 * kEvalBlock] = p2;
          if (u + 3 * kEvalBlock < nvec) t4[u + 3 * kEvalBlock] = p3;
        }
      }
      for (uint32_t u = threadIdx.x + PRE * kEvalBlock; u < nvec; u += kEvalBlock)
        reinterpret_cast<uint4 *>(tab)[u] = src[u];
      __syncthreads();
      if (i0 + q + 1 < L) prefetch(reinterpret_cast<const uint4 *>(a.tables + (t + a.C) * pt_words));
      if (active) {
        typename A::Sum acc;  // begun from the first term's value
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint64_t x = ix[k];
          T mv = load_value(tab, (uint32_t)x & 0xffff);
#pragma unroll
          for (int f = 1; f < NF; ++f) {
            if constexpr (sizeof(T) == 4) {  // Montgomery form: no quotient to read
              mv = mont_mul32(mv, load_value(tab, (uint32_t)(x >> (16 * f)) & 0xffff), a.m.p, pneg);
            } else {
              T tv, tq;
              load_entry(tab, (uint32_t)(x >> (16 * f)) & 0xffff, tv, tq);
              mv = A::mul_lazy(mv, tv, tq, a.m);
            }
          }
          const T v = A::mul_lazy(mv, av[k], aq[k], a.m);
          if (k == 0)
            acc = A::sum_first(v);
          else
            A::sum_add(acc, v);
        }
        stage[warp].put(lane, q, A::stage(acc, a.m));
      }
    }
    if (active) {
      wave_sync();
      segmented_walk<A, P, false>(stage[warp], lane, np, emask, sbase, a.partial, c, a.C, a.Lmax, i0, a.m);
      wave_sync();
    }
  }
}

}  // namespace peval
