// Single-launch evaluation for small runs (the steps of Section 2.3 fused).
//
// A run of a few thousand terms and a few hundred evaluations does too little
// work to fill the chip, so its time is the launch and dependency latency of
// the four-kernel path (tables, chain starts, evaluation, combine).  Here one
// kernel does all of it.  Block b owns the L consecutive evaluations
// t0 + bL .. t0 + bL + L - 1 and all s terms:
//
//   1. the tables beta_k^j go to LDS (values and Shoup quotients);
//   2. each thread forms m_i = M_i(beta) for its terms, the chain start
//      a_i m_i^{t0+bL} by square-and-multiply, then L - 1 further products
//      by m_i (one independent chain per block, as in Alg. 7), and stores
//      the L term values of each term in LDS, [evaluation][term];
//   3. each thread sums one (evaluation, group) cell over the group's terms
//      (adjacent in the sorted order) and writes that image coefficient.
//
// Everything a block needs stays in LDS; the only HBM traffic is the term
// data (read once per block, from L2 after the first block) and the images.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "modarith.hpp"

namespace peval {

constexpr int kSmallBlock = 1024;              // threads per block
constexpr uint32_t kSmallLds = 64 * 1024;      // LDS bytes per block (tables + term values)
constexpr uint32_t kSmallMaxTerms = 8192;      // s limit of the path
constexpr uint32_t kSmallRowBytes = 32 * 1024;  // s * residue bytes limit: beyond it the few blocks
                                                // of a short run each carry too many terms
constexpr uint64_t kSmallMaxWork = 1ull << 20;  // s * T limit of the path
constexpr uint32_t kSmallMaxGroup = 256;       // terms of the largest group
constexpr uint32_t kSmallTargetBlocks = 256;   // blocks aimed at (one per CU)

template <class A>
struct SmallArgs {
  const typename A::T *coeff;  // s sorted coefficients, canonical
  const uint16_t *exps;        // ntail arrays of s: exps[v * s + i] = exponent of x_{v+3}
  const uint32_t *grp_off;     // G + 1 offsets of the groups in the sorted order
  typename A::T *out;          // T x G images, row-major
  BetaArg beta;                // base point, reduced
  TableOffsets to;             // power-table offsets per tail variable
  uint64_t t0;                 // first evaluation index
  uint32_t s, G, T, L;         // terms, groups, evaluations, evaluations per block
  uint32_t ntail, tab_total;
  typename A::M m;
};

// Table entry idx = beta_k^j.  The variable k is found by a loop over the
// uniform offsets (scalar loads of the kernel arguments), so that the table
// phase issues no vector memory load and waits for none.
template <class A>
__device__ __forceinline__ void small_table_entry(const SmallArgs<A> &a, uint32_t idx, typename A::T *tv,
                                                  typename A::T *tq) {
  using T = typename A::T;
  uint32_t base = 0;
  T b = 0;
  for (uint32_t v = 0; v < a.ntail; ++v) {
    const uint32_t o = a.to.off[v];
    if (idx >= o) {
      base = o;
      b = (T)a.beta.b[v];
    }
  }
  const T val = pow_mod(b, (uint64_t)(idx - base), a.m);
  tv[idx] = val;
  tq[idx] = shoup_quot(val, a.m);
}

template <class A>
__global__ __launch_bounds__(kSmallBlock) void small_run_kernel(SmallArgs<A> a) {
  using T = typename A::T;
  extern __shared__ __align__(16) unsigned char small_lds[];
  T *tv = (T *)small_lds;        // [tab_total] beta_k^j
  T *tq = tv + a.tab_total;      // [tab_total] their Shoup quotients
  T *vals = tq + a.tab_total;    // [L][s] term values, canonical
  const uint32_t tid = threadIdx.x;
  const T p = (T)a.m.p;
  const uint32_t *off = a.to.off;  // through a pointer: no dynamically indexed copy in scratch
  const uint32_t j0 = blockIdx.x * a.L;
  const uint32_t nj = min(a.L, a.T - j0);
  const uint64_t ts = a.t0 + j0;
  const uint32_t cells = nj * a.G;

  // The run is latency-bound, so the global loads that do not depend on the
  // tables go first and overlap the table computation: each thread's first
  // term (coefficient and up to kPre tail exponents) and the group bounds of
  // its first output cell.
  constexpr uint32_t kPre = 4;
  T c_first = 0;
  uint32_t e_first[kPre] = {0, 0, 0, 0};
  if (tid < a.s) {
    c_first = a.coeff[tid];
#pragma unroll
    for (uint32_t v = 0; v < kPre; ++v)
      if (v < a.ntail) e_first[v] = a.exps[(uint64_t)v * a.s + tid];
  }
  uint32_t gb_first = 0, ge_first = 0;
  if (tid < cells) {
    const uint32_t g = tid % a.G;
    gb_first = a.grp_off[g];
    ge_first = a.grp_off[g + 1];
  }

  for (uint32_t idx = tid; idx < a.tab_total; idx += blockDim.x) small_table_entry<A>(a, idx, tv, tq);
  __syncthreads();

  for (uint32_t i = tid; i < a.s; i += blockDim.x) {
    const bool first = i == tid;
    T mi = (T)(1 % p);
#pragma unroll
    for (uint32_t v = 0; v < kPre; ++v) {
      if (v < a.ntail) {
        const uint32_t at = off[v] + (first ? e_first[v] : a.exps[(uint64_t)v * a.s + i]);
        mi = (v == 0) ? tv[at] : A::mul_lazy(mi, tv[at], tq[at], a.m);
      }
    }
    for (uint32_t v = kPre; v < a.ntail; ++v) {
      const uint32_t at = off[v] + a.exps[(uint64_t)v * a.s + i];
      mi = A::mul_lazy(mi, tv[at], tq[at], a.m);
    }
    mi = canon(mi, p);
    const T mq = shoup_quot(mi, a.m);
    const T mt = pow_mod(mi, ts, a.m);
    const T c = first ? c_first : a.coeff[i];
    T lam = A::mul_lazy(c, mt, shoup_quot(mt, a.m), a.m);  // a_i m_i^{ts}, in [0, 2p)
    vals[i] = canon(lam, p);
    for (uint32_t j = 1; j < nj; ++j) {
      lam = A::mul_lazy(lam, mi, mq, a.m);
      vals[(uint64_t)j * a.s + i] = canon(lam, p);
    }
  }
  __syncthreads();

  for (uint32_t q = tid; q < cells; q += blockDim.x) {
    const uint32_t j = q / a.G, g = q - j * a.G;
    const T *row = vals + (uint64_t)j * a.s;
    auto acc = A::zero();
    const uint32_t b = (q == tid) ? gb_first : a.grp_off[g], e = (q == tid) ? ge_first : a.grp_off[g + 1];
    for (uint32_t i = b; i < e; ++i) A::add(acc, row[i]);
    a.out[(uint64_t)(j0 + j) * a.G + g] = A::reduce(acc, a.m);
  }
}

}  // namespace peval
