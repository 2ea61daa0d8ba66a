// HIP kernels of the matrix method (paper, Section 2.3, Alg. 1 and Alg. 7),
// laid out for gfx950.
//
//   power_table_kernel   beta_k^j for 0 <= j <= deg(f, x_k)       (Section 2.3)
//   monomial_kernel      m_i = M_i(beta) with n-3 products from the tables;
//                        chain starts Lambda_c = a_i m_i^{t0+c}, Gamma = m_i^C
//                        (the independent evaluations of Section 4.2 / Alg. 7)
//   eval_kernel          per evaluation: coefficient reduction of the running
//                        values, then their Hadamard product with Gamma
//   combine_kernel       sums the partial coefficients of groups that were
//                        split between sub-tiles and writes the dense images
//
// Thread layout.  Terms are sorted by (x1, x2) exponents so that like
// monomials are adjacent (Section 2.3); each group is split into runs of K
// terms and each run goes to one thread, padded with zero terms.  So every
// thread belongs to exactly one group and the coefficient reduction is a
// plain sum within a thread, then a segmented sum across threads.  Terms are
// stored "k-major" ([k][thread]) so that every load is coalesced.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.hpp"

namespace peval {

constexpr int kMaxTail = 30;  // n - 2 <= 30

struct BetaArg {
  uint64_t b[kMaxTail];
};

struct TableOffsets {
  uint32_t off[kMaxTail + 1];  // entries of variable k are off[k] .. off[k+1]-1
};

// ---------------------------------------------------------------------------
// A2: tables of powers beta_k^j (value and Shoup quotient)
// ---------------------------------------------------------------------------
template <class A>
__global__ void power_table_kernel(BetaArg beta, TableOffsets to, uint32_t ntail, uint32_t total,
                                   typename A::T *val, typename A::T *quot, typename A::M m) {
  uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  uint32_t k = 0;
  while (k + 1 < ntail && idx >= to.off[k + 1]) ++k;
  uint32_t j = idx - to.off[k];
  typename A::T b = (typename A::T)beta.b[k];  // reduced on the host
  typename A::T v = pow_mod(b, (uint64_t)j, m);
  val[idx] = v;
  quot[idx] = shoup_quot(v, m);
}

// ---------------------------------------------------------------------------
// A3: monomial values and chain starts
// ---------------------------------------------------------------------------
template <class A>
struct MonoArgs {
  const typename A::T *coeff;   // s sorted coefficients, canonical
  const uint16_t *exps;         // ntail arrays of s: exps[v * s + i] = exponent of x_{v+3}
  const typename A::T *tval;    // power tables
  const typename A::T *tquot;
  TableOffsets to;
  const uint32_t *thr_first;    // first sorted term of each thread
  const uint8_t *thr_cnt;       // number of real terms of each thread (0..K)
  typename A::T *lam;           // [C][K][NT] chain starts (lazy, < 2p)
  typename A::T *gam;           // [K][NT] Gamma = m^C (canonical)
  typename A::T *gamq;          // [K][NT] Shoup quotients of Gamma
  uint64_t s, NT;
  uint64_t t0;
  uint32_t ntail, K, C;
  typename A::M m;
};

template <class A>
__global__ void monomial_kernel(MonoArgs<A> a) {
  using T = typename A::T;
  uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)a.K * a.NT) return;
  uint32_t k = (uint32_t)(idx / a.NT);
  uint64_t j = idx - (uint64_t)k * a.NT;
  const uint64_t NTK = (uint64_t)a.K * a.NT;
  if (k >= a.thr_cnt[j]) {  // padding: a zero term stays zero
    for (uint32_t c = 0; c < a.C; ++c) a.lam[c * NTK + idx] = 0;
    a.gam[idx] = 0;
    a.gamq[idx] = 0;
    return;
  }
  const uint64_t i = (uint64_t)a.thr_first[j] + k;
  const uint64_t p = a.m.p;
  // m_i = prod_k beta_k^{g_ik}, n-3 products using the tables (Section 2.3)
  T mi = (T)(1 % p);
  for (uint32_t v = 0; v < a.ntail; ++v) {
    uint32_t e = a.exps[(uint64_t)v * a.s + i];
    uint32_t at = a.to.off[v] + e;
    mi = (v == 0) ? a.tval[at] : A::mul_lazy(mi, a.tval[at], a.tquot[at], a.m);
  }
  mi = canon(mi, (T)p);
  const T mq = shoup_quot(mi, a.m);
  // Lambda_0 = a_i m_i^{t0}; Lambda_c = Lambda_{c-1} m_i
  T lam;
  if (a.t0 == 1) {
    lam = A::mul_lazy(a.coeff[i], mi, mq, a.m);
  } else {
    T mt = pow_mod(mi, a.t0, a.m);
    lam = A::mul_lazy(a.coeff[i], mt, shoup_quot(mt, a.m), a.m);
  }
  a.lam[idx] = lam;
  for (uint32_t c = 1; c < a.C; ++c) {
    lam = A::mul_lazy(lam, mi, mq, a.m);
    a.lam[c * NTK + idx] = lam;
  }
  // Gamma = m_i^C, the multiplier of every chain
  T g = (a.C == 1) ? mi : pow_mod(mi, (uint64_t)a.C, a.m);
  a.gam[idx] = g;
  a.gamq[idx] = shoup_quot(g, a.m);
}

// ---------------------------------------------------------------------------
// A4-A6: Hadamard products and coefficient reductions
// ---------------------------------------------------------------------------
template <class A>
struct EvalArgs {
  const typename A::T *lam;     // [C][K][NT]
  const typename A::T *gam;     // [K][NT]
  const typename A::T *gamq;    // [K][NT]
  const uint64_t *endmask;      // per wave: bit l set if lane l closes a segment
  const uint32_t *slot_base;    // per wave: index of its first segment slot
  typename A::T *partial;       // [T][nslots] canonical partial coefficients
  uint64_t NT, NW, nslots;
  uint32_t C, T;                // chains, evaluations in this launch
  typename A::M m;
};

// LDS staging of one wave's per-thread sums: [lane][point] with one pad column.
template <class A, int P>
struct Stage;

template <int P>
struct Stage<W64, P> {
  uint64_t lo[64][P + 1];
  uint32_t hi[64][P + 1];
  __device__ __forceinline__ void put(int lane, int q, const W64::Acc &a) {
    lo[lane][q] = ((uint64_t)a.w1 << 32) | a.w0;
    hi[lane][q] = a.w2;
  }
  __device__ __forceinline__ W64::Acc get(int lane, int q) const {
    uint64_t v = lo[lane][q];
    return W64::Acc{(uint32_t)v, (uint32_t)(v >> 32), hi[lane][q]};
  }
};

template <int P>
struct Stage<W32, P> {
  uint64_t v[64][P + 1];
  __device__ __forceinline__ void put(int lane, int q, const W32::Acc &a) { v[lane][q] = a.v; }
  __device__ __forceinline__ W32::Acc get(int lane, int q) const { return W32::Acc{v[lane][q]}; }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kEvalBlock = 256;  // 4 waves, each independent

template <class A, int K, int P>
__global__ __launch_bounds__(kEvalBlock) void eval_kernel(EvalArgs<A> a) {
  using T = typename A::T;
  static_assert(64 % P == 0, "P must divide the wave size");
  __shared__ Stage<A, P> stage[kEvalBlock / 64];

  const int lane = threadIdx.x & 63;
  const int warp = threadIdx.x >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * (kEvalBlock / 64) + warp;
  if (wave >= a.NW) return;  // whole waves leave; no block-wide barrier is used
  const uint32_t c = blockIdx.y;
  const uint64_t j = wave * 64 + lane;
  const uint64_t NTK = (uint64_t)K * a.NT;

  T lam[K], g[K], gq[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lam[k] = a.lam[c * NTK + (uint64_t)k * a.NT + j];
    g[k] = a.gam[(uint64_t)k * a.NT + j];
    gq[k] = a.gamq[(uint64_t)k * a.NT + j];
  }
  const uint64_t emask = a.endmask[wave];
  const uint32_t sbase = a.slot_base[wave];
  const uint32_t L = (c < a.T) ? (a.T - 1 - c) / a.C + 1 : 0;  // evaluations of chain c
  const int h = lane / P, pp = lane % P;
  Stage<A, P> &st = stage[warp];

  for (uint32_t i0 = 0; i0 < L; i0 += P) {
    const int np = (L - i0 < (uint32_t)P) ? (int)(L - i0) : P;
    // P evaluations: reduce (sum the running values), then multiply by Gamma
#pragma unroll 1
    for (int q = 0; q < np; ++q) {
      typename A::Acc acc = A::zero();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        A::add(acc, lam[k]);
        lam[k] = A::mul_lazy(lam[k], g[k], gq[k], a.m);
      }
      st.put(lane, q, acc);
    }
    wave_sync();
    // transposed segmented sum: lane (h, pp) walks sub-tile h for evaluation pp
    if (pp < np) {
      typename A::Acc sum = A::zero();
      const uint64_t row = (uint64_t)c + (uint64_t)(i0 + pp) * a.C;
      T *prow = a.partial + row * a.nslots;
#pragma unroll 4
      for (int jj = 0; jj < P; ++jj) {
        const int src = h * P + jj;
        A::add(sum, st.get(src, pp));
        if ((emask >> src) & 1ull) {
          const uint32_t slot = sbase + (uint32_t)__popcll(emask & ((1ull << src) - 1ull));
          prow[slot] = A::reduce(sum, a.m);
          sum = A::zero();
        }
      }
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// A7: combine partial coefficients into the dense images
// ---------------------------------------------------------------------------
template <class A>
__global__ void combine_kernel(const typename A::T *partial, const uint32_t *slot_off,
                               typename A::T *out, uint64_t G, uint64_t nslots, uint64_t total,
                               typename A::M m) {
  using T = typename A::T;
  uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  uint64_t row = idx / G;
  uint64_t g = idx - row * G;
  const T *prow = partial + row * nslots;
  T acc = 0;
  for (uint32_t sl = slot_off[g]; sl < slot_off[g + 1]; ++sl) acc = add_mod(acc, prow[sl], (T)m.p);
  out[idx] = acc;
}

}  // namespace peval
