// HIP kernels of the matrix method (paper, Section 2.3, Alg. 1 and Alg. 7),
// laid out for gfx950.
//
//   power_table_kernel   beta_k^j for 0 <= j <= deg(f, x_k)       (Section 2.3)
//   monomial_kernel      m_i = M_i(beta) with n-3 products from the tables;
//                        chain starts Lambda_c = a_i m_i^{t0+c}, Gamma = m_i^C
//                        (the independent evaluations of Section 4.2 / Alg. 7)
//   eval_kernel          per evaluation: coefficient reduction of the running
//                        values, then their Hadamard product with Gamma
//   combine_kernel       sums the partial coefficients of groups that span
//                        several waves (or sub-tiles, in the point mode's
//                        layout) and writes the dense images
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

#include <type_traits>

#include "modarith.hpp"

namespace peval {

constexpr int kMaxTail = 30;  // n - 2 <= 30

struct BetaArg {
  uint64_t b[kMaxTail];
};

struct TableOffsets {
  uint32_t off[kMaxTail + 1];  // entries of variable k are off[k] .. off[k+1]-1
};

// Workgroups are dealt to the eight XCDs in turn (block b runs on XCD b % 8),
// and each XCD has its own L2.  A kernel whose neighbouring blocks read the
// same cache lines renumbers its blocks so that XCD x runs the consecutive
// logical blocks x chunk .. x chunk + chunk - 1: its grid has 8 chunk blocks,
// and logical blocks past the end return.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint64_t xcd_logical_block(uint32_t chunk) {
  return (uint64_t)(blockIdx.x % kXcds) * chunk + blockIdx.x / kXcds;
}

// ---------------------------------------------------------------------------
// A2: tables of powers beta_k^j (value and Shoup quotient)
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void power_entry(const BetaArg &beta, const uint32_t *off, uint32_t ntail, uint32_t idx,
                                            typename A::T *val, typename A::T *quot, const typename A::M &m) {
  uint32_t k = 0;
  while (k + 1 < ntail && idx >= off[k + 1]) ++k;
  uint32_t j = idx - off[k];
  typename A::T b = (typename A::T)beta.b[k];  // reduced on the host
  typename A::T v = pow_mod(b, (uint64_t)j, m);
  val[idx] = v;
  quot[idx] = shoup_quot(v, m);
}

template <class A>
__global__ void power_table_kernel(BetaArg beta, TableOffsets to, uint32_t ntail, uint32_t total,
                                   typename A::T *val, typename A::T *quot, typename A::M m) {
  uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  power_entry<A>(beta, to.off, ntail, idx, val, quot, m);
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
  uint32_t as_double;           // store canonical values as doubles (for the FP64 product)
  uint32_t R;                   // slots per work-item: 1 or mono_slots(K)
  uint32_t tab_total;           // power-table entries (all tail variables)
  uint32_t xchunk;              // logical blocks per XCD (grid = 8 xchunk blocks of 256)
  typename A::M m;
};

// Slots of one thread handled by one work-item of the monomial kernels: the
// R slots share the thread's term range, and their loads are all issued
// before any product, so a work-item waits for memory a few times instead
// of each slot waiting on its own.  A launch of fewer slots than a few
// rounds of the chip's resident threads keeps R = 1 (more threads waiting
// at once, and the first round is the whole launch).
__host__ __device__ constexpr uint32_t mono_slots(uint32_t K) { return K >= 4 ? 4 : K; }
constexpr uint64_t kMonoMultiSlots = 4ull << 20;
__host__ __device__ constexpr uint32_t mono_slots_for(uint32_t K, uint64_t slots) {
  return slots >= kMonoMultiSlots ? mono_slots(K) : 1u;
}
constexpr int kMonoFastTail = 8;  // tail exponents held in registers per slot

// off: power-table offsets per tail variable (read through a pointer so that
// a dynamically indexed copy never lands in scratch memory).
// idx enumerates tiles of 64 threads x K/R work-items of R consecutive
// slots, the item changing every 64 indices: the lanes of a wave store 64
// consecutive threads' values of one slot (coalesced, [k][thread] layout),
// and the few consecutive blocks that cover one tile read all K terms of its
// threads, so every cache line of term data is fetched once.  (With idx =
// k NT + j the waves of slot k read one term in K, and the term data came
// from HBM about K times over.)  NT is a multiple of 64, K a power of two
// and R (1, 2 or 4) divides K.
template <class A, int R>
__device__ __forceinline__ void monomial_entries(const MonoArgs<A> &a, const uint32_t *off, uint64_t idx,
                                                 const typename A::T *tval, const typename A::T *tquot) {
  using T = typename A::T;
  const uint32_t sh = 6 + __builtin_ctz(a.K / R);  // log2(64 K / R)
  const uint64_t tile = idx >> sh;
  const uint32_t r = (uint32_t)(idx & ((1ull << sh) - 1));
  const uint32_t k0 = (r >> 6) * R;
  const uint64_t j = (tile << 6) + (r & 63);
  const uint64_t NTK = (uint64_t)a.K * a.NT;
  const uint64_t p = a.m.p;
  // canonical value, or its double image when the evaluation uses Alg. 2
  auto out = [&](T v) -> T {
    if constexpr (sizeof(T) == 8) {
      if (a.as_double) return (T)__double_as_longlong((double)canon(v, (T)a.m.p));
    }
    return v;
  };
  const uint32_t cnt = a.thr_cnt[j];
  const uint64_t first = a.thr_first[j];
  bool live[R];
  T co[R];
  uint32_t ex[R][kMonoFastTail];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    live[u] = k0 + u < cnt;
    const uint64_t i = first + k0 + u;
    co[u] = live[u] ? a.coeff[i] : (T)0;
#pragma unroll
    for (int v = 0; v < kMonoFastTail; ++v)
      ex[u][v] = (live[u] && (uint32_t)v < a.ntail) ? a.exps[(uint64_t)v * a.s + i] : 0u;
  }
  // m_i = prod_k beta_k^{g_ik}, n-3 products using the tables (Section 2.3);
  // a padding slot's exponents are 0 and its product is never stored
  T mi[R];
#pragma unroll
  for (int v = 0; v < kMonoFastTail; ++v) {
    if ((uint32_t)v >= a.ntail) break;
    T tv[R], tq[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t at = off[v] + ex[u][v];
      tv[u] = tval[at];
      tq[u] = tquot[at];
    }
#pragma unroll
    for (int u = 0; u < R; ++u) mi[u] = (v == 0) ? tv[u] : A::mul_lazy(mi[u], tv[u], tq[u], a.m);
  }
  if (a.ntail == 0) {
#pragma unroll
    for (int u = 0; u < R; ++u) mi[u] = (T)(1 % p);
  }
  for (uint32_t v = kMonoFastTail; v < a.ntail; ++v) {  // more than 8 tail variables
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t e = live[u] ? a.exps[(uint64_t)v * a.s + first + k0 + u] : 0u;
      const uint32_t at = off[v] + e;
      mi[u] = A::mul_lazy(mi[u], tval[at], tquot[at], a.m);
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const uint64_t pos = (uint64_t)(k0 + u) * a.NT + j;  // slot (k, j) in the [k][thread] arrays
    if (!live[u]) {  // padding: a zero term stays zero (0.0 has the same bits)
      for (uint32_t c = 0; c < a.C; ++c) a.lam[c * NTK + pos] = 0;
      a.gam[pos] = 0;
      a.gamq[pos] = 0;
      continue;
    }
    const T m1 = canon(mi[u], (T)p);
    const T mq = shoup_quot(m1, a.m);
    // Lambda_0 = a_i m_i^{t0}; Lambda_c = Lambda_{c-1} m_i
    T lam;
    if (a.t0 == 1) {
      lam = A::mul_lazy(co[u], m1, mq, a.m);
    } else {
      T mt = pow_mod(m1, a.t0, a.m);
      lam = A::mul_lazy(co[u], mt, shoup_quot(mt, a.m), a.m);
    }
    a.lam[pos] = out(lam);
    // Gamma = m_i^C, the multiplier of every chain: for a few chains by the
    // same products that step the chain starts, else by squaring
    const bool stepped = a.C <= 16;
    T g = m1;
    for (uint32_t c = 1; c < a.C; ++c) {
      lam = A::mul_lazy(lam, m1, mq, a.m);
      a.lam[c * NTK + pos] = out(lam);
      if (stepped) g = A::mul_lazy(g, m1, mq, a.m);
    }
    g = stepped ? canon(g, (T)p) : pow_mod(m1, (uint64_t)a.C, a.m);
    a.gam[pos] = out(g);
    a.gamq[pos] = shoup_quot(g, a.m);
  }
}

template <class A>
__device__ __forceinline__ void monomial_entry(const MonoArgs<A> &a, const uint32_t *off, uint64_t idx,
                                               const typename A::T *tval, const typename A::T *tquot) {
  switch (a.R) {
    case 4: monomial_entries<A, 4>(a, off, idx, tval, tquot); break;
    case 2: monomial_entries<A, 2>(a, off, idx, tval, tquot); break;
    default: monomial_entries<A, 1>(a, off, idx, tval, tquot); break;
  }
}

// The power tables of a run (a few hundred entries for the usual degrees)
// are copied into LDS by every block of the monomial kernels, so that the
// tail variables' lookups, one after another, wait on LDS instead of L2;
// larger tables are read where they are.
constexpr uint32_t kMonoLdsEntries = 1024;

template <class A>
struct MonoTables {
  typename A::T val[kMonoLdsEntries], quot[kMonoLdsEntries];
};

// Every thread of the block calls this (it holds a barrier when the tables
// are staged); idx past `total` does nothing.
template <class A>
__device__ __forceinline__ void monomial_block(const MonoArgs<A> &a, const uint32_t *off, uint64_t idx,
                                               uint64_t total, uint32_t tab_total, MonoTables<A> &lds) {
  if (tab_total <= kMonoLdsEntries) {  // uniform over the block
    for (uint32_t e = threadIdx.x; e < tab_total; e += blockDim.x) {
      lds.val[e] = a.tval[e];
      lds.quot[e] = a.tquot[e];
    }
    __syncthreads();
    if (idx < total) monomial_entry<A>(a, off, idx, lds.val, lds.quot);
  } else if (idx < total) {
    monomial_entry<A>(a, off, idx, a.tval, a.tquot);
  }
}

// The work-items of one tile (64 K / R of them: at most one block for
// K <= 16) share their term data's cache lines; neighbouring tiles are kept
// on one XCD.
template <class A>
__global__ void monomial_kernel(MonoArgs<A> a) {
  __shared__ MonoTables<A> lds;
  const uint64_t idx = xcd_logical_block(a.xchunk) * blockDim.x + threadIdx.x;
  monomial_block<A>(a, a.to.off, idx, (uint64_t)a.K * a.NT / a.R, a.ntail ? a.tab_total : 0, lds);
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
  typename A::PT *partial;      // [nslots][C][Lmax] partial coefficients (64-bit: any representative)
  uint64_t NT, NW, nslots;
  uint32_t C, T;                // chains, evaluations in this launch
  uint32_t Lmax;                // ceil(T / C): evaluations of the longest chain
  typename A::M m;
  // direct layout (every group within one thread's K terms, so thread j
  // holds exactly group j): images straight to out, no partial sums
  uint32_t direct;
  uint64_t G;
  typename A::PT *out;          // [T][G] of this launch (direct layout)
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
struct Stage<WF64, P> {
  double v[64][P + 1];
  __device__ __forceinline__ void put(int lane, int q, const WF64::Acc &a) { v[lane][q] = a.s; }
  __device__ __forceinline__ WF64::Acc get(int lane, int q) const { return WF64::Acc{v[lane][q]}; }
};

template <int P>
struct Stage<W32, P> {
  uint64_t v[64][P + 1];
  __device__ __forceinline__ void put(int lane, int q, const W32::Acc &a) { v[lane][q] = a.v; }
  __device__ __forceinline__ W32::Acc get(int lane, int q) const { return W32::Acc{v[lane][q]}; }
};

// the pseudo-Mersenne policies stage exactly what their Shoup counterparts do
template <int P>
struct Stage<W64PM, P> : Stage<W64, P> {};
template <int P>
struct Stage<W32PM, P> : Stage<W32, P> {};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kEvalBlock = 256;  // 4 waves, each independent

// Transposed segmented sum of one pass of np <= P evaluations staged in st.
// The wave's endmask marks the last lane of every segment: group ends and
// the wave's last lane.  Lane (h, pp) walks sub-tile h (lanes h*P ..
// h*P+P-1) for evaluation pp: segments that start and end inside the
// sub-tile are emitted at once; the open segment before the sub-tile's first
// end (its head) and the one after its last end (its tail) are handed, through
// the stage, to lanes (0, pp), which chain the sub-tiles: a group that spans
// several sub-tiles of the wave leaves it as one partial.
// Partials are written as the policy's reduce_partial: canonical, except
// 64-bit residues, which may be any 64-bit representative (the combine makes
// them canonical).
// partial[(slot * C + c) * Lmax + i]: the P lanes of a sub-tile write P
// consecutive evaluations of one slot.  Merge = false is the plain walk for
// layouts whose endmask also closes every sub-tile: every end is emitted.
template <class A, int P, bool Merge = true>
__device__ __forceinline__ void segmented_walk(Stage<A, P> &st, int lane, int np, uint64_t emask, uint32_t sbase,
                                               typename A::PT *partial, uint32_t c, uint32_t C, uint32_t Lmax,
                                               uint32_t i0, const typename A::M &m) {
  constexpr int S = 64 / P;  // sub-tiles per wave
  constexpr uint64_t kSubMask = (P == 64) ? ~0ull : ((1ull << P) - 1ull);
  const int h = lane / P, pp = lane % P;
  const bool live = pp < np;
  typename A::PT *pcol = partial + (uint64_t)c * Lmax + i0 + pp;
  const uint64_t slot_stride = (uint64_t)C * Lmax;
  typename A::Acc head = A::zero(), sum = A::zero();
  if (live) {
    static_assert(P <= 32, "a sub-tile's segment ends fit one 32-bit word");
    // this sub-tile's end bits, and the slot of its first end (one slot per
    // end of the wave, in lane order)
    const uint32_t mybits = (uint32_t)((emask >> (h * P)) & kSubMask);
    uint32_t slot = sbase + (uint32_t)__popcll(emask & ((1ull << (h * P)) - 1ull));
    bool first = true;
#pragma unroll 4
    for (int jj = 0; jj < P; ++jj) {
      A::add_walk(sum, st.get(h * P + jj, pp), m);
      if ((mybits >> jj) & 1u) {
        if (Merge && first) {
          head = sum;
          first = false;
        } else {
          pcol[slot * slot_stride] = A::reduce_partial(sum, m);
        }
        ++slot;
        sum = A::zero();
      }
    }
  }
  if (!Merge) return;
  wave_sync();  // the staged values are read; rows h*P and h*P+1 now take head and tail
  if (live) {
    st.put(h * P, pp, head);
    st.put(h * P + 1, pp, sum);
  }
  wave_sync();
  if (h == 0 && live) {
    typename A::Acc carry = A::zero();
#pragma unroll
    for (int hh = 0; hh < S; ++hh) {
      const uint64_t bits = (emask >> (hh * P)) & kSubMask;
      if (bits) {  // wave-uniform: the carried segment closes at this sub-tile's first end
        typename A::Acc hd = st.get(hh * P, pp);
        A::add_walk(hd, carry, m);
        const int first_end = hh * P + (int)__builtin_ctzll(bits);
        const uint32_t slot = sbase + (uint32_t)__popcll(emask & ((1ull << first_end) - 1ull));
        pcol[slot * slot_stride] = A::reduce_partial(hd, m);
        carry = st.get(hh * P + 1, pp);
      } else {
        A::add_walk(carry, st.get(hh * P + 1, pp), m);
      }
    }
    // the wave's last lane always ends a segment, so the final carry is empty
  }
}

// A thread's whole group as a canonical coefficient (direct layout).  Few
// 64-bit values are made canonical and added modulo p (about 7 ops each);
// more, and every other product, go through the lazy sum and one reduction.
template <class A, int K>
__device__ __forceinline__ typename A::PT group_value(const typename A::T (&lam)[K], const typename A::M &m) {
  if constexpr (std::is_same<A, W64>::value && K <= 4) {
    uint64_t v = canon(lam[0], m.p);
#pragma unroll
    for (int k = 1; k < K; ++k) v = add_mod(v, canon(lam[k], m.p), m.p);
    return v;
  } else {
    typename A::Sum acc = A::sum_zero();
#pragma unroll
    for (int k = 0; k < K; ++k) A::sum_add(acc, lam[k]);
    return A::reduce(A::stage(acc, m), m);
  }
}

// One wave's share of the evaluations: threads wave*64 .. wave*64+63, chain c.
template <class A, int K, int P>
__device__ __forceinline__ void eval_wave(const EvalArgs<A> &a, uint64_t wave, uint32_t c, Stage<A, P> &st,
                                          int lane) {
  using T = typename A::T;
  static_assert(64 % P == 0, "P must divide the wave size");
  const uint64_t j = wave * 64 + lane;
  const uint64_t NTK = (uint64_t)K * a.NT;

  T lam[K], g[K], gq[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lam[k] = a.lam[c * NTK + (uint64_t)k * a.NT + j];
    g[k] = a.gam[(uint64_t)k * a.NT + j];
    gq[k] = a.gamq[(uint64_t)k * a.NT + j];
  }
  // evaluations of chain c, the same for the whole wave (the division is
  // done in vector registers; read back into a scalar one)
  const uint32_t L = __builtin_amdgcn_readfirstlane((c < a.T) ? (a.T - 1 - c) / a.C + 1 : 0);

  if (a.direct) {  // wave-uniform: thread j's sum is the coefficient of group j
    const bool live = j < a.G;
    typename A::PT *col = a.out + (uint64_t)c * a.G + j;
    const uint64_t row_stride = (uint64_t)a.C * a.G;
#pragma unroll 1
    for (uint32_t i = 0; i < L; ++i) {
      const typename A::PT v = group_value<A, K>(lam, a.m);
#pragma unroll
      for (int k = 0; k < K; ++k) lam[k] = A::mul_lazy(lam[k], g[k], gq[k], a.m);
      if (live) col[(uint64_t)i * row_stride] = v;  // neighbouring lanes: neighbouring groups
    }
    return;
  }
  const uint64_t emask = a.endmask[wave];
  const uint32_t sbase = a.slot_base[wave];

  for (uint32_t i0 = 0; i0 < L; i0 += P) {
    // (kept in a scalar register: the compiler forms the clamp with a vector
    // instruction, and the row loop would count in vector registers)
    const int np = __builtin_amdgcn_readfirstlane((L - i0 < (uint32_t)P) ? (int)(L - i0) : P);
    // P evaluations: reduce (sum the running values), then multiply by Gamma
#pragma unroll 1
    for (int q = 0; q < np; ++q) {
      typename A::Sum acc = A::sum_first(lam[0]);
      lam[0] = A::mul_lazy(lam[0], g[0], gq[0], a.m);
#pragma unroll
      for (int k = 1; k < K; ++k) {
        A::sum_add(acc, lam[k]);
        lam[k] = A::mul_lazy(lam[k], g[k], gq[k], a.m);
      }
      st.put(lane, q, A::stage(acc, a.m));
    }
    wave_sync();
    segmented_walk<A, P>(st, lane, np, emask, sbase, a.partial, c, a.C, a.Lmax, i0, a.m);
    wave_sync();
  }
}

// Three waves per SIMD for P <= 16: the 64-bit K = 16 variants need a few
// registers more than that allows (two spilled, outside the evaluation
// passes), and two waves hide the latency of the stage and walk less well.
// With P = 32 the stages alone hold a block's LDS to one or two blocks per
// CU, so a register bound would only cost spills.
template <class A, int K, int P>
__global__ __launch_bounds__(kEvalBlock, (P <= 16 ? (K >= 32 ? 2 : 3) : 1)) void eval_kernel(EvalArgs<A> a) {
  __shared__ Stage<A, P> stage[kEvalBlock / 64];
  const int lane = threadIdx.x & 63;
  const int warp = threadIdx.x >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * (kEvalBlock / 64) + warp;
  if (wave >= a.NW) return;  // whole waves leave; no block-wide barrier is used
  eval_wave<A, K, P>(a, wave, blockIdx.y, stage[warp], lane);
}

// ---------------------------------------------------------------------------
// A7: combine partial coefficients into the dense images
// ---------------------------------------------------------------------------
constexpr int kCombineTile = 64;   // groups x evaluations per block
constexpr int kCombineLoads = 16;  // partial sums in flight per lane
constexpr int kCombineBlock = 256;

template <class A>
struct CombineArgs {
  const typename A::T *partial;   // [nslots][C][Lmax]
  const uint32_t *slot_off;       // G + 1
  typename A::T *out;             // [T][G]
  uint64_t G;
  uint32_t C, T, Lmax;
  typename A::M m;
};

// One tile: groups g0..g0+63 x evaluations i0..i0+63 of chain c.  Each wave
// sums 16 groups with one lane per evaluation (coalesced reads along i),
// the tile is transposed in LDS and written row by row (coalesced along g).
template <class A>
__device__ __forceinline__ void combine_tile(const CombineArgs<A> &a, uint64_t g0, uint32_t c, uint32_t i0,
                                             typename A::T (*tile)[kCombineTile + 1]) {
  using T = typename A::T;
  const int lane = threadIdx.x & 63, warp = threadIdx.x >> 6;
  const uint32_t Lc = (c < a.T) ? (a.T - 1 - c) / a.C + 1 : 0;
  const bool live = i0 + lane < Lc;
  const uint64_t slot_stride = (uint64_t)a.C * a.Lmax;
  const T *col = a.partial + (uint64_t)c * a.Lmax + i0 + lane;
  // the wave's 16 groups own one contiguous run of slots; walk it with
  // kCombineLoads independent loads in flight (the kernel waits on memory,
  // not on its few VALU operations) and close a group whenever its slots end
  const int gl_first = warp * (kCombineTile / 4), gl_last = gl_first + kCombineTile / 4;
  for (int gl = gl_first; gl < gl_last; ++gl) tile[gl][lane] = 0;
  const uint64_t ga = g0 + gl_first;
  if (ga < a.G) {
    const uint64_t gb = (g0 + gl_last < a.G) ? g0 + gl_last : a.G;
    const uint32_t s_begin = a.slot_off[ga], s_end = a.slot_off[gb];
    int gl = gl_first;
    uint32_t next_end = a.slot_off[ga + 1];
    T acc = 0;
    for (uint32_t sl = s_begin; sl < s_end; sl += kCombineLoads) {
      T v[kCombineLoads];
#pragma unroll
      for (int u = 0; u < kCombineLoads; ++u)
        v[u] = (live && sl + u < s_end) ? col[(uint64_t)(sl + u) * slot_stride] : 0;
#pragma unroll
      for (int u = 0; u < kCombineLoads; ++u) {
        if (sl + u >= s_end) break;
        while (sl + u >= next_end) {  // uniform: slot boundaries are the same for every lane
          tile[gl][lane] = acc;
          acc = 0;
          ++gl;
          next_end = a.slot_off[g0 + gl + 1];
        }
        acc = add_mod(acc, A::canon_partial(v[u], a.m), (T)a.m.p);
      }
    }
    tile[gl][lane] = acc;  // last group of the run
  }
  __syncthreads();
  for (int r = warp; r < kCombineTile; r += 4) {
    const uint32_t i = i0 + r;
    const uint64_t g = g0 + lane;
    if (i < Lc && g < a.G) a.out[((uint64_t)c + (uint64_t)i * a.C) * a.G + g] = tile[lane][r];
  }
}

template <class A>
__global__ __launch_bounds__(kCombineBlock) void combine_kernel(CombineArgs<A> a) {
  __shared__ typename A::T tile[kCombineTile][kCombineTile + 1];
  combine_tile<A>(a, (uint64_t)blockIdx.x * kCombineTile, blockIdx.y, blockIdx.z * kCombineTile, tile);
}

}  // namespace peval
