// Sparse interpolation from the images: the step that follows the
// evaluations in Zippel's method (paper, Section 2.1).  Evaluating at the
// powers beta^t makes each group's linear system a transposed Vandermonde
// system, solvable in O(m^2) operations and O(m) space for a group of m
// terms (Zippel 1990).
//
// For a group with terms i_1..i_m, monomial values v_j = M_{i_j}(beta) and
// image coefficients c_t (t = 1..m), c_t = sum_j a_j v_j^t.  With the
// master polynomial Q(z) = prod_j (z - v_j) = sum_k q_k z^k, the quotient
// Q(z) / (z - v_j) has coefficients r_k = sum_{l>k} q_l v_j^{l-k-1}, and
// sum_k r_k c_{k+1} = a_j v_j Q'(v_j), because Q(z)/(z - v_j) vanishes at
// every other v.  Exchanging the sums gives sum_k r_k c_{k+1} = B(v_j) with
// B(z) = sum_l b_l z^l, b_l = sum_{k=0}^{m-1-l} q_{k+l+1} c_{k+1}.  So
//
//   a_j = B(v_j) / (v_j Q'(v_j)).
//
//   interp_prep_kernel   v_i (from the power tables) and the group's image
//                        column c laid out along the sorted terms, with
//                        Shoup quotients
//   interp_group_kernel  one block per part of a group: the product of its
//                        (z - v_j) in LDS (parts of 1024 roots or more)
//   interp_wave_group_kernel  the same product, one wave per part, in
//                        registers (parts below 1024 roots)
//   interp_merge_kernel  few groups: parts multiplied pairwise over the chip
//   interp_bcoef_kernel  over the whole chip: the coefficients of B and Q'
//   interp_solve_kernel  per term, over the whole chip: B(v_j) and Q'(v_j)
//                        by Horner, one inversion, the result scattered to
//                        the caller's term order
//
// Every multiplier that is used more than once (v_j in Q and in Horner, c_k
// in b_l) carries its precomputed Shoup quotient.  The inversion is by
// Fermat's little theorem, so p must be prime; a zero or non-invertible
// denominator (two equal monomial values in a group, a zero monomial value,
// a composite p) sets the status word and yields 0 for that term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace peval {

constexpr int kInterpPer = 8;               // coefficients per thread in the per-group kernel
constexpr uint32_t kInterpMaxGroup = 8191;  // terms per group: 1024 threads x 8, and Q in 64 KiB of LDS

template <class T>
__device__ __forceinline__ T sub_mod(T a, T b, T p) {  // canonical in/out
  return a >= b ? a - b : a + (p - b);
}

template <class A>
struct InterpArgs {
  using T = typename A::T;
  const T *images;          // [Timg][G] caller's images (any residues of the handle's width)
  const T *tval, *tquot;    // power tables of beta
  TableOffsets to;
  const uint16_t *exps;     // ntail arrays of s (sorted terms)
  const uint32_t *grp_off;  // G + 1
  const uint32_t *gorder;   // groups, largest first
  const uint32_t *order;    // sorted position -> caller's term index
  T *mval, *mquot;          // s: monomial values and quotients
  T *cval, *cquot;          // s: group image columns along the sorted terms
  T *bval;                  // s: coefficients of B per group
  T *dval;                  // s: coefficients of Q' per group
  T *qval;                  // s + G: coefficients of Q per group (group g at grp_off[g] + g)
  // Q as H sub-products per group, merged pairwise: with H_l parts per
  // group, part h of group g sits at grp_off[g] + g*H_l + start + h, where
  // start = (h*m)/H_l is its first root.  Values and Shoup quotients.
  T *part_val, *part_quot;  // the H parts of the group kernel (H > 1)
  uint32_t H;               // sub-products per group (1, 4 or 8)
  const uint32_t *task_group, *task_first;  // per wave of the solve: group, first term
  uint64_t ntasks;
  uint64_t *out;            // s coefficients in the caller's order
  int32_t *status;          // set to 1 when some group cannot be solved
  uint64_t s, G;
  uint32_t ntail;
  typename A::M m;
  // 64-bit residues with 2^31 <= p < 2^50 and the handle's product FP64:
  // B's and Q''s coefficients are stored as doubles and the solve's Horner
  // steps use the FP64 product (0 otherwise)
  uint32_t fp64;
  ModF64 mf;
};

template <class A>
__global__ void interp_prep_kernel(InterpArgs<A> a) {
  using T = typename A::T;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.s) return;
  // monomial value v_i = prod_k beta_k^{g_ik} from the tables
  T v = (T)(1 % a.m.p);
  for (uint32_t k = 0; k < a.ntail; ++k) {
    const uint32_t at = a.to.off[k] + a.exps[(uint64_t)k * a.s + i];
    v = (k == 0) ? a.tval[at] : A::mul_lazy(v, a.tval[at], a.tquot[at], a.m);
  }
  v = canon(v, (T)a.m.p);
  a.mval[i] = v;
  a.mquot[i] = shoup_quot(v, a.m);
  // c_{k+1} of the term's group, k = position of the term in its group
  uint32_t lo = 0, hi = (uint32_t)a.G;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (a.grp_off[mid] <= i) lo = mid;
    else hi = mid;
  }
  const uint64_t k = i - a.grp_off[lo];
  const T c = (T)reduce64((uint64_t)a.images[k * a.G + lo], a.m);
  a.cquot[i] = shoup_quot(c, a.m);
  a.cval[i] = c;
  if constexpr (sizeof(T) == 8) {
    if (a.fp64) a.cval[i] = (T)__double_as_longlong((double)c);  // read only by the b_l sums
  }
}

// Per part of a group (H blocks per group): prod (z - v_i) over the part's
// roots in LDS, written out at the end (with quotients when parts are
// merged afterwards).  Thread tid owns coefficients tid + r*BS, r <
// kInterpPer, so a part may have up to kInterpPer * BS - 1 roots.  The next
// root is loaded one step ahead.
template <class A, int BS>
__global__ __launch_bounds__(BS) void interp_group_kernel(InterpArgs<A> a) {
  using T = typename A::T;
  constexpr int R = kInterpPer;
  extern __shared__ __align__(16) unsigned char smem[];
  T *q = reinterpret_cast<T *>(smem);  // d + 1 coefficients
  const T p = (T)a.m.p;
  const uint32_t g = a.gorder[blockIdx.x / a.H];
  const uint32_t h = blockIdx.x % a.H;
  const uint64_t base = a.grp_off[g];
  const uint32_t m = a.grp_off[g + 1] - (uint32_t)base;
  const uint32_t r0 = (uint32_t)(((uint64_t)h * m) / a.H), r1 = (uint32_t)(((uint64_t)(h + 1) * m) / a.H);
  const uint32_t d = r1 - r0;  // roots of this part (may be 0)
  const int tid = threadIdx.x;

  // prod (z - v_i) over the part's roots, starting from 1
  for (uint32_t k = tid; k <= d; k += BS) q[k] = (k == 0) ? (T)(1 % p) : (T)0;
  __syncthreads();
  T v = d ? a.mval[base + r0] : (T)0, vq = d ? a.mquot[base + r0] : (T)0;
  for (uint32_t i = 0; i < d; ++i) {
    const uint32_t inext = (i + 1 < d) ? i + 1 : i;
    const T vn = a.mval[base + r0 + inext], vqn = a.mquot[base + r0 + inext];
    T nv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = tid + r * BS;
      if (k <= i + 1) {
        const T lo = k ? q[k - 1] : (T)0;
        const T hi = (k <= i) ? q[k] : (T)0;
        nv[r] = sub_mod(lo, canon(A::mul_lazy(hi, v, vq, a.m), p), p);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = tid + r * BS;
      if (k <= i + 1) q[k] = nv[r];
    }
    __syncthreads();
    v = vn;
    vq = vqn;
  }

  // the part leaves LDS: straight into Q when there is one part per group
  const uint64_t at = base + (uint64_t)g * a.H + r0 + h;
  T *out = (a.H == 1) ? a.qval + at : a.part_val + at;
  T *outq = (a.H == 1) ? nullptr : a.part_quot + at;
  for (uint32_t k = tid; k <= d; k += BS) {
    out[k] = q[k];
    if (outq) outq[k] = shoup_quot(q[k], a.m);
  }
}

// Lane l receives lane l - 1's value, lane 0 lane 63's (DPP wave rotation).
__device__ __forceinline__ uint32_t wave_ror1(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x13C, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t wave_ror1(uint64_t x) {
  return ((uint64_t)wave_ror1((uint32_t)(x >> 32)) << 32) | wave_ror1((uint32_t)x);
}
// Lane l's value for the whole wave (l wave-uniform).
__device__ __forceinline__ uint32_t read_lane(uint32_t x, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}
__device__ __forceinline__ uint64_t read_lane(uint64_t x, uint32_t l) {
  return ((uint64_t)read_lane((uint32_t)(x >> 32), l) << 32) | read_lane((uint32_t)x, l);
}

constexpr int kWaveGroupSlots = 16;  // parts of up to 16 * 64 - 1 roots in one wave

// Steps i_begin .. i_end - 1 of the wave product below, all with RA slots
// holding coefficients: straight-line code over the slots, so that the
// slots' independent products interleave.
template <class A, int RA, int RMAX>
__device__ __forceinline__ void wave_group_steps(typename A::T (&q)[RMAX], uint32_t i_begin, uint32_t i_end,
                                                 typename A::T &vbuf, typename A::T &qbuf, const typename A::T *mv,
                                                 const typename A::T *mq, uint32_t d, int lane,
                                                 const typename A::M &m) {
  using T = typename A::T;
  const T p = (T)m.p;
  for (uint32_t i = i_begin; i < i_end; ++i) {
    if ((i & 63) == 0) {  // the next 64 roots, one per lane
      const uint32_t j = i + lane;
      vbuf = (j < d) ? mv[j] : (T)0;
      qbuf = (j < d) ? mq[j] : (T)0;
    }
    const T v = read_lane(vbuf, i & 63), vq = read_lane(qbuf, i & 63);
    T rot[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) rot[r] = wave_ror1(q[r]);
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const T lo = (lane == 0) ? (r ? rot[r - 1] : (T)0) : rot[r];
      q[r] = sub_mod(lo, canon(A::mul_lazy(q[r], v, vq, m), p), p);
    }
  }
}

template <class A, int RA, int RMAX>
__device__ __forceinline__ void wave_group_chunk(uint32_t ra, typename A::T (&q)[RMAX], uint32_t i_begin,
                                                 uint32_t i_end, typename A::T &vbuf, typename A::T &qbuf,
                                                 const typename A::T *mv, const typename A::T *mq, uint32_t d,
                                                 int lane, const typename A::M &m) {
  if constexpr (RA <= RMAX) {
    if (ra == RA)
      wave_group_steps<A, RA, RMAX>(q, i_begin, i_end, vbuf, qbuf, mv, mq, d, lane, m);
    else
      wave_group_chunk<A, RA + 1, RMAX>(ra, q, i_begin, i_end, vbuf, qbuf, mv, mq, d, lane, m);
  }
}

// The same product with one wave per part and the coefficients in
// registers: coefficient k sits in lane k % 64 of slot k / 64.  Multiplying
// by (z - v) is q'_k = q_{k-1} - v q_k; every q_{k-1} comes from the
// neighbouring lane by a wave rotation (lane 0 takes lane 63 of the slot
// below), so a step uses no LDS and no barrier, and only the slots that
// already hold coefficients are updated (ra = (i + 1) / 64 + 1 of them at
// step i, constant over runs of 64 steps).  Parts are taken largest group
// first, one wave each.
template <class A, int RMAX>
__global__ __launch_bounds__(256) void interp_wave_group_kernel(InterpArgs<A> a, uint32_t nparts) {
  using T = typename A::T;
  const uint32_t part = (blockIdx.x * 256 + threadIdx.x) / 64;
  if (part >= nparts) return;  // whole waves leave together
  const int lane = threadIdx.x & 63;
  const T p = (T)a.m.p;
  const uint32_t g = __builtin_amdgcn_readfirstlane(a.gorder[part / a.H]);
  const uint32_t h = part % a.H;
  const uint64_t base = __builtin_amdgcn_readfirstlane(a.grp_off[g]);
  const uint32_t m = __builtin_amdgcn_readfirstlane(a.grp_off[g + 1]) - (uint32_t)base;
  const uint32_t r0 = (uint32_t)(((uint64_t)h * m) / a.H), r1 = (uint32_t)(((uint64_t)(h + 1) * m) / a.H);
  const uint32_t d = r1 - r0;  // roots of this part, d < RMAX * 64 (checked on the host)

  T q[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) q[r] = (r == 0 && lane == 0) ? (T)(1 % p) : (T)0;
  const T *mv = a.mval + base + r0, *mq = a.mquot + base + r0;
  T vbuf = 0, qbuf = 0;  // roots i0 .. i0 + 63, one per lane, taken by lane reads
  for (uint32_t c = 0; c < (uint32_t)RMAX; ++c) {  // steps with c + 1 slots
    const uint32_t ib = c ? 64 * c - 1 : 0, ie = min(d, 64 * c + 63);
    if (ib >= ie) break;
    wave_group_chunk<A, 1, RMAX>(c + 1, q, ib, ie, vbuf, qbuf, mv, mq, d, lane, a.m);
  }

  const uint64_t at = base + (uint64_t)g * a.H + r0 + h;
  T *out = (a.H == 1) ? a.qval + at : a.part_val + at;
  T *outq = (a.H == 1) ? nullptr : a.part_quot + at;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const uint32_t k = (uint32_t)r * 64 + lane;
    if (k <= d) {
      out[k] = q[r];
      if (outq) outq[k] = shoup_quot(q[r], a.m);
    }
  }
}

// One merge level: for every group, parts 2j and 2j+1 of a level with H_l
// parts per group multiply into part j of the next level (H_l / 2 parts).  One wave per
// 64 consecutive coefficients of one product (tasks built on the host);
// the left operand's coefficient is wave-uniform, the right one carries its
// Shoup quotient.
template <class A>
__global__ __launch_bounds__(256) void interp_merge_kernel(InterpArgs<A> a, const typename A::T *in_v,
                                                           const typename A::T *in_q, typename A::T *out_v,
                                                           typename A::T *out_q, uint32_t Hl,
                                                           const uint32_t *mt_group, const uint32_t *mt_pair,
                                                           const uint32_t *mt_first, uint64_t ntasks) {
  using T = typename A::T;
  const uint64_t task = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  if (task >= ntasks) return;  // whole waves leave together
  const uint32_t g = __builtin_amdgcn_readfirstlane(mt_group[task]);
  const uint32_t j = __builtin_amdgcn_readfirstlane(mt_pair[task]);
  const uint32_t k0 = __builtin_amdgcn_readfirstlane(mt_first[task]);
  const uint64_t base = __builtin_amdgcn_readfirstlane(a.grp_off[g]);
  const uint32_t m = __builtin_amdgcn_readfirstlane(a.grp_off[g + 1]) - (uint32_t)base;
  auto start = [&](uint32_t hh, uint32_t HH) { return (uint32_t)(((uint64_t)hh * m) / HH); };
  const uint32_t ha = 2 * j, hb = 2 * j + 1;
  const uint32_t ra = start(ha, Hl), rb = start(hb, Hl), re = start(hb + 1, Hl);
  const uint32_t da = rb - ra, db = re - rb;
  const T *av = in_v + base + (uint64_t)g * Hl + ra + ha;
  const T *bv = in_v + base + (uint64_t)g * Hl + rb + hb;
  const T *bq = in_q + base + (uint64_t)g * Hl + rb + hb;
  const uint32_t Hn = Hl / 2;
  const uint64_t at = base + (uint64_t)g * Hn + start(j, Hn) + j;
  T *out = out_v + at;
  T *outq = out_q ? out_q + at : nullptr;  // quotients only where the part is merged again
  const uint32_t k = k0 + (threadIdx.x & 63);
  typename A::Sum acc = A::sum_zero();
  // out_k = sum_i a_i b_{k-i}; the wave's 64 outputs need i in [k0-db, k0+63]
  const uint32_t i_lo = (k0 > db) ? k0 - db : 0;
  const uint32_t i_hi = (k0 + 63 < da) ? k0 + 63 : da;
  // four steps per iteration, their loads issued together
  uint32_t i = i_lo;
  for (; i + 3 <= i_hi; i += 4) {
    T b[4], q[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const bool in = k >= i + u && k - (i + u) <= db;
      b[u] = in ? bv[k - (i + u)] : (T)0;
      q[u] = in ? bq[k - (i + u)] : (T)0;
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) A::sum_add(acc, A::mul_lazy(av[i + u], b[u], q[u], a.m));
  }
  for (; i <= i_hi; ++i) {
    const bool in = k >= i && k - i <= db;
    const T b = in ? bv[k - i] : (T)0, q = in ? bq[k - i] : (T)0;
    A::sum_add(acc, A::mul_lazy(av[i], b, q, a.m));
  }
  if (k <= da + db) {
    const T r = A::reduce(A::stage(acc, a.m), a.m);
    out[k] = r;
    if (outq) outq[k] = shoup_quot(r, a.m);
  }
}

// b_l = sum_{k=0}^{m-1-l} q_{k+l+1} c_{k+1} and the Q' coefficient
// (l+1) q_{l+1}, over the whole chip: one wave per 64 consecutive l of one
// group (the solve kernel's tasks), so c_{k+1} is wave-uniform.
template <class A>
__global__ __launch_bounds__(256) void interp_bcoef_kernel(InterpArgs<A> a) {
  using T = typename A::T;
  const uint64_t task = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  if (task >= a.ntasks) return;  // whole waves leave together
  const uint32_t g = __builtin_amdgcn_readfirstlane(a.task_group[task]);
  const uint32_t l0 = __builtin_amdgcn_readfirstlane(a.task_first[task]);
  const uint64_t base = __builtin_amdgcn_readfirstlane(a.grp_off[g]);
  const uint32_t m = __builtin_amdgcn_readfirstlane(a.grp_off[g + 1]) - (uint32_t)base;
  const uint32_t l = l0 + (threadIdx.x & 63);
  const T *qg = a.qval + base + g;
  const T *cv = a.cval + base, *cq = a.cquot + base;
  // lanes of the wave stop at m-1-l: the longest runs first, the others idle
  const uint32_t kend = (l < m) ? m - l : 0;  // k < m - l
  const uint32_t kmax = m - l0;                // longest run in the wave
  if (a.fp64) {  // set for 64-bit residues only
    // FP64 product (Alg. 2, quotient rounded to nearest): q (an integer
    // residue, converted) times c (stored as a double) lands within 7p/8 of
    // zero; four of them added to a folded sum stay below 4p, folded again
    const double pf = a.mf.p, uf = a.mf.u;
    const double *cvf = reinterpret_cast<const double *>(cv);
    double accf = 0.0;
    uint32_t k = 0;
    for (; k + 4 <= kmax; k += 4) {
      T qv[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) qv[u] = (k + u < kend) ? qg[k + u + l + 1] : (T)0;
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) accf += alg2_mul_signed((double)qv[u], cvf[k + u], pf, uf);
      accf = fp_fold(accf, pf, uf);
    }
    for (; k < kmax; ++k) {
      const T q = (k < kend) ? qg[k + l + 1] : (T)0;
      accf = fp_fold(accf + alg2_mul_signed((double)q, cvf[k], pf, uf), pf, uf);
    }
    if (l < m) {
      const double bl = accf < 0.0 ? accf + pf : accf;  // canonical, as the solve reads it
      const T dl = mul_mod(qg[l + 1], (T)((l + 1) % a.m.p), a.m);
      a.bval[base + l] = (T)__double_as_longlong(bl);
      a.dval[base + l] = (T)__double_as_longlong((double)dl);
    }
    return;
  }
  typename A::Sum acc = A::sum_zero();
  // four steps per iteration, their loads issued together
  uint32_t k = 0;
  for (; k + 4 <= kmax; k += 4) {
    T qv[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) qv[u] = (k + u < kend) ? qg[k + u + l + 1] : (T)0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) A::sum_add(acc, A::mul_lazy(qv[u], cv[k + u], cq[k + u], a.m));
  }
  for (; k < kmax; ++k) {
    const T q = (k < kend) ? qg[k + l + 1] : (T)0;
    A::sum_add(acc, A::mul_lazy(q, cv[k], cq[k], a.m));
  }
  if (l < m) {
    a.bval[base + l] = A::reduce(A::stage(acc, a.m), a.m);
    a.dval[base + l] = mul_mod(qg[l + 1], (T)((l + 1) % a.m.p), a.m);
  }
}

// Per term: a_j = B(v_j) / (v_j Q'(v_j)) by Horner.  Every wave works on
// one group (a task = group and first term), so the group's b_l and Q'
// coefficients are read at wave-uniform addresses.
template <class A>
__global__ __launch_bounds__(256) void interp_solve_kernel(InterpArgs<A> a) {
  using T = typename A::T;
  const T p = (T)a.m.p;
  const uint64_t task = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  if (task >= a.ntasks) return;  // whole waves leave together
  const uint32_t g = __builtin_amdgcn_readfirstlane(a.task_group[task]);
  const uint32_t j0 = __builtin_amdgcn_readfirstlane(a.task_first[task]);
  const uint64_t base = __builtin_amdgcn_readfirstlane(a.grp_off[g]);
  const uint32_t m = __builtin_amdgcn_readfirstlane(a.grp_off[g + 1]) - (uint32_t)base;
  const uint32_t j = j0 + (threadIdx.x & 63);
  const bool live = j < m;
  const T v = live ? a.mval[base + j] : (T)0, vq = live ? a.mquot[base + j] : (T)0;
  const T *bv = a.bval + base, *dv = a.dval + base;
  T b = 0, d = 0;
  if (a.fp64) {  // set for 64-bit residues only
    // FP64 product (Alg. 2, quotient rounded to nearest): a running value
    // in (-p, p) times v gives one within 7p/8 of zero, plus a coefficient
    // in [0, p) below 2p in magnitude, folded back within p/2 of zero
    // (exact integers throughout); made canonical at the end
    const double pf = a.mf.p, uf = a.mf.u, vf = (double)v;
    const double *bvf = reinterpret_cast<const double *>(bv), *dvf = reinterpret_cast<const double *>(dv);
    double bf = 0.0, df = 0.0;
    for (uint32_t l = m; l-- > 0;) {
      bf = fp_fold(alg2_mul_signed(bf, vf, pf, uf) + bvf[l], pf, uf);
      df = fp_fold(alg2_mul_signed(df, vf, pf, uf) + dvf[l], pf, uf);
    }
    b = (T)fp_to_u64(bf < 0.0 ? bf + pf : bf);
    d = (T)fp_to_u64(df < 0.0 ? df + pf : df);
  } else if (a.m.p < (T)(~(T)0 / 3)) {
    // 3p fits the word: the running values stay lazy in [0, 3p) (a Shoup
    // product takes any input below 2^64 and returns below 2p)
    for (uint32_t l = m; l-- > 0;) {
      b = A::mul_lazy(b, v, vq, a.m) + bv[l];
      d = A::mul_lazy(d, v, vq, a.m) + dv[l];
    }
    b = canon(canon(b, p), p);
    d = canon(canon(d, p), p);
  } else {
    // 3p does not fit: one conditional subtraction per step keeps the
    // running values in [0, 2p), still a valid Shoup input
    for (uint32_t l = m; l-- > 0;) {
      b = canon(A::mul_lazy(b, v, vq, a.m), p) + bv[l];
      d = canon(A::mul_lazy(d, v, vq, a.m), p) + dv[l];
    }
    b = canon(b, p);
    d = canon(d, p);
  }
  if (!live) return;
  const T den = canon(A::mul_lazy(d, v, vq, a.m), p);
  T res = 0;
  const T inv = den ? pow_mod(den, (uint64_t)a.m.p - 2, a.m) : (T)0;
  if (den && mul_mod(den, inv, a.m) == (T)(1 % p)) {
    res = mul_mod(b, inv, a.m);
  } else {
    a.status[0] = 1;
  }
  a.out[a.order[base + j]] = (uint64_t)res;
}

}  // namespace peval
