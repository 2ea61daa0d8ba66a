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
//   interp_group_kernel  one block per group: Q by m multiplications with
//                        (z - v_j) in LDS, then b_l, then per term B(v_j)
//                        and Q'(v_j) by Horner, one inversion, the result
//                        scattered to the caller's term order
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

constexpr int kInterpBlock = 1024;
constexpr int kInterpPer = 8;                                  // LDS entries per thread in a Q update
constexpr uint32_t kInterpMaxGroup = kInterpBlock * kInterpPer - 1;  // 8191 terms

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
  uint64_t *out;            // s coefficients in the caller's order
  int32_t *status;          // set to 1 when some group cannot be solved
  uint64_t s, G;
  uint32_t ntail;
  typename A::M m;
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
  a.cval[i] = c;
  a.cquot[i] = shoup_quot(c, a.m);
}

template <class A>
__global__ __launch_bounds__(kInterpBlock) void interp_group_kernel(InterpArgs<A> a) {
  using T = typename A::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T *q = reinterpret_cast<T *>(smem);  // m + 1 coefficients
  const T p = (T)a.m.p;
  const uint32_t g = a.gorder[blockIdx.x];
  const uint64_t base = a.grp_off[g];
  const uint32_t m = a.grp_off[g + 1] - (uint32_t)base;
  const int tid = threadIdx.x;

  // Q(z) = 1, then multiply by (z - v_i) for each term of the group
  for (uint32_t k = tid; k <= m; k += kInterpBlock) q[k] = (k == 0) ? (T)(1 % p) : (T)0;
  __syncthreads();
  for (uint32_t i = 0; i < m; ++i) {
    const T v = a.mval[base + i], vq = a.mquot[base + i];
    T nv[kInterpPer];
#pragma unroll
    for (int r = 0; r < kInterpPer; ++r) {
      const uint32_t k = tid + r * kInterpBlock;
      if (k <= i + 1) {
        const T lo = k ? q[k - 1] : (T)0;
        const T hi = (k <= i) ? q[k] : (T)0;
        nv[r] = sub_mod(lo, canon(A::mul_lazy(hi, v, vq, a.m), p), p);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kInterpPer; ++r) {
      const uint32_t k = tid + r * kInterpBlock;
      if (k <= i + 1) q[k] = nv[r];
    }
    __syncthreads();
  }

  // b_l = sum_{k=0}^{m-1-l} q_{k+l+1} c_{k+1}
  for (uint32_t l = tid; l < m; l += kInterpBlock) {
    typename A::Acc acc = A::zero();
    for (uint32_t k = 0; k + l < m; ++k)
      A::add(acc, A::mul_lazy(q[k + l + 1], a.cval[base + k], a.cquot[base + k], a.m));
    a.bval[base + l] = A::reduce(acc, a.m);
  }
  // Q'(z) = sum_l (l+1) q_{l+1} z^l, in place of q
  {
    T nv[kInterpPer];
#pragma unroll
    for (int r = 0; r < kInterpPer; ++r) {
      const uint32_t l = tid + r * kInterpBlock;
      if (l < m) nv[r] = mul_mod(q[l + 1], (T)((l + 1) % a.m.p), a.m);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kInterpPer; ++r) {
      const uint32_t l = tid + r * kInterpBlock;
      if (l < m) q[l] = nv[r];
    }
  }
  __threadfence_block();  // b_l written by other threads of the block
  __syncthreads();

  // a_j = B(v_j) / (v_j Q'(v_j))
  for (uint32_t j = tid; j < m; j += kInterpBlock) {
    const T v = a.mval[base + j], vq = a.mquot[base + j];
    T b = 0, d = 0;
    for (uint32_t l = m; l-- > 0;) {
      b = add_mod(canon(A::mul_lazy(b, v, vq, a.m), p), a.bval[base + l], p);
      d = add_mod(canon(A::mul_lazy(d, v, vq, a.m), p), q[l], p);
    }
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
}

}  // namespace peval
