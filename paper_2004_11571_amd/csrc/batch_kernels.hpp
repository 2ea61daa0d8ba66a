// Batched evaluation of many polynomials in one pass: flattened prologue and
// combine kernels plus persistent evaluation kernels, one per kind of member
// (product, residue width, range of K), each pulling work items
// (polynomial, wave, chain) from its own queue, biggest first.
//
// Each polynomial keeps its own modulus, residue width, thread layout and
// chains; the per-wave work is exactly eval_wave of the single-polynomial
// path, selected per item by a wave-uniform switch on K.  The queue counter
// only decides which wave does an item; every item writes its own
// partial-sum slots, so results never depend on the schedule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "batch_types.hpp"
#include "kernels.hpp"

namespace peval {

// index of the polynomial whose flattened range holds idx (prefix has count+1 entries)
__device__ __forceinline__ uint32_t find_poly(const uint64_t *prefix, uint32_t count, uint64_t idx) {
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (prefix[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Member of entry idx for a flattened kernel: thread 0 finds the member of
// the block's first entry (blocks cover consecutive entries), and each thread
// steps forward from there, rarely more than once.
__device__ __forceinline__ uint32_t find_poly_block(const uint64_t *prefix, uint32_t count, uint64_t idx,
                                                    uint64_t block_first, uint32_t *shared_first) {
  if (threadIdx.x == 0) shared_first[0] = find_poly(prefix, count, block_first);
  __syncthreads();
  uint32_t j = shared_first[0];
  while (j + 1 < count && prefix[j + 1] <= idx) ++j;
  return j;
}

__global__ void batch_reset_kernel(uint32_t *counter) {  // the work queues, one per kind
  if (blockIdx.x == 0 && threadIdx.x < kKinds) counter[threadIdx.x] = 0;
}

__global__ void batch_power_kernel(const BatchDesc *D, const BatchRun *R, uint32_t count, const uint64_t *prefix) {
  __shared__ uint32_t first;
  const uint64_t block_first = (uint64_t)blockIdx.x * blockDim.x;
  const uint64_t idx = block_first + threadIdx.x;
  uint32_t j = find_poly_block(prefix, count, idx, block_first, &first);  // every thread takes part in the barrier
  if (idx >= prefix[count]) return;
  const BatchDesc &d = D[j];
  uint32_t local = (uint32_t)(idx - prefix[j]);
  if (d.w == 4)
    power_entry<W32>(R[j].beta, d.to.off, d.ntail, local, (uint32_t *)d.tval, (uint32_t *)d.tquot, d.m32);
  else
    power_entry<W64>(R[j].beta, d.to.off, d.ntail, local, (uint64_t *)d.tval, (uint64_t *)d.tquot, d.m64);
}

template <class A>
__device__ __forceinline__ void batch_mono_one(const BatchDesc &d, uint64_t t0, uint64_t local, const typename A::M &m,
                                               MonoTables<A> &lds) {
  using T = typename A::T;
  MonoArgs<A> a;
  a.coeff = (const T *)d.coeff;
  a.exps = d.exps;
  a.tval = (const T *)d.tval;
  a.tquot = (const T *)d.tquot;
  a.thr_first = d.thr_first;
  a.thr_cnt = d.thr_cnt;
  a.lam = (T *)d.lam;
  a.gam = (T *)d.gam;
  a.gamq = (T *)d.gamq;
  a.s = d.s;
  a.NT = d.NT;
  a.t0 = t0;
  a.ntail = d.ntail;
  a.K = d.K;
  a.C = d.C;
  a.as_double = d.kind == kKindF64;  // FP64 members take chain starts and Gamma as doubles
  a.R = mono_slots(d.K);             // fixed per member: its work-items are counted when the batch is planned
  a.tab_total = d.tab_total;
  a.m = m;
  monomial_block<A>(a, d.to.off, local, (uint64_t)d.K * d.NT / a.R, d.ntail ? d.tab_total : 0, lds);
}

// Each member's entries start on a block boundary (its range padded to whole
// blocks of kMonoBlock, the members of one kind together), so a block belongs
// to one member, read from a table: the member and its descriptor are
// uniform over the block.  A launch covers blocks base .. base + nblocks - 1,
// renumbered per XCD as in monomial_kernel (xchunk logical blocks per XCD,
// grid 8 xchunk).
constexpr uint32_t kMonoBlock = 256;

__global__ __launch_bounds__(kMonoBlock) void batch_mono_kernel(const BatchDesc *__restrict__ D,
                                                                const BatchRun *__restrict__ R,
                                                                const uint32_t *__restrict__ block_member,
                                                                const uint64_t *__restrict__ prefix, uint64_t base,
                                                                uint64_t nblocks, uint32_t xchunk) {
  __shared__ union {
    MonoTables<W32> w32;
    MonoTables<W64> w64;
  } lds;
  const uint64_t rel = xcd_logical_block(xchunk);
  if (rel >= nblocks) return;  // uniform over the block
  const uint64_t lb = base + rel;  // blocks base .. base + nblocks - 1 of the pass
  const uint32_t j = __builtin_amdgcn_readfirstlane(block_member[lb]);
  const BatchDesc &d = D[j];
  const uint64_t local = lb * kMonoBlock - prefix[j] + threadIdx.x;  // past the member's items: padding
  if (d.w == 4) batch_mono_one<W32>(d, R[j].t0, local, d.m32, lds.w32);
  else batch_mono_one<W64>(d, R[j].t0, local, d.m64, lds.w64);
}

template <class A, int K, int P>
__device__ __forceinline__ void batch_eval_item(const BatchDesc &d, const BatchItem &it, void *out, void *lds,
                                                int lane, const typename A::M &m) {
  using T = typename A::T;
  EvalArgs<A> a;
  a.lam = (const T *)d.lam;
  a.gam = (const T *)d.gam;
  a.gamq = (const T *)d.gamq;
  a.endmask = d.endmask;
  a.slot_base = d.slot_base;
  a.partial = (typename A::PT *)d.partial;
  a.NT = d.NT;
  a.NW = d.NW;
  a.nslots = d.nslots;
  a.C = d.C;
  a.T = d.T;
  a.Lmax = d.Lmax;
  a.m = m;
  a.direct = d.direct;
  a.G = d.G;
  a.out = (typename A::PT *)out;
  eval_wave<A, K, P>(a, it.wave, it.chain, *reinterpret_cast<Stage<A, P> *>(lds), lane);
}

template <class A>
__device__ __forceinline__ const typename A::M &member_mod(const BatchDesc &d);
template <>
__device__ __forceinline__ const Mod32 &member_mod<W32>(const BatchDesc &d) { return d.m32; }
template <>
__device__ __forceinline__ const Mod64 &member_mod<W64>(const BatchDesc &d) { return d.m64; }
template <>
__device__ __forceinline__ const ModF64 &member_mod<WF64>(const BatchDesc &d) { return d.mf; }

// Persistent evaluation over the work queue of the members of one kind
// (policy A, terms per thread KLO..KHI, P evaluations per pass, WAVES
// waves per SIMD as a register bound).  A wave takes the next item; an item
// of another kind is never planned into this queue and is skipped rather
// than misread.
template <class A, int KLO, int KHI, int P, int WAVES, uint32_t KIND>
__global__ __launch_bounds__(kEvalBlock, WAVES) void batch_eval_kernel(const BatchDesc *D, const BatchRun *R,
                                                                       const BatchItem *items, uint32_t n_items,
                                                                       uint32_t *counter) {
  __shared__ __align__(16) unsigned char stage[kEvalBlock / 64][sizeof(Stage<A, P>)];
  const int lane = threadIdx.x & 63;
  const int warp = threadIdx.x >> 6;
  void *lds = stage[warp];
  while (true) {
    uint32_t next = 0;
    if (lane == 0) next = atomicAdd(counter, 1u);
    next = __builtin_amdgcn_readfirstlane(next);
    if (next >= n_items) break;  // every wave reaches this once the queue is drained
    const BatchItem it = items[next];
    const BatchDesc &d = D[it.poly];
    if (d.kind != KIND) continue;
    const typename A::M &m = member_mod<A>(d);
    void *out = R[it.poly].out;
    switch (d.K) {
      case 1: if constexpr (KLO <= 1 && 1 <= KHI) batch_eval_item<A, 1, P>(d, it, out, lds, lane, m); break;
      case 2: if constexpr (KLO <= 2 && 2 <= KHI) batch_eval_item<A, 2, P>(d, it, out, lds, lane, m); break;
      case 4: if constexpr (KLO <= 4 && 4 <= KHI) batch_eval_item<A, 4, P>(d, it, out, lds, lane, m); break;
      case 8: if constexpr (KLO <= 8 && 8 <= KHI) batch_eval_item<A, 8, P>(d, it, out, lds, lane, m); break;
      case 16: if constexpr (KLO <= 16 && 16 <= KHI) batch_eval_item<A, 16, P>(d, it, out, lds, lane, m); break;
      case 32: if constexpr (KLO <= 32 && 32 <= KHI) batch_eval_item<A, 32, P>(d, it, out, lds, lane, m); break;
      default: break;
    }
  }
}

// The kernel of each kind.  The FP64 product sums at most 8 doubles exactly,
// so its members are planned with K <= 8; 32 running values per thread are
// held for 32-bit residues only.  Waves per SIMD: those of the widest
// single-polynomial kernel of the range (the 64-bit K = 16 one needs
// three to issue nearly every cycle).
using BatchEvalFn = void (*)(const BatchDesc *, const BatchRun *, const BatchItem *, uint32_t, uint32_t *);
template <int P>
inline BatchEvalFn batch_eval_fn_p(uint32_t kind) {
  switch (kind) {
    case kKindW64K16: return batch_eval_kernel<W64, 16, 16, P, kind_waves(kKindW64K16, P), kKindW64K16>;
    case kKindW64Lo: return batch_eval_kernel<W64, 1, 8, P, kind_waves(kKindW64Lo, P), kKindW64Lo>;
    case kKindF64: return batch_eval_kernel<WF64, 1, 8, P, kind_waves(kKindF64, P), kKindF64>;
    case kKindW32K32: return batch_eval_kernel<W32, 32, 32, P, kind_waves(kKindW32K32, P), kKindW32K32>;
    default: return batch_eval_kernel<W32, 1, 16, P, kind_waves(kKindW32Lo, P), kKindW32Lo>;
  }
}
// P: evaluations per pass, 8 or 16
inline BatchEvalFn batch_eval_fn(uint32_t kind, uint32_t P) {
  return P == 8 ? batch_eval_fn_p<8>(kind) : batch_eval_fn_p<16>(kind);
}

// Flattened combine tiles: member j owns its tiles from prefix[j] on (the
// members of one kind together), ordered (evaluation tile, chain, group
// tile) with the group tile fastest.
template <class A>
__device__ __forceinline__ void batch_combine_one(const BatchDesc &d, void *out, uint64_t local, const typename A::M &m,
                                                  void *lds) {
  using T = typename A::T;
  CombineArgs<A> a;
  a.partial = (const T *)d.partial;
  a.slot_off = d.slot_off;
  a.out = (T *)out;
  a.G = d.G;
  a.C = d.C;
  a.T = d.T;
  a.Lmax = d.Lmax;
  a.m = m;
  const uint64_t gt = (d.G + kCombineTile - 1) / kCombineTile;
  const uint64_t g_tile = local % gt;
  const uint64_t rest = local / gt;
  const uint32_t c = (uint32_t)(rest % d.C);
  const uint32_t i_tile = (uint32_t)(rest / d.C);
  combine_tile<A>(a, g_tile * kCombineTile, c, i_tile * kCombineTile,
                  reinterpret_cast<T(*)[kCombineTile + 1]>(lds));
}

// One tile per block; the tile's member from a table (uniform over the block).
__global__ __launch_bounds__(kCombineBlock) void batch_combine_kernel(const BatchDesc *__restrict__ D,
                                                                      const BatchRun *__restrict__ R,
                                                                      const uint32_t *__restrict__ tile_member,
                                                                      const uint64_t *__restrict__ prefix, uint64_t base) {
  __shared__ __align__(16) uint64_t tile[kCombineTile][kCombineTile + 1];
  const uint64_t idx = base + blockIdx.x;  // the grid is exactly tiles base .. base + gridDim.x - 1
  const uint32_t j = __builtin_amdgcn_readfirstlane(tile_member[idx]);
  const BatchDesc &d = D[j];
  const uint64_t local = idx - prefix[j];
  if (d.w == 4) batch_combine_one<W32>(d, R[j].out, local, d.m32, tile);
  else batch_combine_one<W64>(d, R[j].out, local, d.m64, tile);
}

}  // namespace peval
