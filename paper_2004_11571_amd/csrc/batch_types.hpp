// Data structures shared by the batched launch and the server (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace peval {

constexpr int kBatchP = 16;  // evaluations per pass in batched launches (all kinds but kKindW64Lo)

// The product a member's evaluations take and the range of its terms per
// thread K.  Each kind has its own work queue and persistent evaluation
// kernel, compiled for that K range only, so that it gets the registers
// (and waves per SIMD) of its own widest member rather than those of the
// widest of all: one kernel for every 64-bit K held two waves per SIMD,
// where the K = 16 evaluation alone fits three.
enum BatchKind : uint32_t {
  kKindW64K16 = 0,  // 64-bit residues, Shoup product, K = 16
  kKindW64Lo = 1,   // 64-bit residues, Shoup product, K <= 8; 8 evaluations per pass
  kKindF64 = 2,     // 64-bit residues, FP64 product (Alg. 2, 2^31 <= p < 2^50), K <= 8
  kKindW32K32 = 3,  // 32-bit residues, K = 32
  kKindW32Lo = 4,   // 32-bit residues, K <= 16
  kKinds = 5
};

// Evaluations per pass of a kind's kernel by default: the small-K 64-bit
// kernel stages 8, so that its stage leaves room for more waves per CU.
// Every kind is compiled for 8 and 16 (the batch tuner picks one per kind);
// 32 would leave one or two blocks per CU for the stages in LDS.
__host__ __device__ constexpr int kind_P(uint32_t kind) { return kind == kKindW64Lo ? 8 : kBatchP; }
constexpr uint32_t kKindPOptions[2] = {8, 16};
// Waves per SIMD a kind's kernel is compiled for (its register bound): the
// 32-bit K = 32 one holds 96 running values, Gammas and quotients and needs
// about 200 registers (two waves; with three it spilled over a hundred); the
// small-K 64-bit one fits four with 8 evaluations per pass, three with 16.
__host__ __device__ constexpr int kind_waves(uint32_t kind, int P) {
  return kind == kKindW32K32 ? 2 : kind == kKindW64K16 ? 3 : (kind == kKindW64Lo && P > 8) ? 3 : 4;
}

// Static part of one polynomial in a batch (device table).
struct BatchDesc {
  uint32_t w, ntail, K, C, T, Lmax;
  uint32_t kind;
  uint32_t direct;  // every group within one thread's K terms: images written by the evaluation kernel
  uint64_t s, NT, NW, nslots, G;
  Mod64 m64;
  Mod32 m32;
  ModF64 mf;
  TableOffsets to;
  uint32_t tab_total;
  const void *coeff;
  const uint16_t *exps;
  void *tval, *tquot;
  const uint32_t *thr_first;
  const uint8_t *thr_cnt;
  const uint64_t *endmask;
  const uint32_t *slot_base;
  const uint32_t *slot_off;
  void *lam, *gam, *gamq, *partial;
};

// Per-launch part (device table, refreshed before every launch).
struct BatchRun {
  BetaArg beta;   // reduced base point
  uint64_t t0;    // first evaluation index
  void *out;      // T x G residues
};

struct BatchItem {
  uint32_t poly, wave, chain, pad;
};

}  // namespace peval
