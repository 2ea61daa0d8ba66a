// Data structures shared by the batched launch and the server (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace peval {

constexpr int kBatchP = 16;  // evaluations per pass in batched launches

// Product a member's evaluations take; one work queue and one persistent
// evaluation kernel per kind.
enum BatchKind : uint32_t {
  kKindW64 = 0,  // 64-bit residues, Shoup product
  kKindF64 = 1,  // 64-bit residues, FP64 product (Alg. 2, 2^31 <= p < 2^50)
  kKindW32 = 2,  // 32-bit residues, Shoup product
  kKinds = 3
};

// Static part of one polynomial in a batch (device table).
struct BatchDesc {
  uint32_t w, ntail, K, C, T, Lmax;
  uint32_t kind, pad;
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
