// Shared machinery of batched launches (used by peval_batch_* and the server).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "batch_types.hpp"
#include "peval_internal.hpp"

namespace peval {

struct BatchMember {
  peval_poly *h;
  Plan *plan;
  uint32_t C;  // chains
  uint32_t T;  // evaluations
};

// Device state of one batched pass.
// Side streams on which the kernels of the second and later kinds of member
// run beside the first kind's (forked after the power tables, joined at the
// end of the pass; see batch_enqueue).  Every wait is on an event recorded
// earlier in submission order, so streams sharing a hardware queue only
// lose overlap, never progress.  Owned by whoever owns the launches.
struct BatchFork {
  hipStream_t aux[kKinds] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kKinds] = {};
  int create();   // PEVAL_OK or an error; default-priority non-blocking streams
  void destroy();
};

struct BatchCore {
  uint32_t count = 0;
  uint32_t n_items = 0;
  uint32_t kind_first[kKinds + 1] = {};  // items of kind k: kind_first[k] .. kind_first[k+1]-1
  int eval_blocks[kKinds] = {};          // persistent blocks of each kind's evaluation kernel
  uint32_t kind_p[kKinds] = {};          // evaluations per pass of each kind's kernel (8 or 16)
  uint64_t tab_total = 0, mono_total = 0, out_total = 0;
  uint64_t mono_blocks = 0;  // blocks of the monomial kernel (each member's entries padded to whole blocks)
  uint64_t kind_mono[kKinds + 1] = {};   // monomial blocks of kind k: kind_mono[k] .. kind_mono[k+1]-1
  uint64_t kind_tiles[kKinds + 1] = {};  // combine tiles of kind k, likewise
  size_t scratch_bytes = 0;
  std::vector<BatchDesc> descs;
  void *d_blob = nullptr;  // descriptors, run table, items, prefixes, queue counter
  BatchDesc *d_desc = nullptr;
  BatchRun *d_run = nullptr;
  BatchItem *d_items = nullptr;
  uint64_t *d_ptab = nullptr, *d_pmono = nullptr, *d_pout = nullptr;
  uint32_t *d_bmono = nullptr, *d_bout = nullptr;  // member of each monomial block, of each combine tile
  uint32_t *d_counter = nullptr;
  void *arena = nullptr;  // per-member scratch
  bool own_arena = false;
  // host image of the blob and its layout
  std::vector<char> image;
  size_t blob_bytes = 0;
  size_t off_desc = 0, off_run = 0, off_items = 0, off_ptab = 0, off_pmono = 0, off_pout = 0, off_ctr = 0;
  size_t off_bmono = 0, off_bout = 0;
};

size_t member_scratch_bytes(const peval_poly *h, const Plan &pl, uint32_t C, uint32_t T);
uint32_t member_chains(const Plan &pl, uint32_t T, double target_cost);
uint32_t member_kind(const peval_poly *h, uint32_t K);
// Chains of every member from its kind's work, items' target cost times scale.
int batch_chains(std::vector<BatchMember> &mem, double scale);
size_t batch_scratch_need(const std::vector<BatchMember> &mem);
// Host planning: descriptors pointing into `arena` (batch_scratch_need bytes),
// work items in decreasing cost, prefixes, and the blob image (with the run
// table if `runs` is given).  No device call.
void batch_plan(BatchCore &b, const std::vector<BatchMember> &mem, void *arena, const BatchRun *runs);
// Points the device-side fields at a blob allocation holding the image.
void batch_bind(BatchCore &b, void *d_blob);
// Allocates scratch and blob with hipMalloc and uploads the image.  Handles
// must stay alive while the batch is used.
// kind_p: evaluations per pass per kind (nullptr: each kind's default).
int batch_build(BatchCore &b, const std::vector<BatchMember> &mem, const uint32_t *kind_p = nullptr);
// fork: optional side streams, one per kind of member (nullptr: all on st)
int batch_enqueue(const BatchCore &b, hipStream_t st, const BatchFork *fork = nullptr);
void batch_release(BatchCore &b);
// Persistent blocks of the evaluation kernels for this batch's items.
int batch_set_blocks(BatchCore &b);

}  // namespace peval
