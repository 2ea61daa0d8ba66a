// Batched evaluation: many resident polynomials, uneven sizes, mixed moduli,
// one persistent launch captured in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "batch_internal.hpp"
#include "batch_kernels.hpp"
#include "errors.hpp"
#include "peval.h"
#include "peval_internal.hpp"

namespace peval {

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void batch_release(BatchCore &b) {
  if (b.d_blob) (void)hipFree(b.d_blob);
  if (b.arena && b.own_arena) (void)hipFree(b.arena);
  b.d_blob = nullptr;
  b.arena = nullptr;
}

// Blocks that fill the chip with each kind's evaluation kernel.
// Blocks of each kind's evaluation kernel that the chip holds at once, for
// its pass size (occupancy x CUs; per (kind, P), cached).
static int persistent_blocks(int blocks[kKinds], const uint32_t *kind_p = nullptr) {
  static int cached[kKinds][2] = {};
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[0][0]) {
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    for (uint32_t k = 0; k < kKinds; ++k)
      for (int i = 0; i < 2; ++i) {
        int per_cu = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_eval_fn(k, kKindPOptions[i]),
                                                             kEvalBlock, 0));
        cached[k][i] = std::max(1, per_cu) * prop.multiProcessorCount;
      }
  }
  for (uint32_t k = 0; k < kKinds; ++k) {
    const uint32_t P = kind_p ? kind_p[k] : (uint32_t)kind_P(k);
    blocks[k] = cached[k][P == kKindPOptions[0] ? 0 : 1];
  }
  return PEVAL_OK;
}

int batch_set_blocks(BatchCore &b) {
  for (uint32_t k = 0; k < kKinds; ++k)
    if (!b.kind_p[k]) b.kind_p[k] = kind_P(k);
  int bl[kKinds];
  PEVAL_TRY(persistent_blocks(bl, b.kind_p));
  for (int k = 0; k < kKinds; ++k) {
    const uint64_t n = (uint64_t)b.kind_first[k + 1] - b.kind_first[k];
    b.eval_blocks[k] = (int)std::min<uint64_t>((uint64_t)bl[k], (n + 3) / 4);
  }
  return PEVAL_OK;
}

// The product a member's evaluations take: that of its handle when the
// batch is planned (FP64 where the handle's arithmetic resolves to it and
// the plan keeps K <= 8, so that a thread's sum of doubles stays exact;
// the Shoup product, exact for every p, otherwise); and the kernel of its K.
uint32_t member_kind(const peval_poly *h, uint32_t K) {
  if (h->w == 4) return K == 32 ? kKindW32K32 : kKindW32Lo;
  if (h->arith == 1 && K <= 8) return kKindF64;
  return K == 16 ? kKindW64K16 : kKindW64Lo;
}

// Bytes of device scratch one member needs (power tables, chain starts,
// Gamma, Gamma', partial sums).
// A member whose groups all fit in one thread's K terms (thread j holds
// group j) has its images written by the evaluation kernel.
static bool member_direct(const peval_poly *h, const Plan &pl) { return (uint64_t)pl.K >= h->max_group; }

size_t member_scratch_bytes(const peval_poly *h, const Plan &pl, uint32_t C, uint32_t T) {
  const size_t w = h->w;
  size_t b = 0;
  b += align_up((size_t)std::max<uint32_t>(h->tab_total, 1) * w, 256) * 2;
  b += align_up((size_t)C * pl.K * pl.NT * w, 256);
  b += align_up((size_t)pl.K * pl.NT * w, 256) * 2;
  const size_t lmax = ((size_t)T + C - 1) / C;
  if (!member_direct(h, pl)) b += align_up((size_t)C * lmax * pl.nslots * w, 256);
  return b;
}

// Chains for one member so that its work items cost about target_cost
// term-evaluations each, but no more than keep each chain's start (about
// 2 log2 T + 2 products per term in the monomial kernel) below a quarter of
// its rows: a lone large member otherwise got so many chains that its
// chain starts cost as much as its evaluations.
uint32_t member_chains(const Plan &pl, uint32_t T, double target_cost) {
  double per_chain_full = 64.0 * pl.K * T;  // one wave, one chain over all T
  double c = std::ceil(per_chain_full / std::max(target_cost, 1.0));
  c = std::min(c, std::floor(T / (4.0 * (2.0 * std::log2(std::max<double>(T, 2.0)) + 2.0))));
  c = std::min<double>(std::max(c, 1.0), std::min<uint32_t>(T, 256));
  return (uint32_t)c;
}

// Chains of every member: each kind's kernel runs on its own, so each kind
// sizes its work items from its own work: about eight items per wave slot
// of its kernel on the chip (so that the last items, the smallest, leave
// little idle), none below one wave's 64 x 8 x 64 term-evaluations, times
// `scale`.  One target for the whole batch left a kind with little work too
// few items to fill the chip, waiting on its longest one.
int batch_chains(std::vector<BatchMember> &mem, double scale) {
  int blocks[kKinds];
  PEVAL_TRY(persistent_blocks(blocks));
  double work[kKinds] = {};
  for (const auto &m : mem) work[member_kind(m.h, m.plan->K)] += 64.0 * m.plan->K * m.plan->NW * m.T;
  for (auto &m : mem) {
    const uint32_t k = member_kind(m.h, m.plan->K);
    const double slots = (double)blocks[k] * (kEvalBlock / 64);  // waves of the kernel on the chip
    const double target = std::max(work[k] / (8.0 * slots), 64.0 * 8 * 64) * scale;
    m.C = member_chains(*m.plan, m.T, target);
  }
  return PEVAL_OK;
}

size_t batch_scratch_need(const std::vector<BatchMember> &mem) {
  size_t need = 0;
  for (const auto &m : mem) need += member_scratch_bytes(m.h, *m.plan, m.C, m.T);
  return need;
}

void batch_plan(BatchCore &b, const std::vector<BatchMember> &mem, void *arena, const BatchRun *runs) {
  const uint32_t count = (uint32_t)mem.size();
  b.count = count;
  b.descs.assign(count, BatchDesc{});
  std::vector<uint64_t> ptab(count + 1, 0), pmono(count + 1, 0), pout(count + 1, 0), mblocks(count), tiles(count);
  std::vector<BatchItem> items;
  b.scratch_bytes = batch_scratch_need(mem);
  b.arena = arena;
  char *cur = (char *)arena;
  auto take = [&](size_t bytes) {
    void *p = cur;
    cur += align_up(bytes, 256);
    return p;
  };
  for (uint32_t j = 0; j < count; ++j) {
    const peval_poly *h = mem[j].h;
    const Plan &pl = *mem[j].plan;
    BatchDesc &d = b.descs[j];
    const size_t w = h->w;
    d.w = h->w;
    d.kind = member_kind(h, pl.K);
    d.ntail = h->n - 2;
    d.K = pl.K;
    d.C = mem[j].C;
    d.T = mem[j].T;
    d.Lmax = (d.T + d.C - 1) / d.C;
    d.s = h->s;
    d.NT = pl.NT;
    d.NW = pl.NW;
    d.nslots = pl.nslots;
    d.G = h->G;
    d.m64 = h->m64;
    d.m32 = h->m32;
    d.mf = h->mf;
    d.to = h->tab;
    d.tab_total = h->tab_total;
    d.coeff = h->d_coeff;
    d.exps = h->d_exps;
    d.tval = take((size_t)std::max<uint32_t>(h->tab_total, 1) * w);
    d.tquot = take((size_t)std::max<uint32_t>(h->tab_total, 1) * w);
    d.thr_first = pl.d_thr_first;
    d.thr_cnt = pl.d_thr_cnt;
    d.endmask = pl.d_endmask;
    d.slot_base = pl.d_slot_base;
    d.slot_off = pl.d_slot_off;
    d.direct = member_direct(h, pl) ? 1 : 0;
    d.lam = take((size_t)d.C * pl.K * pl.NT * w);
    d.gam = take((size_t)pl.K * pl.NT * w);
    d.gamq = take((size_t)pl.K * pl.NT * w);
    d.partial = d.direct ? nullptr : take((size_t)d.C * d.Lmax * pl.nslots * w);
    ptab[j + 1] = ptab[j] + (d.ntail ? h->tab_total : 0);
    // whole blocks per member, so that a block's member is one table entry
    mblocks[j] = align_up((size_t)pl.K * pl.NT / mono_slots(pl.K), kMonoBlock) / kMonoBlock;
    // combine tiles; none for a direct member
    tiles[j] = d.direct ? 0
                        : ((h->G + kCombineTile - 1) / kCombineTile) * d.C *
                              (((uint64_t)d.Lmax + kCombineTile - 1) / kCombineTile);
  }
  // monomial blocks and combine tiles grouped by kind (each kind's members
  // in index order), so that every kind's range is contiguous: pmono[j] and
  // pout[j] are member j's first entry and first tile
  uint64_t mcur = 0, tcur = 0;
  for (uint32_t kind = 0; kind < kKinds; ++kind) {
    b.kind_mono[kind] = mcur / kMonoBlock;
    b.kind_tiles[kind] = tcur;
    for (uint32_t j = 0; j < count; ++j) {
      if (b.descs[j].kind != kind) continue;
      pmono[j] = mcur;
      pout[j] = tcur;
      mcur += mblocks[j] * kMonoBlock;
      tcur += tiles[j];
    }
  }
  b.kind_mono[kKinds] = mcur / kMonoBlock;
  b.kind_tiles[kKinds] = tcur;
  pmono[count] = mcur;
  pout[count] = tcur;
  // Work items, biggest first.  An item costs K x (evaluations of its chain);
  // within one member the chains differ by at most one evaluation, so
  // ordering members by K x Lmax and emitting each member's items chain by
  // chain gives the decreasing order without sorting every item.
  std::vector<uint32_t> order(count);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    return (uint64_t)b.descs[x].K * b.descs[x].Lmax > (uint64_t)b.descs[y].K * b.descs[y].Lmax;
  });
  uint64_t n_items = 0;
  for (uint32_t j = 0; j < count; ++j) n_items += (uint64_t)b.descs[j].C * b.descs[j].NW;
  items.reserve(n_items);
  // items grouped by kind (one queue and one evaluation kernel per kind),
  // each group in decreasing cost
  for (uint32_t kind = 0; kind < kKinds; ++kind) {
    b.kind_first[kind] = (uint32_t)items.size();
    for (uint32_t j : order) {
      if (b.descs[j].kind != kind) continue;
      for (uint32_t c = 0; c < b.descs[j].C; ++c)
        for (uint64_t wv = 0; wv < b.descs[j].NW; ++wv) items.push_back(BatchItem{j, (uint32_t)wv, c, 0});
    }
  }
  b.kind_first[kKinds] = (uint32_t)items.size();
  b.n_items = (uint32_t)items.size();
  b.tab_total = ptab[count];
  b.mono_total = pmono[count];
  b.out_total = pout[count];
  b.mono_blocks = b.mono_total / kMonoBlock;
  std::vector<uint32_t> bmono(b.mono_blocks), bout(b.out_total);
  for (uint32_t j = 0; j < count; ++j) {
    std::fill(bmono.begin() + pmono[j] / kMonoBlock, bmono.begin() + pmono[j] / kMonoBlock + mblocks[j], j);
    std::fill(bout.begin() + pout[j], bout.begin() + pout[j] + tiles[j], j);
  }

  // blob image: descriptors, runs, items, prefixes, queue counter
  b.off_desc = 0;
  b.off_run = align_up(b.off_desc + count * sizeof(BatchDesc), 256);
  b.off_items = align_up(b.off_run + count * sizeof(BatchRun), 256);
  b.off_ptab = align_up(b.off_items + std::max<size_t>(items.size(), 1) * sizeof(BatchItem), 256);
  b.off_pmono = align_up(b.off_ptab + (count + 1) * 8, 256);
  b.off_pout = align_up(b.off_pmono + (count + 1) * 8, 256);
  b.off_bmono = align_up(b.off_pout + (count + 1) * 8, 256);
  b.off_bout = align_up(b.off_bmono + bmono.size() * 4, 256);
  b.off_ctr = align_up(b.off_bout + bout.size() * 4, 256);
  b.blob_bytes = b.off_ctr + 256;
  b.image.assign(b.blob_bytes, 0);
  char *img = b.image.data();
  memcpy(img + b.off_desc, b.descs.data(), count * sizeof(BatchDesc));
  if (runs) memcpy(img + b.off_run, runs, count * sizeof(BatchRun));
  if (!items.empty()) memcpy(img + b.off_items, items.data(), items.size() * sizeof(BatchItem));
  memcpy(img + b.off_ptab, ptab.data(), (count + 1) * 8);
  memcpy(img + b.off_pmono, pmono.data(), (count + 1) * 8);
  memcpy(img + b.off_pout, pout.data(), (count + 1) * 8);
  if (!bmono.empty()) memcpy(img + b.off_bmono, bmono.data(), bmono.size() * 4);
  if (!bout.empty()) memcpy(img + b.off_bout, bout.data(), bout.size() * 4);
}

void batch_bind(BatchCore &b, void *d_blob) {
  char *base = (char *)d_blob;
  b.d_blob = d_blob;
  b.d_desc = (BatchDesc *)(base + b.off_desc);
  b.d_run = (BatchRun *)(base + b.off_run);
  b.d_items = (BatchItem *)(base + b.off_items);
  b.d_ptab = (uint64_t *)(base + b.off_ptab);
  b.d_pmono = (uint64_t *)(base + b.off_pmono);
  b.d_pout = (uint64_t *)(base + b.off_pout);
  b.d_bmono = (uint32_t *)(base + b.off_bmono);
  b.d_bout = (uint32_t *)(base + b.off_bout);
  b.d_counter = (uint32_t *)(base + b.off_ctr);
}

int batch_build(BatchCore &b, const std::vector<BatchMember> &mem, const uint32_t *kind_p) {
  void *arena = nullptr, *blob = nullptr;
  size_t need = batch_scratch_need(mem);
  HIP_TRY(hipMalloc(&arena, std::max<size_t>(need, 256)));
  b.own_arena = true;
  batch_plan(b, mem, arena, nullptr);
  HIP_TRY(hipMalloc(&blob, b.blob_bytes));
  batch_bind(b, blob);
  HIP_TRY(hipMemcpy(blob, b.image.data(), b.blob_bytes, hipMemcpyHostToDevice));
  for (uint32_t k = 0; k < kKinds; ++k) b.kind_p[k] = kind_p ? kind_p[k] : (uint32_t)kind_P(k);
  return batch_set_blocks(b);
}

int BatchFork::create() {
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return fail(PEVAL_EDEVICE, "event creation");
  for (uint32_t k = 0; k < kKinds; ++k) {
    if (hipStreamCreateWithFlags(&aux[k], hipStreamNonBlocking) != hipSuccess)
      return fail(PEVAL_EDEVICE, "stream creation");
    if (hipEventCreateWithFlags(&join[k], hipEventDisableTiming) != hipSuccess)
      return fail(PEVAL_EDEVICE, "event creation");
  }
  return PEVAL_OK;
}

void BatchFork::destroy() {
  for (uint32_t k = 0; k < kKinds; ++k) {
    if (aux[k]) (void)hipStreamDestroy(aux[k]);
    if (join[k]) (void)hipEventDestroy(join[k]);
    aux[k] = nullptr;
    join[k] = nullptr;
  }
  if (fork) (void)hipEventDestroy(fork);
  fork = nullptr;
}

// Monomial blocks [b0, b1) and combine tiles [t0, t1) of one batched pass.
static int enqueue_mono(const BatchCore &b, hipStream_t st, uint64_t b0, uint64_t b1) {
  if (b1 <= b0) return PEVAL_OK;
  const uint32_t xchunk = (uint32_t)((b1 - b0 + kXcds - 1) / kXcds);
  batch_mono_kernel<<<kXcds * xchunk, kMonoBlock, 0, st>>>(b.d_desc, b.d_run, b.d_bmono, b.d_pmono, b0, b1 - b0,
                                                           xchunk);
  HIP_TRY(hipGetLastError());
  return PEVAL_OK;
}

static int enqueue_combine(const BatchCore &b, hipStream_t st, uint64_t t0, uint64_t t1) {
  if (t1 <= t0) return PEVAL_OK;
  batch_combine_kernel<<<(unsigned)(t1 - t0), kCombineBlock, 0, st>>>(b.d_desc, b.d_run, b.d_bout, b.d_pout, t0);
  HIP_TRY(hipGetLastError());
  return PEVAL_OK;
}

static int enqueue_eval(const BatchCore &b, hipStream_t st, uint32_t kind) {
  const uint32_t first = b.kind_first[kind], n = b.kind_first[kind + 1] - first;
  if (!n) return PEVAL_OK;
  batch_eval_fn(kind, b.kind_p[kind])<<<b.eval_blocks[kind], kEvalBlock, 0, st>>>(b.d_desc, b.d_run,
                                                                                    b.d_items + first, n,
                                                                                    b.d_counter + kind);
  HIP_TRY(hipGetLastError());
  return PEVAL_OK;
}

// Kernels of one batched pass (the run table must already be on the device).
// With side streams (fork) and more than one kind of member, each kind's
// monomial, evaluation and combine kernels run in order on a stream of their
// own, the streams side by side after the power tables: one kind's
// memory-bound monomial and combine kernels overlap another kind's ALU-bound
// evaluation, and each evaluation kernel's last items drain while other
// kernels take the freed CUs.  Without, all kernels follow one another on st.
int batch_enqueue(const BatchCore &b, hipStream_t st, const BatchFork *fork) {
  batch_reset_kernel<<<1, 64, 0, st>>>(b.d_counter);
  HIP_TRY(hipGetLastError());
  if (b.tab_total) {
    batch_power_kernel<<<(unsigned)((b.tab_total + 255) / 256), 256, 0, st>>>(b.d_desc, b.d_run, b.count, b.d_ptab);
    HIP_TRY(hipGetLastError());
  }
  uint32_t kinds_present = 0;
  for (uint32_t kind = 0; kind < kKinds; ++kind) kinds_present += b.kind_first[kind + 1] > b.kind_first[kind];
  if (!fork || kinds_present < 2) {
    PEVAL_TRY(enqueue_mono(b, st, 0, b.mono_blocks));
    for (uint32_t kind = 0; kind < kKinds; ++kind) PEVAL_TRY(enqueue_eval(b, st, kind));
    return enqueue_combine(b, st, 0, b.out_total);
  }
  HIP_TRY(hipEventRecord(fork->fork, st));  // reset and power tables done
  bool joins[kKinds] = {}, first_kind = true;
  for (uint32_t kind = 0; kind < kKinds; ++kind) {
    if (b.kind_first[kind + 1] == b.kind_first[kind]) continue;
    hipStream_t ks = st;
    if (!first_kind) {
      ks = fork->aux[kind];
      HIP_TRY(hipStreamWaitEvent(ks, fork->fork, 0));
    }
    first_kind = false;
    PEVAL_TRY(enqueue_mono(b, ks, b.kind_mono[kind], b.kind_mono[kind + 1]));
    PEVAL_TRY(enqueue_eval(b, ks, kind));
    PEVAL_TRY(enqueue_combine(b, ks, b.kind_tiles[kind], b.kind_tiles[kind + 1]));
    if (ks != st) {
      HIP_TRY(hipEventRecord(fork->join[kind], ks));
      joins[kind] = true;
    }
  }
  for (uint32_t kind = 0; kind < kKinds; ++kind)
    if (joins[kind]) HIP_TRY(hipStreamWaitEvent(st, fork->join[kind], 0));
  return PEVAL_OK;
}

}  // namespace peval

using namespace peval;

constexpr int kRunSlots = 4;  // run tables staged in rotation, so that runs pipeline

struct peval_batch {
  BatchCore core;
  std::vector<peval_poly *> polys;
  std::vector<uint32_t> Ts;
  BatchRun *h_run[kRunSlots] = {};        // pinned staging for the run table
  hipEvent_t copied[kRunSlots] = {};      // its upload has been consumed
  bool slot_used[kRunSlots] = {};
  int next_slot = 0;
  hipStream_t cap_stream = nullptr;
  BatchFork fork;  // a stream per kind of member (see batch_enqueue)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool have_done = false;
  bool use_graph = true;
  uint32_t tune_trials = 0;  // passes timed by the batch tuner (0: not tuned)
  float tuned_ms = 0;        // the chosen plan's pass time while tuning
  std::mutex mu;
};

static void batch_free(peval_batch *b) {
  if (!b) return;
  if (b->have_done) (void)hipEventSynchronize(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  b->fork.destroy();
  if (b->done) (void)hipEventDestroy(b->done);
  for (int k = 0; k < kRunSlots; ++k) {
    if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
    if (b->h_run[k]) (void)hipHostFree(b->h_run[k]);
  }
  batch_release(b->core);
  delete b;
}

// ---------------------------------------------------------------------------
// planning and tuning of a batch
// ---------------------------------------------------------------------------
// Members whose tiles the tuner moves together: product and width (64-bit
// Shoup, FP64, 32-bit Shoup) times whether their own heuristic K is the
// largest the product allows (big groups) or smaller.
constexpr int kTuneClasses = 6;
static uint32_t k_max(const peval_poly *h) { return h->arith == 1 ? 8 : (h->w == 4 && h->arith == 0) ? 32 : 16; }
static int tune_class(const peval_poly *h, uint32_t K0) {
  const int prod = h->w == 4 ? 2 : (h->arith == 1 ? 1 : 0);
  return prod * 2 + (K0 >= k_max(h) ? 1 : 0);
}

struct BatchChoice {
  int shift[kTuneClasses] = {0, 0, 0, 0, 0, 0};  // K moved by this many doublings from its own choice
  double chain_scale = 1.0;                      // work items' target cost, relative to the default
  uint32_t kind_p[kKinds] = {kind_P(0), kind_P(1), kind_P(2), kind_P(3), kind_P(4)};  // evaluations per pass
};

// Members' plans for one choice: K from the tuning cache or the heuristic,
// moved by the class's shift (within 1 .. the product's largest K), then the
// chains that give items of similar cost.
static int plan_members(const std::vector<peval_poly *> &polys, const std::vector<uint32_t> &Ts,
                        const BatchChoice &ch, std::vector<BatchMember> &mem) {
  const uint32_t count = (uint32_t)polys.size();
  mem.assign(count, BatchMember{});
  for (uint32_t j = 0; j < count; ++j) {
    peval_poly *h = polys[j];
    std::lock_guard<std::mutex> lk(h->mu);
    const uint32_t K0 = choose_tuning(h, Ts[j]).K;
    uint32_t K = K0;
    const int sh = ch.shift[tune_class(h, K0)];
    for (int i = 0; i < sh && K < k_max(h); ++i) K *= 2;
    for (int i = 0; i > sh && K > 1; --i) K /= 2;
    Plan *pl = nullptr;
    PEVAL_TRY(get_plan(h, K, kBatchP, &pl));
    mem[j] = BatchMember{h, pl, 1, Ts[j]};
  }
  return batch_chains(mem, ch.chain_scale);
}

// Device time of one pass of a planned batch (base points 2, outputs in
// `outs`): the median of five passes timed one by one after a warm-up.
static int time_pass(const std::vector<BatchMember> &mem, const uint32_t *kind_p, const std::vector<void *> &outs,
                     hipStream_t st, const BatchFork *fork, float *ms) {
  constexpr int kTimed = 5;
  BatchCore core;
  int rc = batch_build(core, mem, kind_p);
  hipEvent_t ev[kTimed + 1] = {};
  if (rc == PEVAL_OK) {
    std::vector<BatchRun> runs(mem.size());
    for (size_t j = 0; j < mem.size(); ++j) {
      memset(&runs[j], 0, sizeof(BatchRun));
      for (uint32_t k = 0; k + 2 < mem[j].h->n; ++k) runs[j].beta.b[k] = 2;
      runs[j].t0 = 1;
      runs[j].out = outs[j];
    }
    do {
      if (hipMemcpy(core.d_run, runs.data(), runs.size() * sizeof(BatchRun), hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(PEVAL_EDEVICE, "tuning set-up");
        break;
      }
      for (auto &e : ev)
        if (rc == PEVAL_OK && hipEventCreate(&e) != hipSuccess) rc = fail(PEVAL_EDEVICE, "tuning set-up");
      if (rc != PEVAL_OK) break;
      if ((rc = batch_enqueue(core, st, fork)) != PEVAL_OK) break;
      if (hipEventRecord(ev[0], st) != hipSuccess) { rc = fail(PEVAL_EDEVICE, "event record"); break; }
      for (int r = 0; r < kTimed && rc == PEVAL_OK; ++r) {
        rc = batch_enqueue(core, st, fork);
        if (rc == PEVAL_OK && hipEventRecord(ev[r + 1], st) != hipSuccess) rc = fail(PEVAL_EDEVICE, "event record");
      }
      if (rc != PEVAL_OK) break;
      if (hipEventSynchronize(ev[kTimed]) != hipSuccess) { rc = fail(PEVAL_EDEVICE, "tuning timing"); break; }
      float t[kTimed];
      for (int r = 0; r < kTimed && rc == PEVAL_OK; ++r)
        if (hipEventElapsedTime(&t[r], ev[r], ev[r + 1]) != hipSuccess) rc = fail(PEVAL_EDEVICE, "tuning timing");
      if (rc != PEVAL_OK) break;
      std::sort(t, t + kTimed);
      *ms = t[kTimed / 2];
    } while (false);
  }
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(st);
  batch_release(core);
  return rc;
}

// Coordinate search over the classes' K shifts (one doubling either way),
// then over the items' target cost (half, double): the analogue for a batch
// of the paper's sweep of its tiling parameters.  Every candidate pass runs
// on the device into scratch outputs.
static int tune_batch(const std::vector<peval_poly *> &polys, const std::vector<uint32_t> &Ts, BatchChoice *best,
                      float *best_ms, uint32_t *trials) {
  const uint32_t count = (uint32_t)polys.size();
  std::vector<size_t> off(count + 1, 0);
  bool present[kTuneClasses] = {};
  for (uint32_t j = 0; j < count; ++j) {
    off[j + 1] = off[j] + (((size_t)Ts[j] * polys[j]->G * polys[j]->w + 255) & ~(size_t)255);
    std::lock_guard<std::mutex> lk(polys[j]->mu);
    present[tune_class(polys[j], choose_tuning(polys[j], Ts[j]).K)] = true;
  }
  void *obuf = nullptr;
  hipStream_t st = nullptr;
  HIP_TRY(hipMalloc(&obuf, std::max<size_t>(off[count], 256)));
  std::vector<void *> outs(count);
  for (uint32_t j = 0; j < count; ++j) outs[j] = (char *)obuf + off[j];
  int rc = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess ? PEVAL_OK
                                                                            : fail(PEVAL_EDEVICE, "stream creation");
  BatchFork fork;  // candidates run as the batch will
  if (rc == PEVAL_OK) rc = fork.create();
  *trials = 0;
  auto measure = [&](const BatchChoice &ch, float *ms) {
    std::vector<BatchMember> mem;
    int r = plan_members(polys, Ts, ch, mem);
    if (r == PEVAL_OK) r = time_pass(mem, ch.kind_p, outs, st, &fork, ms);
    ++*trials;
    return r;
  };
  *best = BatchChoice{};
  if (rc == PEVAL_OK) rc = measure(*best, best_ms);
  for (int c = 0; c < kTuneClasses && rc == PEVAL_OK; ++c) {
    if (!present[c]) continue;
    for (int d : {-1, 1}) {
      BatchChoice ch = *best;
      ch.shift[c] += d;
      float ms = 0;
      if ((rc = measure(ch, &ms)) != PEVAL_OK) break;
      if (ms < *best_ms * 0.99f) {  // a clear gain only: timings vary by about 1%
        *best = ch;
        *best_ms = ms;
      }
    }
  }
  for (double sc : {0.5, 2.0}) {
    if (rc != PEVAL_OK) break;
    BatchChoice ch = *best;
    ch.chain_scale = sc;
    float ms = 0;
    if ((rc = measure(ch, &ms)) != PEVAL_OK) break;
    if (ms < *best_ms * 0.99f) {
      *best = ch;
      *best_ms = ms;
    }
  }
  // then each present kind's evaluations per pass (8 or 16)
  bool kind_present[kKinds] = {};
  if (rc == PEVAL_OK) {
    std::vector<BatchMember> mem;
    rc = plan_members(polys, Ts, *best, mem);
    for (const auto &m : mem) kind_present[member_kind(m.h, m.plan->K)] = true;
  }
  for (uint32_t k = 0; k < kKinds && rc == PEVAL_OK; ++k) {
    if (!kind_present[k]) continue;
    BatchChoice ch = *best;
    ch.kind_p[k] = ch.kind_p[k] == kKindPOptions[0] ? kKindPOptions[1] : kKindPOptions[0];
    float ms = 0;
    if ((rc = measure(ch, &ms)) != PEVAL_OK) break;
    if (ms < *best_ms * 0.99f) {
      *best = ch;
      *best_ms = ms;
    }
  }
  fork.destroy();
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(obuf);
  return rc;
}

extern "C" int peval_batch_create(uint32_t count, peval_poly *const *polys, const uint32_t *Ts, uint32_t flags,
                                  peval_batch **out) {
  if (!out) return fail(PEVAL_EINVAL, "out is NULL");
  *out = nullptr;
  if (count == 0 || !polys || !Ts) return fail(PEVAL_EINVAL, "empty batch or null arrays");
  for (uint32_t j = 0; j < count; ++j) {
    if (!polys[j]) return fail(PEVAL_EINVAL, "polys[%u] is NULL", j);
    if (Ts[j] == 0) return fail(PEVAL_EINVAL, "Ts[%u] is 0", j);
    if ((uint64_t)Ts[j] * polys[j]->G > (1ull << 40)) return fail(PEVAL_EUNSUPPORTED, "T*G too large");
  }
  peval_batch *b = new (std::nothrow) peval_batch();
  if (!b) return fail(PEVAL_ENOMEM, "host allocation");
  b->polys.assign(polys, polys + count);
  b->Ts.assign(Ts, Ts + count);
  b->use_graph = !(flags & PEVAL_BATCH_NO_GRAPH);
  auto bail = [&](int rc) {
    batch_free(b);
    return rc;
  };

  // plans: K from the tuning cache or the heuristic (moved by the batch
  // tuner when asked); P is set by the member's kind and does not change
  // the layout
  BatchChoice choice;
  if (flags & PEVAL_BATCH_PASS8)
    for (auto &pk : choice.kind_p) pk = kKindPOptions[0];
  if (flags & PEVAL_BATCH_TUNE) {
    float ms = 0;
    int trc = tune_batch(b->polys, b->Ts, &choice, &ms, &b->tune_trials);
    if (trc != PEVAL_OK) return bail(trc);
    b->tuned_ms = ms;
  }
  std::vector<BatchMember> mem;
  int rc = plan_members(b->polys, b->Ts, choice, mem);
  if (rc != PEVAL_OK) return bail(rc);
  rc = batch_build(b->core, mem, choice.kind_p);
  if (rc != PEVAL_OK) return bail(rc);
  for (int k = 0; k < kRunSlots; ++k) {
    if (hipHostMalloc((void **)&b->h_run[k], count * sizeof(BatchRun), hipHostMallocDefault) != hipSuccess)
      return bail(fail(PEVAL_ENOMEM, "pinned staging"));
    memset(b->h_run[k], 0, count * sizeof(BatchRun));
    if (hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming) != hipSuccess)
      return bail(fail(PEVAL_EDEVICE, "event creation"));
  }
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
    return bail(fail(PEVAL_EDEVICE, "event creation"));
  if ((rc = b->fork.create()) != PEVAL_OK) return bail(rc);
  if (b->use_graph) {
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(PEVAL_EDEVICE, "stream creation"));
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail(fail(PEVAL_EDEVICE, "begin capture"));
    int erc = batch_enqueue(b->core, b->cap_stream, &b->fork);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (erc != PEVAL_OK) return bail(erc);
    if (e != hipSuccess) return bail(fail(PEVAL_EDEVICE, "end capture: %s", hipGetErrorString(e)));
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
      return bail(fail(PEVAL_EDEVICE, "graph instantiate"));
  }
  *out = b;
  return PEVAL_OK;
}

extern "C" int peval_batch_run(peval_batch *b, const uint64_t *const *betas, const uint64_t *t0s,
                               void *const *dev_outs, void *stream) {
  if (!b || !dev_outs) return fail(PEVAL_EINVAL, "null argument");
  const uint32_t count = b->core.count;
  for (uint32_t j = 0; j < count; ++j) {
    if (!dev_outs[j]) return fail(PEVAL_EINVAL, "dev_outs[%u] is NULL", j);
    if (b->polys[j]->n > 2 && (!betas || !betas[j])) return fail(PEVAL_EINVAL, "betas[%u] is NULL", j);
    if (t0s && t0s[j] < 1) return fail(PEVAL_EINVAL, "t0s[%u] must be >= 1", j);
  }
  std::lock_guard<std::mutex> lk(b->mu);
  hipStream_t st = (hipStream_t)stream;
  // staging slots rotate: only a slot whose upload (kRunSlots runs back) has
  // not been consumed yet makes the host wait
  const int slot = b->next_slot;
  b->next_slot = (slot + 1) % kRunSlots;
  if (b->slot_used[slot]) HIP_TRY(hipEventSynchronize(b->copied[slot]));
  for (uint32_t j = 0; j < count; ++j) {
    BatchRun &r = b->h_run[slot][j];
    memset(&r.beta, 0, sizeof r.beta);
    const peval_poly *h = b->polys[j];
    for (uint32_t k = 0; k + 2 < h->n; ++k) r.beta.b[k] = betas[j][k] % h->p;
    r.t0 = t0s ? t0s[j] : 1;
    r.out = dev_outs[j];
  }
  // runs share the device run table and scratch: a run on another stream
  // starts after the previous one on the device, not on the host
  if (b->have_done) HIP_TRY(hipStreamWaitEvent(st, b->done, 0));
  HIP_TRY(hipMemcpyAsync(b->core.d_run, b->h_run[slot], count * sizeof(BatchRun), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(b->copied[slot], st));
  b->slot_used[slot] = true;
  if (b->use_graph) {
    HIP_TRY(hipGraphLaunch(b->exec, st));
  } else {
    PEVAL_TRY(batch_enqueue(b->core, st, &b->fork));
  }
  HIP_TRY(hipEventRecord(b->done, st));
  b->have_done = true;
  return PEVAL_OK;
}

extern "C" int peval_batch_info(const peval_batch *b, uint64_t *info) {
  if (!b || !info) return fail(PEVAL_EINVAL, "null argument");
  info[0] = b->core.count;
  info[1] = b->core.n_items;
  info[2] = 0;
  for (int k = 0; k < kKinds; ++k) info[2] += (uint64_t)b->core.eval_blocks[k];
  info[3] = b->core.scratch_bytes;
  uint64_t te = 0;
  for (uint32_t j = 0; j < b->core.count; ++j) te += b->polys[j]->s * (uint64_t)b->Ts[j];
  info[4] = te;
  return PEVAL_OK;
}

extern "C" int peval_batch_members(const peval_batch *b, uint32_t *K, uint32_t *C, uint32_t *kind, float *tuned_ms,
                                   uint32_t *tune_trials) {
  if (!b) return fail(PEVAL_EINVAL, "null batch");
  for (uint32_t j = 0; j < b->core.count; ++j) {
    if (K) K[j] = b->core.descs[j].K;
    if (C) C[j] = b->core.descs[j].C;
    if (kind) kind[j] = b->core.descs[j].kind;
  }
  if (tuned_ms) *tuned_ms = b->tuned_ms;
  if (tune_trials) *tune_trials = b->tune_trials;
  return PEVAL_OK;
}

extern "C" int peval_batch_kinds(const peval_batch *b, uint32_t *P, uint32_t *blocks) {
  if (!b || !P || !blocks) return fail(PEVAL_EINVAL, "null argument");
  for (uint32_t k = 0; k < kKinds; ++k) {
    const bool present = b->core.kind_first[k + 1] > b->core.kind_first[k];
    P[k] = present ? b->core.kind_p[k] : 0;
    blocks[k] = present ? (uint32_t)b->core.eval_blocks[k] : 0;
  }
  return PEVAL_OK;
}

extern "C" int peval_batch_destroy(peval_batch *b) {
  batch_free(b);
  return PEVAL_OK;
}
