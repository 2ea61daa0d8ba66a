// Serving loop: resident polynomials under an HBM budget, admission control,
// continuous batching of evaluation requests of different sizes.
//
// Requests are cut into slices of consecutive evaluations (a slice starts at
// its own t0, so its chain starts are a m^{t0+c}); every pass batches one
// slice of each admitted request into one batched launch (the same kernels
// as peval_batch).  Two passes are in flight on two streams, so requests
// that arrive while a pass runs join the next one, and finished requests
// leave as soon as their last slice is done.  Results are bit-identical to
// a plain run of the same request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch_internal.hpp"
#include "errors.hpp"
#include "peval.h"
#include "peval_internal.hpp"

using namespace peval;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SPoly {
  uint64_t id = 0;
  uint64_t p = 0;
  uint32_t n = 0, w = 8;
  uint64_t s = 0, G = 0;
  uint64_t tab_total = 0;      // power-table entries (sum of tail degrees + 1)
  uint32_t max_exp[32] = {0};  // largest exponent of each variable
  std::vector<uint32_t> exps;  // host copy for re-upload after eviction
  std::vector<uint64_t> coeffs;
  peval_poly *h = nullptr;     // resident handle (null when not resident)
  Plan *plan = nullptr;        // its thread layout for batched passes
  uint64_t bytes = 0;          // device bytes while resident
  uint64_t last_used = 0;
  uint32_t refs = 0;           // admitted requests using it
  bool removed = false;
  bool uploading = false;      // queued for (or in) an upload by an uploader thread
};

struct SReq {
  uint64_t id = 0, poly = 0;
  std::vector<uint64_t> beta;
  uint32_t T = 0;
  void *host_out = nullptr;
  double t_submit = 0, t_done = 0;
  uint32_t t_next = 1;        // next evaluation to launch
  uint32_t launched_passes = 0, finished_passes = 0;
  void *d_out = nullptr;
  uint64_t out_bytes = 0;
  uint64_t out_alloc = 0;     // size of the pooled output block
  uint64_t reserve = 0;       // scratch reserved for its slices while admitted
  uint32_t ts = 0;            // evaluations per slice
  uint32_t cmax = 1;          // chains per slice allowed by the reservation
  bool admitted = false;
  int status = 1;             // 1 pending, 0 done, < 0 error
};

struct Pass {
  int slot = 0;
  double t_launch = 0, t_sim_end = 0;
  std::vector<uint64_t> reqs;  // requests with a slice in this pass
  uint64_t term_evals = 0;
};

constexpr int kStreams = 2;
constexpr int kUploaders = 4;  // threads making polynomials resident (each ingest is multi-threaded itself)

}  // namespace

struct peval_server {
  uint64_t budget = 0;
  bool simulate = false;
  double sim_rate = 1.0e12;          // simulated term-evaluations per second
  double slice_work = 2.0e9;         // target term-evaluations per request slice
  double pass_work = 1.5e10;         // term-evaluations per pass (bounds the latency one pass adds)
  uint32_t max_members = 512;        // slices per pass (bounds the host work of one pass)
  uint64_t slices = 0;               // stats: slices launched
  double host_pass_s = 0;            // stats: scheduler time spent building and launching passes
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  int device = 0;

  std::map<uint64_t, SPoly> polys;
  std::map<uint64_t, SReq> reqs;
  std::deque<uint64_t> pending;      // submitted, not admitted (FIFO)
  std::vector<uint64_t> active;      // admitted, not finished
  std::deque<Pass> inflight;
  uint64_t next_id = 1, clock = 0;
  uint64_t used = 0, peak = 0;       // budget accounting
  // stats
  uint64_t submitted = 0, completed = 0, rejected = 0, passes = 0, te_done = 0, uploads = 0, evictions = 0;
  std::vector<double> lat_ms;
  double t_start = 0, t_last_done = 0;
  // device resources
  hipStream_t st[kStreams] = {nullptr, nullptr};
  BatchFork fork[kStreams];  // side streams of each pass stream's kinds
  hipStream_t copy_st = nullptr;
  hipEvent_t ev[kStreams] = {nullptr, nullptr};
  hipEvent_t ev0[kStreams] = {nullptr, nullptr};  // pass start (timing)
  double gpu_pass_s = 0;                           // stats: sum of pass durations on the device
  char *staging[kStreams] = {nullptr, nullptr};  // pinned blob images
  void *slot_arena[kStreams] = {nullptr, nullptr};  // per-slot pass scratch (grow-only)
  size_t slot_arena_bytes[kStreams] = {0, 0};
  void *slot_blob[kStreams] = {nullptr, nullptr};   // per-slot descriptor blob (grow-only)
  size_t slot_blob_bytes[kStreams] = {0, 0};
  size_t staging_bytes[kStreams] = {0, 0};
  bool slot_busy[kStreams] = {false, false};
  // device output blocks by size (powers of two), kept for reuse: a free
  // waits for the whole device, so blocks are only freed under budget
  // pressure; cached blocks count as used
  std::map<uint64_t, std::vector<void *>> out_free;
  uint64_t out_free_bytes = 0;
  std::deque<uint64_t> to_copy;      // finished on the device, result not yet in host memory
  std::deque<uint64_t> done_q;       // finished requests, in completion order (for next_done)
  std::condition_variable cv_copy;
  std::vector<std::thread> copiers;
  // uploads and frees off the scheduler thread: polynomials to make resident
  // (in admission order), and evicted handles and trimmed output blocks to
  // release (hipFree waits for the device, so it never runs under the lock
  // or on the scheduler thread)
  std::deque<uint64_t> upload_q;
  std::vector<peval_poly *> reclaim_h;
  std::vector<void *> reclaim_blocks;
  std::condition_variable cv_upload;
  std::vector<std::thread> uploaders;
  hipStream_t copy_sts[4] = {nullptr, nullptr, nullptr, nullptr};
  int err = PEVAL_OK;                // sticky device error
};

// ---------------------------------------------------------------------------
// residency
// ---------------------------------------------------------------------------
static uint64_t estimate_poly_bytes(const SPoly &sp) {
  // resident terms + one thread layout (K <= 32, P = 16) + tables
  uint64_t b = sp.s * (sp.w + 2ull * (sp.n - 2));
  b += (sp.s + 64) * 5 + (sp.s / 64 + 2) * 12 + sp.G * 4;
  return b + 4096;
}

// Upper bound of the scratch one slice of ts evaluations with at most c
// chains needs (any K <= 32, P = 16): power tables, chain starts, Gamma,
// Gamma', partial sums.  Used for reservations, so that every pass fits.
static uint64_t slice_scratch_bound(const SPoly &sp, uint32_t ts, uint32_t c) {
  const uint64_t w = sp.w;
  const uint64_t kn = sp.s + 32 * sp.G + 2048;           // >= K * NT for K <= 32
  const uint64_t slots = (sp.s + sp.G) / 16 + 2 * sp.G + 64;  // >= nslots for K >= 1, P = 16
  const uint64_t lmax = ((uint64_t)ts + c - 1) / c;
  uint64_t b = 2 * (std::max<uint64_t>(sp.tab_total, 1) * w + 256);
  b += (uint64_t)c * kn * w + 256 + 2 * (kn * w + 256);
  b += (uint64_t)c * lmax * slots * w + 256;
  return b;
}

static uint32_t slice_evals(const peval_server *S, const SPoly &sp, uint32_t T) {
  double ts = std::floor(S->slice_work / (double)std::max<uint64_t>(sp.s, 1));
  return (uint32_t)std::min<double>(T, std::max(16.0, ts));
}

// Evict least recently used resident polynomials with no request in flight
// until `need` more bytes fit; `keep` (the polynomial of the request being
// admitted, whose residency the caller has already counted) is never chosen.
static void evict_for(peval_server *S, uint64_t need, uint64_t keep) {
  while (S->used + need > S->budget) {
    SPoly *victim = nullptr;
    for (auto &kv : S->polys) {
      SPoly &sp = kv.second;
      if (kv.first == keep) continue;
      if ((sp.h || (S->simulate && sp.bytes)) && sp.refs == 0 && (!victim || sp.last_used < victim->last_used))
        victim = &sp;
    }
    if (!victim) return;
    if (victim->h) {  // released by an uploader thread; its bytes count as free now
      S->reclaim_h.push_back(victim->h);
      S->cv_upload.notify_one();
    }
    victim->h = nullptr;
    victim->plan = nullptr;
    S->used -= victim->bytes;
    victim->bytes = 0;
    S->evictions++;
  }
}

static int make_resident(peval_server *S, SPoly &sp) {
  if (sp.h || (S->simulate && sp.bytes)) return PEVAL_OK;
  if (S->simulate) {
    S->uploads++;
    sp.bytes = estimate_poly_bytes(sp);
    S->used += sp.bytes;
    return PEVAL_OK;
  }
  return fail(PEVAL_EINVAL, "device residency goes through upload_poly");
}

// Device part of residency: create the handle and its batched thread layout.
// Touches no server state (called without the server lock).
static int upload_poly(const SPoly &sp, peval_poly **out, Plan **plan_out, uint64_t *bytes) {
  peval_poly *h = nullptr;
  *out = nullptr;
  PEVAL_TRY(peval_create(sp.p, sp.n, sp.s, sp.exps.data(), sp.coeffs.data(), &h));
  Plan *pl = nullptr;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    Tuning t = choose_tuning(h, 64);
    int rc = get_plan(h, t.K, kBatchP, &pl);
    if (rc != PEVAL_OK) {
      peval_destroy(h);
      return rc;
    }
  }
  peval_info_t inf;
  peval_info(h, &inf);
  *out = h;
  *plan_out = pl;
  *bytes = inf.device_bytes;
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// scheduler
// ---------------------------------------------------------------------------
static uint64_t out_block(uint64_t bytes) {
  uint64_t b = 65536;
  while (b < bytes) b <<= 1;
  return b;
}

// The request's output block goes back to the pool and its scratch
// reservation to the budget.
static void release_output(peval_server *S, SReq &r) {
  if (r.d_out) {
    S->out_free[r.out_alloc].push_back(r.d_out);
    S->out_free_bytes += r.out_alloc;
    r.d_out = nullptr;
  } else {
    S->used -= r.out_alloc;  // simulated: nothing was allocated
  }
  S->used -= r.reserve;
}

// Free cached output blocks, largest first, until `need` more bytes fit.
static void trim_out_cache(peval_server *S, uint64_t need) {
  while (S->used + need > S->budget && !S->out_free.empty()) {
    auto it = std::prev(S->out_free.end());
    if (it->second.empty()) {
      S->out_free.erase(it);
      continue;
    }
    S->reclaim_blocks.push_back(it->second.back());  // freed by an uploader thread
    S->cv_upload.notify_one();
    it->second.pop_back();
    S->used -= it->first;
    S->out_free_bytes -= it->first;
  }
}

static void finish_request(peval_server *S, SReq &r, double t) {
  r.status = 0;
  S->done_q.push_back(r.id);
  r.t_done = t;
  S->completed++;
  S->te_done += S->polys[r.poly].s * (uint64_t)r.T;
  S->lat_ms.push_back((r.t_done - r.t_submit) * 1e3);
  S->t_last_done = t;
  SPoly &sp = S->polys[r.poly];
  sp.refs--;
  release_output(S, r);
}

// Retire passes whose work is complete (oldest first).
static void retire(peval_server *S) {
  while (!S->inflight.empty()) {
    Pass &ps = S->inflight.front();
    if (S->simulate) {
      if (now_s() < ps.t_sim_end) return;
    } else {
      hipError_t q = hipEventQuery(S->ev[ps.slot]);
      if (q == hipErrorNotReady) return;
      if (q != hipSuccess) {
        S->err = fail(PEVAL_EDEVICE, "pass failed: %s", hipGetErrorString(q));
        S->cv_done.notify_all();  // waiters return the error instead of waiting on
        return;
      }
      float ms = 0;
      if (hipEventElapsedTime(&ms, S->ev0[ps.slot], S->ev[ps.slot]) == hipSuccess) S->gpu_pass_s += ms * 1e-3;
    }
    S->slot_busy[ps.slot] = false;
    for (uint64_t rid : ps.reqs) {
      SReq &r = S->reqs[rid];
      r.finished_passes++;
      if (r.t_next > r.T && r.finished_passes == r.launched_passes) {
        S->active.erase(std::remove(S->active.begin(), S->active.end(), rid), S->active.end());
        if (S->simulate || !r.host_out) {
          finish_request(S, r, now_s());
        } else {
          S->to_copy.push_back(rid);  // the copy threads bring the result home
          S->cv_copy.notify_one();
        }
      }
    }
    S->inflight.pop_front();
    S->cv_done.notify_all();
  }
}

// Admit pending requests in arrival order while the budget allows.  An
// admitted request holds its output and a scratch reservation for its slices
// until it finishes, so passes never need memory beyond the budget.
static void admit(peval_server *S, std::unique_lock<std::mutex> &lk) {
  while (!S->pending.empty()) {
    SReq &r = S->reqs[S->pending.front()];
    SPoly &sp = S->polys[r.poly];
    // a polynomial being uploaded already holds its estimated bytes
    const bool resident = sp.h || (S->simulate && sp.bytes) || sp.uploading;
    if (sp.plan) {  // resident: the reservation follows the actual thread layout
      r.reserve = 2 * (member_scratch_bytes(sp.h, *sp.plan, r.cmax, r.ts) + (uint64_t)r.cmax * sp.plan->nslots * sp.w);
    }
    const uint64_t ob = out_block(r.out_bytes);
    auto cached_block = [&] {
      auto it = S->out_free.find(ob);
      return !S->simulate && it != S->out_free.end() && !it->second.empty();
    };
    auto need_now = [&] { return (cached_block() ? 0 : ob) + r.reserve + (resident ? 0 : estimate_poly_bytes(sp)); };
    if (S->used + need_now() > S->budget) trim_out_cache(S, need_now());
    if (S->used + need_now() > S->budget) evict_for(S, need_now(), r.poly);
    if (S->used + need_now() > S->budget) return;  // head of line waits for memory
    const bool reuse = cached_block();
    if (reuse) {
      r.d_out = S->out_free[ob].back();
      S->out_free[ob].pop_back();
      S->out_free_bytes -= ob;
    }
    r.out_alloc = ob;
    int rc = PEVAL_OK;
    if (S->simulate) {
      rc = make_resident(S, sp);
    } else {
      if (!resident) {  // an uploader thread makes it resident; passes skip the request until then
        sp.uploading = true;
        S->used += estimate_poly_bytes(sp);  // held while uploading
        S->upload_q.push_back(r.poly);
        S->cv_upload.notify_one();
      }
      // the request stays at the head of `pending` meanwhile, which keeps its
      // polynomial from being removed
      if (!reuse) {
        lk.unlock();
        if (hipMalloc(&r.d_out, ob) != hipSuccess) {
          r.d_out = nullptr;
          rc = fail(PEVAL_ENOMEM, "output");
        }
        lk.lock();
      }
    }
    S->pending.pop_front();
    if (rc != PEVAL_OK) {
      if (r.d_out) {  // a reused block goes back to the pool
        S->out_free[ob].push_back(r.d_out);
        S->out_free_bytes += ob;
        r.d_out = nullptr;
      }
      r.status = rc;
      S->done_q.push_back(r.id);
      S->rejected++;
      S->cv_done.notify_all();
      continue;
    }
    sp.refs++;
    sp.last_used = ++S->clock;
    S->used += (reuse ? 0 : ob) + r.reserve;
    S->peak = std::max(S->peak, S->used);
    r.admitted = true;
    S->active.push_back(r.id);
  }
}

// Build and launch one pass over the active requests; returns false if
// nothing could be launched.
static bool launch_pass_impl(peval_server *S, std::unique_lock<std::mutex> &lk);

static bool launch_pass(peval_server *S, std::unique_lock<std::mutex> &lk) {
  const double t0 = now_s();
  bool ok = launch_pass_impl(S, lk);
  S->host_pass_s += now_s() - t0;
  return ok;
}

static bool launch_pass_impl(peval_server *S, std::unique_lock<std::mutex> &lk) {
  int slot = -1;
  for (int k = 0; k < kStreams; ++k)
    if (!S->slot_busy[k]) slot = k;
  if (slot < 0) return false;
  // Candidates: the oldest active request first (no starvation), then the
  // rest by remaining work, shortest first, until the pass holds pass_work.
  std::vector<std::pair<double, uint64_t>> cand;
  for (uint64_t rid : S->active) {
    const SReq &r = S->reqs[rid];
    if (r.t_next > r.T) continue;
    if (!S->simulate && !S->polys[r.poly].h) continue;  // its upload has not finished
    cand.emplace_back((double)S->polys[r.poly].s * (r.T - r.t_next + 1), rid);
  }
  if (cand.empty()) return false;
  std::vector<uint64_t> ids;
  {
    auto oldest = std::min_element(cand.begin(), cand.end(), [](const std::pair<double, uint64_t> &a,
                                                                const std::pair<double, uint64_t> &b) {
      return a.second < b.second;  // ids grow with submission order
    });
    ids.push_back(oldest->second);
    cand.erase(oldest);
    std::sort(cand.begin(), cand.end());
    double work = 0;
    {
      const SReq &r0 = S->reqs[ids[0]];
      work = (double)S->polys[r0.poly].s * std::min<uint32_t>(r0.ts, r0.T - r0.t_next + 1);
    }
    for (auto &c : cand) {
      if (work >= S->pass_work || ids.size() >= S->max_members) break;
      const SReq &r = S->reqs[c.second];
      work += (double)S->polys[r.poly].s * std::min<uint32_t>(r.ts, r.T - r.t_next + 1);
      ids.push_back(c.second);
    }
  }

  struct Slice {
    uint64_t rid;
    uint32_t t0, T;
  };
  std::vector<Slice> sl;
  std::vector<BatchMember> mem;
  std::vector<BatchRun> runs;
  uint64_t te = 0;
  for (uint64_t rid : ids) {
    SReq &r = S->reqs[rid];
    SPoly &sp = S->polys[r.poly];
    const uint32_t ts = std::min<uint32_t>(r.ts, r.T - r.t_next + 1);
    BatchMember m{sp.h, sp.plan, 1, ts};
    sl.push_back(Slice{rid, r.t_next, ts});
    mem.push_back(m);
    te += sp.s * (uint64_t)ts;
  }
  if (sl.empty()) return false;

  Pass ps;
  ps.slot = slot;
  ps.t_launch = now_s();
  ps.term_evals = te;
  if (S->simulate) {
    ps.t_sim_end = std::max(ps.t_launch, S->inflight.empty() ? 0.0 : S->inflight.back().t_sim_end) + te / S->sim_rate;
  } else {
    // chains so that work items have similar costs, as in peval_batch_create,
    // within what each request's scratch reservation allows
    int crc = batch_chains(mem, 1.0);
    if (crc != PEVAL_OK) {
      S->err = crc;
      S->cv_done.notify_all();
      return false;
    }
    for (size_t j = 0; j < mem.size(); ++j) mem[j].C = std::min(mem[j].C, S->reqs[sl[j].rid].cmax);
    const size_t scratch = batch_scratch_need(mem);
    runs.resize(mem.size());
    for (size_t j = 0; j < mem.size(); ++j) {
      SReq &r = S->reqs[sl[j].rid];
      const peval_poly *h = mem[j].h;
      memset(&runs[j], 0, sizeof(BatchRun));
      for (uint32_t k = 0; k + 2 < h->n; ++k) runs[j].beta.b[k] = r.beta[k] % h->p;
      runs[j].t0 = sl[j].t0;
      runs[j].out = (char *)r.d_out + (uint64_t)(sl[j].t0 - 1) * h->G * h->w;
    }
    // Planning and launching use only the copies above, the handles and
    // their plans (which no other thread changes): submitters may proceed.
    lk.unlock();
    int launch_rc = PEVAL_OK;
    hipStream_t st = S->st[slot];
    BatchCore core;
    void *arena = nullptr, *blob = nullptr;
    do {
      (void)hipEventRecord(S->ev0[slot], st);
      // the slot's previous pass has retired, so its buffers are free; they
      // only grow (a larger pass reallocates them once)
      if (S->slot_arena_bytes[slot] < scratch) {
        if (S->slot_arena[slot]) (void)hipFree(S->slot_arena[slot]);
        S->slot_arena[slot] = nullptr;
        S->slot_arena_bytes[slot] = 0;
        size_t want = std::max<size_t>(scratch + scratch / 4, 1 << 20);
        if (hipMalloc(&S->slot_arena[slot], want) != hipSuccess) {
          launch_rc = fail(PEVAL_ENOMEM, "pass scratch of %zu bytes", want);
          break;
        }
        S->slot_arena_bytes[slot] = want;
      }
      arena = S->slot_arena[slot];
      batch_plan(core, mem, arena, runs.data());
      if (S->staging_bytes[slot] < core.blob_bytes) {
        // the slot's previous pass has retired, so its staging buffer is free
        if (S->staging[slot]) (void)hipHostFree(S->staging[slot]);
        S->staging[slot] = nullptr;
        S->staging_bytes[slot] = 0;
        if (hipHostMalloc((void **)&S->staging[slot], core.blob_bytes * 2, hipHostMallocDefault) != hipSuccess) {
          launch_rc = fail(PEVAL_ENOMEM, "pinned staging");
          break;
        }
        S->staging_bytes[slot] = core.blob_bytes * 2;
      }
      memcpy(S->staging[slot], core.image.data(), core.blob_bytes);
      if (S->slot_blob_bytes[slot] < core.blob_bytes) {
        if (S->slot_blob[slot]) (void)hipFree(S->slot_blob[slot]);
        S->slot_blob[slot] = nullptr;
        S->slot_blob_bytes[slot] = 0;
        size_t want = std::max<size_t>(core.blob_bytes * 2, 1 << 20);
        if (hipMalloc(&S->slot_blob[slot], want) != hipSuccess) {
          launch_rc = fail(PEVAL_ENOMEM, "pass descriptors");
          break;
        }
        S->slot_blob_bytes[slot] = want;
      }
      blob = S->slot_blob[slot];
      hipError_t e = hipMemcpyAsync(blob, S->staging[slot], core.blob_bytes, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) {
        launch_rc = fail(PEVAL_EDEVICE, "pass upload: %s", hipGetErrorString(e));
        break;
      }
      batch_bind(core, blob);
      launch_rc = batch_set_blocks(core);
      if (launch_rc == PEVAL_OK) launch_rc = batch_enqueue(core, st, &S->fork[slot]);
      if (launch_rc == PEVAL_OK && hipEventRecord(S->ev[slot], st) != hipSuccess)
        launch_rc = fail(PEVAL_EDEVICE, "event record");
    } while (false);
    lk.lock();
    if (launch_rc != PEVAL_OK) {
      S->err = launch_rc;
      S->cv_done.notify_all();  // waiters return the error instead of waiting on
      return false;
    }
  }
  for (size_t j = 0; j < sl.size(); ++j) {
    SReq &r = S->reqs[sl[j].rid];
    r.t_next += sl[j].T;
    r.launched_passes++;
    ps.reqs.push_back(sl[j].rid);
    S->polys[r.poly].last_used = ++S->clock;
  }
  S->slot_busy[slot] = true;
  S->inflight.push_back(ps);
  S->passes++;
  S->slices += sl.size();
  return true;
}

// Result copies to host memory run here, off the scheduler thread, four at
// a time.  A page-locked destination gets one direct DMA; pageable memory
// goes device -> pinned staging -> destination in chunks, the next chunk's
// DMA overlapping the previous chunk's host copy.
static int copy_result(hipStream_t st, char *const stage[2], hipEvent_t ev[2], size_t chunk, void *dst,
                       const void *src, uint64_t bytes) {
  const uint64_t n = (bytes + chunk - 1) / chunk;
  auto issue = [&](uint64_t i) {
    const uint64_t off = i * chunk, len = std::min<uint64_t>(chunk, bytes - off);
    hipError_t e = hipMemcpyAsync(stage[i & 1], (const char *)src + off, len, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev[i & 1], st);
    return e;
  };
  if (n && issue(0) != hipSuccess) return PEVAL_EDEVICE;
  for (uint64_t i = 0; i < n; ++i) {
    if (i + 1 < n && issue(i + 1) != hipSuccess) return PEVAL_EDEVICE;
    if (hipEventSynchronize(ev[i & 1]) != hipSuccess) return PEVAL_EDEVICE;
    const uint64_t off = i * chunk, len = std::min<uint64_t>(chunk, bytes - off);
    memcpy((char *)dst + off, stage[i & 1], len);
  }
  return PEVAL_OK;
}

static void copier_main(peval_server *S, int idx) {
  (void)hipSetDevice(S->device);
  constexpr size_t kChunk = 8u << 20;
  char *stage[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ready = true;
  for (int k = 0; k < 2; ++k) {
    ready = ready && hipHostMalloc((void **)&stage[k], kChunk, hipHostMallocDefault) == hipSuccess;
    ready = ready && hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) == hipSuccess;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_copy.wait(lk, [&] { return S->stop || !S->to_copy.empty(); });
    if (S->to_copy.empty()) {
      if (S->stop) break;
      continue;
    }
    uint64_t rid = S->to_copy.front();
    S->to_copy.pop_front();
    SReq &r = S->reqs[rid];
    void *dst = r.host_out, *src = r.d_out;
    uint64_t bytes = r.out_bytes;
    lk.unlock();  // the request is unfinished: nobody else touches it
    int rc = PEVAL_OK;
    hipPointerAttribute_t attr;
    bool pinned = hipPointerGetAttributes(&attr, dst) == hipSuccess && attr.type == hipMemoryTypeHost;
    (void)hipGetLastError();  // a pageable pointer is not an error here
    if (pinned) {  // page-locked destination: one direct DMA
      hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, S->copy_sts[idx]);
      if (e == hipSuccess) e = hipStreamSynchronize(S->copy_sts[idx]);
      if (e != hipSuccess) rc = PEVAL_EDEVICE;
    } else {
      rc = ready ? copy_result(S->copy_sts[idx], stage, ev, kChunk, dst, src, bytes) : PEVAL_ENOMEM;
    }
    lk.lock();
    if (rc != PEVAL_OK) {
      r.status = fail(rc, "result copy failed");
      S->done_q.push_back(r.id);
      S->polys[r.poly].refs--;
      release_output(S, r);
      S->cv_done.notify_all();
      continue;
    }
    finish_request(S, r, now_s());
    S->cv_done.notify_all();
    S->cv_work.notify_one();  // memory was released
  }
  lk.unlock();
  for (int k = 0; k < 2; ++k) {
    if (stage[k]) (void)hipHostFree(stage[k]);
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  }
}

// Uploads of polynomials for admitted requests, and the frees of evicted
// handles and trimmed output blocks.
static void uploader_main(peval_server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_upload.wait(lk, [&] {
      return S->stop || !S->upload_q.empty() || !S->reclaim_h.empty() || !S->reclaim_blocks.empty();
    });
    if (!S->reclaim_h.empty() || !S->reclaim_blocks.empty()) {
      std::vector<peval_poly *> hs;
      std::vector<void *> bs;
      hs.swap(S->reclaim_h);
      bs.swap(S->reclaim_blocks);
      lk.unlock();
      for (peval_poly *h : hs) peval_destroy(h);
      for (void *b : bs) (void)hipFree(b);
      lk.lock();
      continue;
    }
    if (S->stop) break;
    const uint64_t pid = S->upload_q.front();
    S->upload_q.pop_front();
    // an admitted request holds the polynomial (refs > 0), so it stays
    // registered; its inputs never change after add_poly
    SPoly &sp = S->polys[pid];
    lk.unlock();
    peval_poly *h = nullptr;
    Plan *plan = nullptr;
    uint64_t bytes = 0;
    int rc = upload_poly(sp, &h, &plan, &bytes);
    lk.lock();
    S->used -= estimate_poly_bytes(sp);
    sp.uploading = false;
    if (rc == PEVAL_OK) {
      sp.h = h;
      sp.plan = plan;
      sp.bytes = bytes;
      S->used += bytes;
      S->peak = std::max(S->peak, S->used);
      S->uploads++;
      // exact reservations now that the layout is known (never above the bound)
      for (uint64_t rid : S->active) {
        SReq &r = S->reqs[rid];
        if (r.poly != pid) continue;
        const uint64_t exact =
            std::min<uint64_t>(r.reserve, 2 * (member_scratch_bytes(h, *plan, r.cmax, r.ts) +
                                               (uint64_t)r.cmax * plan->nslots * sp.w));
        S->used -= r.reserve - exact;
        r.reserve = exact;
      }
    } else {  // every admitted request of the polynomial fails with the upload's error
      for (size_t j = 0; j < S->active.size();) {
        SReq &r = S->reqs[S->active[j]];
        if (r.poly != pid) {
          ++j;
          continue;
        }
        S->active.erase(S->active.begin() + j);
        r.status = rc;
        S->done_q.push_back(r.id);
        S->rejected++;
        sp.refs--;
        release_output(S, r);
      }
      S->cv_done.notify_all();
    }
    S->cv_work.notify_one();
  }
}

static void worker_main(peval_server *S) {
  if (!S->simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    retire(S);
    if (S->err == PEVAL_OK) {
      admit(S, lk);
      while (S->err == PEVAL_OK && launch_pass(S, lk)) {
      }
    }
    bool busy = !S->inflight.empty();
    S->cv_work.wait_for(lk, std::chrono::microseconds(busy ? 50 : 2000));
  }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int peval_server_create(uint64_t hbm_budget_bytes, uint32_t flags, peval_server **out) {
  if (!out) return fail(PEVAL_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < (1u << 20)) return fail(PEVAL_EINVAL, "budget below 1 MiB");
  peval_server *S = new (std::nothrow) peval_server();
  if (!S) return fail(PEVAL_ENOMEM, "host allocation");
  S->budget = hbm_budget_bytes;
  S->simulate = (flags & PEVAL_SERVER_SIMULATE) != 0;
  if (!S->simulate) {
    bool ok = hipGetDevice(&S->device) == hipSuccess;
    for (int k = 0; ok && k < kStreams; ++k)
      ok = hipStreamCreateWithFlags(&S->st[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreate(&S->ev[k]) == hipSuccess && hipEventCreate(&S->ev0[k]) == hipSuccess;
    for (int k = 0; ok && k < kStreams; ++k) ok = S->fork[k].create() == PEVAL_OK;
    ok = ok && hipStreamCreateWithFlags(&S->copy_st, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; ok && k < 4; ++k) ok = hipStreamCreateWithFlags(&S->copy_sts[k], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
      peval_server_destroy(S);
      return fail(PEVAL_EDEVICE, "stream creation");
    }
  }
  S->t_start = now_s();
  S->worker = std::thread(worker_main, S);
  if (!S->simulate) {
    for (int k = 0; k < 4; ++k) S->copiers.emplace_back(copier_main, S, k);
    for (int k = 0; k < kUploaders; ++k) S->uploaders.emplace_back(uploader_main, S);
  }
  *out = S;
  return PEVAL_OK;
}

extern "C" int peval_server_configure(peval_server *S, double slice_work, double pass_work, uint32_t max_members,
                                      double sim_rate) {
  if (!S || slice_work < 1 || pass_work < 1 || max_members < 1 || sim_rate <= 0) return fail(PEVAL_EINVAL, "bad argument");
  std::lock_guard<std::mutex> lk(S->mu);
  S->max_members = max_members;
  S->slice_work = slice_work;
  S->pass_work = pass_work;
  S->sim_rate = sim_rate;
  return PEVAL_OK;
}

extern "C" int peval_server_add_poly(peval_server *S, uint64_t p, uint32_t n, uint64_t s, const uint32_t *exponents,
                                     const uint64_t *coeffs, uint64_t *poly_id) {
  if (!S || !poly_id) return fail(PEVAL_EINVAL, "null argument");
  if (p < 3 || (p & 1) == 0 || p >= (1ull << 63)) return fail(PEVAL_EINVAL, "p must be odd with 3 <= p < 2^63");
  if (n < 2 || n > 32) return fail(PEVAL_EINVAL, "n must be in [2, 32]");
  if (s && (!exponents || !coeffs)) return fail(PEVAL_EINVAL, "null exponents or coefficients");
  SPoly sp;
  sp.p = p;
  sp.n = n;
  sp.s = s;
  sp.w = p < (1ull << 31) ? 4 : 8;
  for (uint64_t i = 0; i < s; ++i)
    for (uint32_t k = 0; k < n; ++k) sp.max_exp[k] = std::max(sp.max_exp[k], exponents[i * n + k]);
  for (uint32_t k = 2; k < n; ++k) {
    if (sp.max_exp[k] > 65535) return fail(PEVAL_EUNSUPPORTED, "tail exponent > 65535");
    sp.tab_total += sp.max_exp[k] + 1;
  }
  sp.exps.assign(exponents, exponents + s * n);
  sp.coeffs.assign(coeffs, coeffs + s);
  {  // number of output columns (distinct (x1, x2) exponents)
    const uint64_t ext0 = (uint64_t)sp.max_exp[0] + 1, ext1 = (uint64_t)sp.max_exp[1] + 1;
    if (s && ext0 * ext1 <= (1ull << 26)) {
      std::vector<uint8_t> seen(ext0 * ext1, 0);
      for (uint64_t i = 0; i < s; ++i) {
        uint8_t &f = seen[(uint64_t)exponents[i * n] * ext1 + exponents[i * n + 1]];
        sp.G += f ^ 1;
        f = 1;
      }
    } else {
      std::vector<uint64_t> keys(s);
      for (uint64_t i = 0; i < s; ++i) keys[i] = ((uint64_t)exponents[i * n] << 32) | exponents[i * n + 1];
      std::sort(keys.begin(), keys.end());
      sp.G = (uint64_t)(std::unique(keys.begin(), keys.end()) - keys.begin());
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  sp.id = S->next_id++;
  *poly_id = sp.id;
  S->polys.emplace(sp.id, std::move(sp));
  return PEVAL_OK;
}

extern "C" int peval_server_poly_info(peval_server *S, uint64_t poly_id, peval_info_t *info) {
  if (!S || !info) return fail(PEVAL_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->polys.find(poly_id);
  if (it == S->polys.end()) return fail(PEVAL_EINVAL, "unknown polynomial");
  const SPoly &sp = it->second;
  memset(info, 0, sizeof *info);
  info->p = sp.p;
  info->n = sp.n;
  info->elem_bytes = sp.w;
  info->s = sp.s;
  info->G = sp.G;
  info->device_bytes = sp.h ? sp.bytes : 0;
  std::copy(sp.max_exp, sp.max_exp + 32, info->max_exp);
  return PEVAL_OK;
}

extern "C" int peval_server_remove_poly(peval_server *S, uint64_t poly_id) {
  if (!S) return fail(PEVAL_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->polys.find(poly_id);
  if (it == S->polys.end()) return fail(PEVAL_EINVAL, "unknown polynomial");
  if (it->second.refs) return fail(PEVAL_EBUSY, "polynomial has requests in flight");
  for (uint64_t rid : S->pending)
    if (S->reqs[rid].poly == poly_id) return fail(PEVAL_EBUSY, "polynomial has queued requests");
  if (it->second.uploading) return fail(PEVAL_EBUSY, "polynomial is being uploaded");
  if (it->second.h) {
    if (S->simulate) {
      peval_destroy(it->second.h);
    } else {
      S->reclaim_h.push_back(it->second.h);
      S->cv_upload.notify_one();
    }
  }
  S->used -= it->second.bytes;
  S->polys.erase(it);
  return PEVAL_OK;
}

extern "C" int peval_server_submit(peval_server *S, uint64_t poly_id, const uint64_t *beta, uint32_t T, void *host_out,
                                   uint64_t *req_id) {
  if (!S || !req_id) return fail(PEVAL_EINVAL, "null argument");
  if (T == 0) return fail(PEVAL_EINVAL, "T must be >= 1");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->err != PEVAL_OK) return S->err;
  auto it = S->polys.find(poly_id);
  if (it == S->polys.end()) return fail(PEVAL_EINVAL, "unknown polynomial");
  SPoly &sp = it->second;
  if (sp.n > 2 && !beta) return fail(PEVAL_EINVAL, "null beta");
  if (!S->simulate && !host_out && sp.G) return fail(PEVAL_EINVAL, "null output");
  SReq r;
  r.id = S->next_id++;
  r.poly = poly_id;
  if (beta) r.beta.assign(beta, beta + (sp.n - 2));
  r.T = T;
  r.host_out = host_out;
  r.out_bytes = (uint64_t)T * sp.G * sp.w;
  r.t_submit = now_s();
  r.ts = slice_evals(S, sp, T);
  // chains: enough to fill the device when the request runs alone (about
  // 8192 waves at 8 terms per thread), within 1/4 of the budget
  const uint64_t want = (8192ull * 512 + sp.s + 8 * sp.G - 1) / (sp.s + 8 * sp.G);
  r.cmax = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(want, 64), r.ts);
  while (r.cmax > 1 && slice_scratch_bound(sp, r.ts, r.cmax) * 4 > S->budget) r.cmax /= 2;
  r.cmax = std::max<uint32_t>(r.cmax, 1);
  // a tight budget takes shorter slices rather than refusing the request
  while (r.ts > 16 && slice_scratch_bound(sp, r.ts, r.cmax) * 4 > S->budget) r.ts = std::max<uint32_t>(16, r.ts / 2);
  r.reserve = slice_scratch_bound(sp, r.ts, r.cmax) * 2;  // two passes may hold slices of it
  // a request that cannot fit even alone is refused now
  const uint64_t alone = out_block(r.out_bytes) + r.reserve + estimate_poly_bytes(sp);
  if (alone > S->budget) {
    S->rejected++;
    return fail(PEVAL_ENOMEM, "request needs about %llu bytes, budget is %llu", (unsigned long long)alone,
                (unsigned long long)S->budget);
  }
  S->submitted++;
  *req_id = r.id;
  if (sp.G == 0) {  // nothing to compute
    r.status = 0;
    r.t_done = r.t_submit;
    S->reqs.emplace(r.id, r);
    S->done_q.push_back(r.id);
    S->completed++;
    S->lat_ms.push_back(0);
    return PEVAL_OK;
  }
  S->reqs.emplace(r.id, r);
  S->pending.push_back(r.id);
  S->cv_work.notify_one();
  return PEVAL_OK;
}

extern "C" int peval_server_poll(peval_server *S, uint64_t req_id, int *done) {
  if (!S || !done) return fail(PEVAL_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(PEVAL_EINVAL, "unknown request");
  *done = it->second.status <= 0;
  return it->second.status < 0 ? it->second.status : PEVAL_OK;
}

extern "C" int peval_server_wait(peval_server *S, uint64_t req_id, int64_t timeout_ms) {
  if (!S) return fail(PEVAL_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(PEVAL_EINVAL, "unknown request");
  auto pred = [&] { return it->second.status <= 0 || S->err != PEVAL_OK; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, pred);
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
    return fail(PEVAL_ETIMEOUT, "request not finished");
  }
  if (it->second.status < 0) return it->second.status;
  if (S->err != PEVAL_OK && it->second.status != 0) return S->err;
  return PEVAL_OK;
}

extern "C" int peval_server_next_done(peval_server *S, int64_t timeout_ms, uint64_t *req_id) {
  if (!S || !req_id) return fail(PEVAL_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto pred = [&] { return !S->done_q.empty() || S->err != PEVAL_OK; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, pred);
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
    return fail(PEVAL_ETIMEOUT, "no request finished");
  }
  if (S->done_q.empty()) return S->err;
  *req_id = S->done_q.front();
  S->done_q.pop_front();
  return PEVAL_OK;
}

extern "C" int peval_server_release(peval_server *S, uint64_t req_id) {
  if (!S) return fail(PEVAL_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(PEVAL_EINVAL, "unknown request");
  if (it->second.status > 0) return fail(PEVAL_EBUSY, "request not finished");
  S->reqs.erase(it);
  auto q = std::find(S->done_q.begin(), S->done_q.end(), req_id);
  if (q != S->done_q.end()) S->done_q.erase(q);
  return PEVAL_OK;
}

extern "C" int peval_server_stats(peval_server *S, peval_server_stats_t *st) {
  if (!S || !st) return fail(PEVAL_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  memset(st, 0, sizeof *st);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->rejected = S->rejected;
  st->queued = S->pending.size();
  st->active = S->active.size();
  st->passes = S->passes;
  st->term_evals = S->te_done;
  st->uploads = S->uploads;
  st->slices = S->slices;
  st->host_pass_s = S->host_pass_s;
  st->gpu_pass_s = S->gpu_pass_s;
  st->evictions = S->evictions;
  st->hbm_in_use = S->used;
  st->hbm_peak = S->peak;
  st->wall_s = (S->t_last_done > S->t_start ? S->t_last_done : now_s()) - S->t_start;
  std::vector<double> v = S->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min<size_t>(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    st->p50_ms = q(0.50);
    st->p99_ms = q(0.99);
    st->max_ms = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_ms = sum / v.size();
  }
  return S->err;
}

extern "C" int peval_server_reset_stats(peval_server *S) {
  if (!S) return fail(PEVAL_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  S->submitted = S->completed = S->rejected = S->passes = S->te_done = S->uploads = S->evictions = 0;
  S->slices = 0;
  S->host_pass_s = 0;
  S->gpu_pass_s = 0;
  S->lat_ms.clear();
  S->t_start = now_s();
  S->t_last_done = 0;
  S->peak = S->used;
  return PEVAL_OK;
}

extern "C" int peval_server_destroy(peval_server *S) {
  if (!S) return PEVAL_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // let in-flight passes drain so that no kernel outlives its buffers
    while (!S->inflight.empty() && S->err == PEVAL_OK) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(200));
      lk.lock();
      if (!S->worker.joinable()) break;
    }
    // and let pending result copies finish
    while (!S->to_copy.empty() && S->err == PEVAL_OK) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(200));
      lk.lock();
    }
    S->stop = true;
    S->cv_work.notify_all();
    S->cv_copy.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (auto &t : S->copiers)
    if (t.joinable()) t.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->cv_upload.notify_all();
  }
  for (auto &t : S->uploaders)
    if (t.joinable()) t.join();
  for (peval_poly *h : S->reclaim_h) peval_destroy(h);
  for (void *b : S->reclaim_blocks) (void)hipFree(b);
  if (!S->simulate) {
    for (int k = 0; k < kStreams; ++k)
      if (S->st[k]) (void)hipStreamSynchronize(S->st[k]);
  }
  for (auto &kv : S->reqs)
    if (kv.second.d_out) (void)hipFree(kv.second.d_out);
  for (auto &kv : S->out_free)
    for (void *p : kv.second) (void)hipFree(p);
  for (auto &kv : S->polys)
    if (kv.second.h) peval_destroy(kv.second.h);
  for (int k = 0; k < kStreams; ++k) {
    if (S->staging[k]) (void)hipHostFree(S->staging[k]);
    if (S->slot_arena[k]) (void)hipFree(S->slot_arena[k]);
    if (S->slot_blob[k]) (void)hipFree(S->slot_blob[k]);
    if (S->ev[k]) (void)hipEventDestroy(S->ev[k]);
    if (S->ev0[k]) (void)hipEventDestroy(S->ev0[k]);
    if (S->st[k]) (void)hipStreamDestroy(S->st[k]);
    S->fork[k].destroy();
  }
  if (S->copy_st) (void)hipStreamDestroy(S->copy_st);
  for (int k = 0; k < 4; ++k)
    if (S->copy_sts[k]) (void)hipStreamDestroy(S->copy_sts[k]);
  delete S;
  return PEVAL_OK;
}
