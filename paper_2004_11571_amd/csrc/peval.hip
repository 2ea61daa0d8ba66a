// C ABI of the peval library: ingest, planning, kernel launches.
#include "peval.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "errors.hpp"
#include "kernels.hpp"
#include "peval_internal.hpp"
#include "small_kernels.hpp"

using namespace peval;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace peval {
std::string &last_error_slot() {
  static thread_local std::string msg;
  return msg;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error_slot() = buf;
  return code;
}
}  // namespace peval


extern "C" const char *peval_strerror(int code) {
  switch (code) {
    case PEVAL_OK: return "ok";
    case PEVAL_EINVAL: return "invalid argument";
    case PEVAL_ENOMEM: return "out of memory";
    case PEVAL_EDEVICE: return "device error";
    case PEVAL_EUNSUPPORTED: return "unsupported input";
    case PEVAL_EBUSY: return "busy";
    case PEVAL_ETIMEOUT: return "timed out";
    case PEVAL_ESINGULAR: return "singular system";
    default: return "unknown error";
  }
}

extern "C" const char *peval_last_error(void) { return last_error_slot().c_str(); }

// ---------------------------------------------------------------------------
// per-modulus constants (host, 128-bit arithmetic)
// ---------------------------------------------------------------------------
typedef unsigned __int128 u128;

namespace peval {
Mod64 make_mod64(uint64_t p) {
  Mod64 m;
  m.p = p;
  uint64_t inv = p;  // Newton iteration for p^{-1} mod 2^64 (p odd)
  for (int i = 0; i < 6; ++i) inv *= 2 - p * inv;
  m.pinv = inv;
  m.R = (uint64_t)(((u128)1 << 64) % p);
  m.Rq = (uint64_t)(((u128)m.R << 64) / p);
  m.oneq = (uint64_t)(((u128)1 << 64) / p);
  return m;
}

Mod32 make_mod32(uint32_t p) {
  Mod32 m;
  m.p = p;
  uint32_t inv = p;
  for (int i = 0; i < 5; ++i) inv *= 2 - p * inv;
  m.pinv = inv;
  m.R = (uint32_t)((1ull << 32) % p);
  m.Rq = (uint32_t)(((uint64_t)m.R << 32) / p);
  m.oneq = (uint32_t)((1ull << 32) / p);
  return m;
}
}  // namespace peval

// Automatic choice of the product (measured on the paper's own workload,
// 5e5 terms x 1e4 evaluations with a 50-bit prime: the evaluation kernel
// takes 2.50 ms with Alg. 2 and 2.88 ms with Shoup products).
static bool fp64_by_default(uint64_t p) { return p >= (1ull << 31) && p < (1ull << 50); }

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
  hipEvent_t a, b;
  int kind;
};
std::atomic<int> g_prof{0};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;
double g_prof_ms[4] = {0, 0, 0, 0};
uint64_t g_prof_n[4] = {0, 0, 0, 0};

}  // namespace

namespace peval {
static thread_local int t_prof_off = 0;
ProfOff::ProfOff() { ++t_prof_off; }
ProfOff::~ProfOff() { --t_prof_off; }

ProfScope::ProfScope(hipStream_t s, int k) : st(s), kind(k) {
  if (!g_prof.load() || t_prof_off) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_recs.push_back({a, b, kind});
}
}  // namespace peval

extern "C" int peval_prof_enable(int enable) {
  g_prof.store(enable ? 1 : 0);
  return PEVAL_OK;
}

extern "C" int peval_prof_read(double *ms, uint64_t *launches) {
  if (!ms || !launches) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof_recs) {
    float t = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      g_prof_ms[r.kind] += t;
      g_prof_n[r.kind] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof_recs.clear();
  for (int k = 0; k < 4; ++k) {
    ms[k] = g_prof_ms[k];
    launches[k] = g_prof_n[k];
    g_prof_ms[k] = 0;
    g_prof_n[k] = 0;
  }
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// layout planning (host)
// ---------------------------------------------------------------------------
namespace peval {

HostPlan build_host_plan(const std::vector<uint64_t> &grp_off, uint32_t K, uint32_t P, bool subtile_ends) {
  HostPlan hp;
  const uint64_t G = grp_off.size() - 1;
  uint64_t nt_real = 0;
  for (uint64_t g = 0; g < G; ++g) nt_real += (grp_off[g + 1] - grp_off[g] + K - 1) / K;
  hp.NT = std::max<uint64_t>(64, (nt_real + 63) / 64 * 64);
  hp.NW = hp.NT / 64;
  hp.thr_first.assign(hp.NT, 0);
  hp.thr_cnt.assign(hp.NT, 0);
  std::vector<uint32_t> tgrp(hp.NT, G ? (uint32_t)(G - 1) : 0);
  uint64_t j = 0;
  for (uint64_t g = 0; g < G; ++g) {
    for (uint64_t f = grp_off[g]; f < grp_off[g + 1]; f += K, ++j) {
      hp.thr_first[j] = (uint32_t)f;
      hp.thr_cnt[j] = (uint8_t)std::min<uint64_t>(K, grp_off[g + 1] - f);
      tgrp[j] = (uint32_t)g;
    }
  }
  hp.endmask.assign(hp.NW, 0);
  hp.slot_base.assign(hp.NW, 0);
  std::vector<uint64_t> per_group(G ? G : 1, 0);
  uint64_t slots = 0;
  for (uint64_t w = 0; w < hp.NW; ++w) {
    hp.slot_base[w] = (uint32_t)slots;
    uint64_t mask = 0;
    for (uint32_t l = 0; l < 64; ++l) {
      uint64_t t = w * 64 + l;
      // segment ends: group changes and the wave's last lane (sub-tiles of one
      // group are merged inside the wave by the walk), or every sub-tile end
      // for the walk that does not merge
      bool end = (l == 63) || (t + 1 == hp.NT) || (tgrp[t] != tgrp[t + 1]) || (subtile_ends && l % P == P - 1);
      if (end) {
        mask |= 1ull << l;
        per_group[tgrp[t]] += 1;
        ++slots;
      }
    }
    hp.endmask[w] = mask;
  }
  hp.nslots = slots;
  hp.slot_off.assign(G + 1, 0);
  for (uint64_t g = 0; g < G; ++g) hp.slot_off[g + 1] = (uint32_t)(hp.slot_off[g] + per_group[g]);
  return hp;
}

}  // namespace peval

extern "C" int peval_layout(const uint64_t *group_sizes, uint64_t G, uint32_t K, uint32_t P,
                            uint64_t *sizes, uint32_t *thr_first, uint8_t *thr_cnt,
                            uint64_t *endmask, uint32_t *slot_base, uint32_t *slot_off) {
  if ((G && !group_sizes) || !sizes) return fail(PEVAL_EINVAL, "null argument");
  if (!valid_K(K)) return fail(PEVAL_EINVAL, "K=%u", K);
  if (!(P == 8 || P == 16 || P == 32)) return fail(PEVAL_EINVAL, "P=%u", P);
  std::vector<uint64_t> off(G + 1, 0);
  for (uint64_t g = 0; g < G; ++g) {
    if (group_sizes[g] == 0) return fail(PEVAL_EINVAL, "empty group %llu", (unsigned long long)g);
    off[g + 1] = off[g] + group_sizes[g];
  }
  HostPlan hp = build_host_plan(off, K, P, false);
  sizes[0] = hp.NT;
  sizes[1] = hp.NW;
  sizes[2] = hp.nslots;
  if (thr_first) std::copy(hp.thr_first.begin(), hp.thr_first.end(), thr_first);
  if (thr_cnt) std::copy(hp.thr_cnt.begin(), hp.thr_cnt.end(), thr_cnt);
  if (endmask) std::copy(hp.endmask.begin(), hp.endmask.end(), endmask);
  if (slot_base) std::copy(hp.slot_base.begin(), hp.slot_base.end(), slot_base);
  if (slot_off) std::copy(hp.slot_off.begin(), hp.slot_off.end(), slot_off);
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace peval {
int ensure(Scratch &sc, size_t bytes, peval_poly *h) {
  if (sc.bytes >= bytes && sc.ptr) return PEVAL_OK;
  if (sc.ptr) {
    if (h->have_done) HIP_TRY(hipEventSynchronize(h->done));
    HIP_TRY(hipFree(sc.ptr));
    sc.ptr = nullptr;
    sc.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  HIP_TRY(hipMalloc(&sc.ptr, want));
  sc.bytes = want;
  return PEVAL_OK;
}
}  // namespace peval

static void release(Scratch &sc) {
  if (sc.ptr) (void)hipFree(sc.ptr);
  sc.ptr = nullptr;
  sc.bytes = 0;
}

template <class T>
static int upload(T **dptr, const std::vector<T> &v) {
  HIP_TRY(hipMalloc((void **)dptr, std::max<size_t>(v.size() * sizeof(T), 16)));
  if (!v.empty()) HIP_TRY(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PEVAL_OK;
}

static void free_plan(Plan &pl) {
  (void)hipFree(pl.d_thr_first);
  (void)hipFree(pl.d_thr_cnt);
  (void)hipFree(pl.d_endmask);
  (void)hipFree(pl.d_slot_base);
  (void)hipFree(pl.d_slot_off);
  pl = Plan();
}

namespace peval {
static uint32_t plan_key(uint32_t K, uint32_t P, bool subtile_ends) {
  return (subtile_ends ? 1u << 16 : 0u) | K << 8 | P;
}

Plan *find_plan(peval_poly *h, uint32_t K, uint32_t P, bool subtile_ends) {
  auto it = h->plans.find(plan_key(K, P, subtile_ends));
  return it == h->plans.end() ? nullptr : &it->second;
}

int get_plan(peval_poly *h, uint32_t K, uint32_t P, Plan **out, bool subtile_ends) {
  uint32_t key = plan_key(K, P, subtile_ends);
  auto it = h->plans.find(key);
  if (it != h->plans.end()) {
    *out = &it->second;
    return PEVAL_OK;
  }
  HostPlan hp = build_host_plan(h->grp_off, K, P, subtile_ends);
  Plan pl;
  pl.K = K;
  pl.P = P;
  pl.NT = hp.NT;
  pl.NW = hp.NW;
  pl.nslots = hp.nslots;
  int rc = PEVAL_OK;
  if ((rc = upload(&pl.d_thr_first, hp.thr_first)) != PEVAL_OK ||
      (rc = upload(&pl.d_thr_cnt, hp.thr_cnt)) != PEVAL_OK ||
      (rc = upload(&pl.d_endmask, hp.endmask)) != PEVAL_OK ||
      (rc = upload(&pl.d_slot_base, hp.slot_base)) != PEVAL_OK ||
      (rc = upload(&pl.d_slot_off, hp.slot_off)) != PEVAL_OK) {
    free_plan(pl);
    return rc;
  }
  pl.device_bytes = hp.NT * 5 + hp.NW * 12 + hp.slot_off.size() * 4;
  auto res = h->plans.emplace(key, pl);
  *out = &res.first->second;
  return PEVAL_OK;
}
}  // namespace peval

// ---------------------------------------------------------------------------
// create / destroy / info
// ---------------------------------------------------------------------------
// Host threads for an ingest pass over n terms: one per 2^16 terms, at most 8.
static unsigned ingest_threads(uint64_t n) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(std::min(hw, 8u), n >> 16));
}

// fn(lo, hi, t) over nt contiguous ranges of [0, n), range t on thread t.
template <class F>
static void par_ranges(uint64_t n, unsigned nt, F &&fn) {
  if (nt <= 1) {
    fn(0, n, 0u);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back([&fn, n, nt, t] { fn(n * t / nt, n * (t + 1) / nt, t); });
  fn(0, n / nt, 0u);
  for (auto &x : th) x.join();
}

extern "C" int peval_create(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exponents,
                            const uint64_t *coeffs, peval_poly **out) {
  if (!out) return fail(PEVAL_EINVAL, "out is NULL");
  *out = nullptr;
  if (p < 3 || (p & 1) == 0 || p >= (1ull << 63))
    return fail(PEVAL_EINVAL, "p must be odd with 3 <= p < 2^63 (got %llu)", (unsigned long long)p);
  if (n < 2 || n > 32) return fail(PEVAL_EINVAL, "n must be in [2, 32] (got %u)", n);
  if (s && (!exponents || !coeffs)) return fail(PEVAL_EINVAL, "null exponents or coefficients");
  if (s >= (1ull << 32) - 64) return fail(PEVAL_EUNSUPPORTED, "s >= 2^32 terms");
  const uint32_t ntail = n - 2;
  const unsigned nt = ingest_threads(s);
  uint32_t maxe[32] = {0};
  {
    std::vector<uint32_t> part((size_t)nt * 32, 0);
    par_ranges(s, nt, [&](uint64_t lo, uint64_t hi, unsigned t) {
      uint32_t *mx = &part[(size_t)t * 32];
      for (uint64_t i = lo; i < hi; ++i)
        for (uint32_t k = 0; k < n; ++k) mx[k] = std::max(mx[k], exponents[i * n + k]);
    });
    for (unsigned t = 0; t < nt; ++t)
      for (uint32_t k = 0; k < n; ++k) maxe[k] = std::max(maxe[k], part[(size_t)t * 32 + k]);
  }
  for (uint32_t k = 2; k < n; ++k)
    if (maxe[k] > 65535)
      return fail(PEVAL_EUNSUPPORTED, "exponent of x%u is %u > 65535", k + 1, maxe[k]);

  peval_poly *h = new (std::nothrow) peval_poly();
  if (!h) return fail(PEVAL_ENOMEM, "host allocation");
  h->p = p;
  h->n = n;
  h->s = s;
  h->w = p < (1ull << 31) ? 4 : 8;
  h->m64 = make_mod64(p);
  if (h->w == 4) h->m32 = make_mod32((uint32_t)p);
  h->mf.p = (double)p;
  h->mf.u = 1.0 / (double)p;
  h->mf.m = h->m64;
  h->arith = fp64_by_default(p) ? 1 : 0;
  std::copy(maxe, maxe + 32, h->max_exp);
  uint32_t off = 0;
  for (uint32_t k = 0; k < ntail; ++k) {
    h->tab.off[k] = off;
    off += maxe[k + 2] + 1;
  }
  h->tab.off[ntail] = off;
  h->tab_total = off;

  // A1: sort terms by (d, e) descending so that like monomials are adjacent
  // (stable: terms of one group keep their input order)
  std::vector<uint32_t> order(s);
  auto key = [&](uint64_t i) { return ((uint64_t)exponents[i * n] << 32) | exponents[i * n + 1]; };
  const uint64_t ext0 = (uint64_t)maxe[0] + 1, ext1 = (uint64_t)maxe[1] + 1;
  if (s && ext0 <= (1ull << 24) && ext1 <= (1ull << 24) && ext0 * ext1 <= (1ull << 24)) {
    // counting sort over the dense (d, e) grid, bin 0 = the largest key; each
    // thread counts its range, then scatters it after the earlier ranges'
    // terms of the same bin
    const uint64_t span = ext0 * ext1;
    const unsigned ns = span * nt <= (1ull << 22) ? nt : 1;  // per-thread counts stay small
    auto dense = [&](uint64_t i) {
      return (uint64_t)(maxe[0] - exponents[i * n]) * ext1 + (maxe[1] - exponents[i * n + 1]);
    };
    std::vector<uint32_t> cnt((size_t)ns * span, 0);
    par_ranges(s, ns, [&](uint64_t lo, uint64_t hi, unsigned t) {
      uint32_t *c = &cnt[(size_t)t * span];
      for (uint64_t i = lo; i < hi; ++i) c[dense(i)]++;
    });
    h->grp_off.push_back(0);
    uint64_t run = 0;
    for (uint64_t b = 0; b < span; ++b) {
      const uint64_t start = run;
      for (unsigned t = 0; t < ns; ++t) {
        const uint32_t c = cnt[(size_t)t * span + b];
        cnt[(size_t)t * span + b] = (uint32_t)run;
        run += c;
      }
      if (run > start) {  // a group: bin b holds terms
        h->gd.push_back((uint32_t)(maxe[0] - b / ext1));
        h->ge.push_back((uint32_t)(maxe[1] - b % ext1));
        h->grp_off.push_back(run);
      }
    }
    par_ranges(s, ns, [&](uint64_t lo, uint64_t hi, unsigned t) {
      uint32_t *c = &cnt[(size_t)t * span];
      for (uint64_t i = lo; i < hi; ++i) order[c[dense(i)]++] = (uint32_t)i;
    });
  } else {
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key(a) > key(b); });
    h->grp_off.push_back(0);
    for (uint64_t r = 0; r < s; ++r) {
      uint64_t k = key(order[r]);
      if (r == 0 || k != key(order[r - 1])) {
        if (r) h->grp_off.push_back(r);
        h->gd.push_back((uint32_t)(k >> 32));
        h->ge.push_back((uint32_t)k);
      }
    }
    if (s) h->grp_off.push_back(s);
  }
  h->G = h->gd.size();
  for (uint64_t g = 0; g < h->G; ++g) h->max_group = std::max(h->max_group, h->grp_off[g + 1] - h->grp_off[g]);

  // sorted structure-of-arrays: coefficients (reduced mod p) and tail exponents
  std::vector<uint8_t> coeff(s * h->w);
  std::vector<uint16_t> ex((size_t)ntail * s);
  par_ranges(s, nt, [&](uint64_t lo, uint64_t hi, unsigned) {
    for (uint64_t r = lo; r < hi; ++r) {
      uint64_t i = order[r];
      uint64_t a = coeffs[i] % p;
      if (h->w == 4) {
        uint32_t a32 = (uint32_t)a;
        memcpy(&coeff[r * 4], &a32, 4);
      } else {
        memcpy(&coeff[r * 8], &a, 8);
      }
      for (uint32_t k = 0; k < ntail; ++k) ex[(size_t)k * s + r] = (uint16_t)exponents[i * n + 2 + k];
    }
  });

  int rc = PEVAL_OK;
  auto bail = [&](int code) {
    peval_destroy(h);
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(PEVAL_EDEVICE, "hipGetDevice failed"));
  if ((rc = upload((uint8_t **)&h->d_coeff, coeff)) != PEVAL_OK) return bail(rc);
  if ((rc = upload(&h->d_exps, ex)) != PEVAL_OK) return bail(rc);
  h->resident_bytes = coeff.size() + ex.size() * 2;
  h->order = std::move(order);
  if (s && s <= kSmallMaxTerms) {  // group offsets for the single-launch path
    std::vector<uint32_t> off32(h->grp_off.begin(), h->grp_off.end());
    if ((rc = upload(&h->d_grp_off32, off32)) != PEVAL_OK) return bail(rc);
  }
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(PEVAL_EDEVICE, "stream creation failed"));
  if (hipEventCreateWithFlags(&h->done, hipEventDisableTiming) != hipSuccess)
    return bail(fail(PEVAL_EDEVICE, "event creation failed"));
  *out = h;
  return PEVAL_OK;
}

extern "C" int peval_destroy(peval_poly *h) {
  if (!h) return PEVAL_OK;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->have_done) (void)hipEventSynchronize(h->done);
    for (auto &kv : h->plans) free_plan(kv.second);
    h->plans.clear();
    release(h->tabval);
    release(h->tabquot);
    release(h->lam);
    release(h->gam);
    release(h->gamq);
    release(h->partial);
    release(h->outbuf);
    release(h->ptab);
    release(h->ptsbuf);
    for (auto &kv : h->pprep) {
      (void)hipFree(kv.second.pa);
      (void)hipFree(kv.second.paq);
      (void)hipFree(kv.second.pidx);
      (void)hipFree(kv.second.slot_term);
    }
    h->pprep.clear();
    release(h->iscr);
    if (h->d_order) (void)hipFree(h->d_order);
    if (h->d_grp_off32) (void)hipFree(h->d_grp_off32);
    if (h->d_gorder) (void)hipFree(h->d_gorder);
    if (h->d_task_group) (void)hipFree(h->d_task_group);
    if (h->d_task_first) (void)hipFree(h->d_task_first);
    for (auto &lv : h->d_mt)
      for (uint32_t *p : lv)
        if (p) (void)hipFree(p);
    if (h->d_coeff) (void)hipFree(h->d_coeff);
    if (h->d_exps) (void)hipFree(h->d_exps);
    if (h->done) (void)hipEventDestroy(h->done);
    if (h->stream) (void)hipStreamDestroy(h->stream);
  }
  delete h;
  return PEVAL_OK;
}

extern "C" int peval_info(const peval_poly *h, peval_info_t *info) {
  if (!h || !info) return fail(PEVAL_EINVAL, "null argument");
  memset(info, 0, sizeof *info);
  info->p = h->p;
  info->n = h->n;
  info->elem_bytes = h->w;
  info->s = h->s;
  info->G = h->G;
  uint64_t b = h->resident_bytes + h->tabval.bytes + h->tabquot.bytes + h->lam.bytes + h->gam.bytes +
               h->gamq.bytes + h->partial.bytes + h->outbuf.bytes + h->ptab.bytes + h->ptsbuf.bytes +
               h->iscr.bytes;
  for (auto &kv : h->plans) b += kv.second.device_bytes;
  for (auto &kv : h->pprep) {
    auto pl = h->plans.find(1u << 16 | kv.first << 8 | peval::kPointsP);
    if (pl != h->plans.end()) b += (uint64_t)kv.first * pl->second.NT * (2ull * h->w + 12);
  }
  if (h->d_order) b += (uint64_t)h->s * 4 + h->G * 4 + h->ntasks * 8;
  if (h->d_grp_off32) b += (h->G + 1) * 4;
  info->device_bytes = b;
  for (uint32_t k = 0; k < h->n && k < 32; ++k) info->max_exp[k] = h->max_exp[k];
  return PEVAL_OK;
}

extern "C" int peval_groups(const peval_poly *h, uint32_t *d, uint32_t *e) {
  if (!h || ((!d || !e) && h->G)) return fail(PEVAL_EINVAL, "null argument");
  if (h->G) {
    memcpy(d, h->gd.data(), h->G * 4);
    memcpy(e, h->ge.data(), h->G * 4);
  }
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
namespace peval {

bool valid_K(uint32_t K) { return K == 1 || K == 2 || K == 4 || K == 8 || K == 16 || K == 32; }
bool valid_P(uint32_t P) { return P == 8 || P == 16 || P == 32; }

uint64_t padded_threads(const peval_poly *h, uint32_t K) {
  uint64_t nt = 0;
  for (uint64_t g = 0; g < h->G; ++g) nt += (h->grp_off[g + 1] - h->grp_off[g] + K - 1) / K;
  return nt;
}

uint32_t chains_for_waves(uint64_t nw, uint64_t target_waves, uint32_t T) {
  uint64_t c = (target_waves + nw - 1) / std::max<uint64_t>(nw, 1);
  c = std::min<uint64_t>(std::max<uint64_t>(c, 1), 256);
  if (T) c = std::min<uint64_t>(c, T);
  return (uint32_t)std::max<uint64_t>(c, 1);
}

static uint64_t eval_block_slots(const peval_poly *h, uint32_t K, uint32_t P);

// Heuristic used before any autotuning: the largest K whose zero padding
// stays under 1/8 of the terms (up to 32 for 32-bit residues under the
// Shoup product, 8 under the FP64 product, 16 otherwise), P = 16, and
// enough chains for about 8192 waves; then up to four times as many chains
// (at least 8) where that fills the last round of blocks on the chip better
// than the extra chains cost.  Every wave of a run does the same work, so the blocks
// run in rounds of as many as the chip holds: 1e7 terms with K = 16 are 2442
// blocks per chain, 3.2 rounds of the 768 that fit, and the last round left
// four fifths of the chip idle (measured: 1 chain 18.7-18.8 ms, 5 chains
// 17.2 ms).  The model: evaluation time at the chip's rate times
// 1 + (idle share of the rounds) / 2 (the last round's waves run faster,
// having their SIMDs to fewer), plus per chain its chain starts written and
// read back (2 w bytes per term at about 4 TB/s).
Tuning heuristic_tuning(const peval_poly *h, uint32_t T) {
  Tuning t{1, 16, 1};
  const uint32_t kmax = h->arith == 1 ? 8 : (h->w == 4 && h->arith == 0) ? 32 : 16;
  for (uint32_t cand : {32u, 16u, 8u, 4u, 2u}) {
    if (cand > kmax) continue;
    if (padded_threads(h, cand) * cand * 8 <= h->s * 9) {
      t.K = cand;
      break;
    }
  }
  // Small groups: a K that holds every group in one thread (the images come
  // straight from the evaluation kernel, no segmented sums, partial sums or
  // combine) is worth up to three times the terms in zero padding.
  uint32_t kd = 1;
  while (kd < h->max_group && kd < kmax) kd *= 2;
  if (kd > t.K && kd >= h->max_group && (double)kd * h->G <= 3.0 * (double)h->s) t.K = kd;
  uint64_t nw = (padded_threads(h, t.K) + 63) / 64;
  t.C = chains_for_waves(nw, 8192, T);
  const uint64_t slots = eval_block_slots(h, t.K, t.P);
  if (slots && T) {
    const double per_chain = (double)((nw + 3) / 4);  // blocks of one chain
    const double terms = (double)nw * 64 * t.K;       // padded
    const double ops = h->arith == 1 ? 7 : (h->w == 4 ? 4 : 14);
    const double eval_s = terms * T * ops / 3.0e13, chain_s = terms * 2.0 * h->w / 4.0e12;
    auto cost = [&](uint32_t c) {
      const double r = c * per_chain / (double)slots;  // rounds of blocks
      return eval_s * (1.0 + 0.5 * (std::ceil(r) - r) / r) + c * chain_s;
    };
    double best = cost(t.C);
    const uint32_t c0 = t.C, cmax = std::min<uint32_t>(std::min<uint32_t>(std::max<uint32_t>(4 * c0, 8), 64), T);
    for (uint32_t c = c0 + 1; c <= cmax; ++c)
      if (cost(c) < best) {
        best = cost(c);
        t.C = c;
      }
  }
  return t;
}

uint32_t single_launch_L(const peval_poly *h, uint32_t T) {
  if (!h->d_grp_off32 || T == 0 || h->s > kSmallMaxTerms || h->s * h->w > kSmallRowBytes ||
      h->s * (uint64_t)T > kSmallMaxWork || h->max_group > kSmallMaxGroup)
    return 0;
  const uint64_t tab = 2ull * h->tab_total * h->w, row = h->s * (uint64_t)h->w;
  if (tab + row > kSmallLds) return 0;
  const uint64_t fit = (kSmallLds - tab) / row;  // evaluations whose term values fit in LDS
  return (uint32_t)std::min<uint64_t>(fit, (T + kSmallTargetBlocks - 1) / kSmallTargetBlocks);
}

// Tuning for a run of T evaluations: explicit settings first, then the
// autotuner's cache for this shape, then the heuristic.  Small runs take the
// single-launch path unless a tuning is set, the autotuner chose a
// multi-kernel tuning for the shape, or the product was chosen explicitly.
Tuning choose_tuning(const peval_poly *h, uint32_t T) {
  Tuning t = heuristic_tuning(h, T);
  Tuning cached;
  const bool hit = tune_cache_lookup(h, T, &cached);
  if (hit && !cached.L) t = cached;
  if (h->tune_K) t.K = h->tune_K;
  if (h->tune_P) t.P = h->tune_P;
  if (h->tune_C) t.C = h->tune_C;
  if (h->arith == 1) t.K = std::min<uint32_t>(t.K, 8);  // exact double sums of at most 8 residues
  if (h->w == 8 || h->arith != 0) t.K = std::min<uint32_t>(t.K, 16);  // K = 32: 32-bit Shoup only
  if (T) t.C = std::min<uint32_t>(t.C, T);
  t.C = std::max<uint32_t>(t.C, 1);
  const bool forced = h->tune_K || h->tune_P || h->tune_C;
  if (!forced && h->arith_auto && (!hit || cached.L)) t.L = single_launch_L(h, T);
  return t;
}

}  // namespace peval

extern "C" int peval_set_tuning(peval_poly *h, uint32_t K, uint32_t P, uint32_t C) {
  if (!h) return fail(PEVAL_EINVAL, "null handle");
  if (K && !valid_K(K)) return fail(PEVAL_EINVAL, "K must be 1, 2, 4, 8, 16 or 32");
  if (K == 32 && h->w != 4) return fail(PEVAL_EINVAL, "K = 32 needs 32-bit residues (p < 2^31)");
  if (P && !valid_P(P)) return fail(PEVAL_EINVAL, "P must be 8, 16 or 32");
  if (C > 65535) return fail(PEVAL_EINVAL, "C must be <= 65535");
  std::lock_guard<std::mutex> lk(h->mu);
  h->tune_K = K;
  h->tune_P = P;
  h->tune_C = C;
  return PEVAL_OK;
}

// p = 2^63 - c with c < 2^20, or p = 2^31 - c with c < 2^12
static bool pseudo_mersenne(uint64_t p) {
  if (p < (1ull << 63) && p > (1ull << 63) - (1ull << 20)) return true;
  return p < (1ull << 31) && p > (1ull << 31) - (1ull << 12);
}

extern "C" int peval_set_arith(peval_poly *h, uint32_t mode) {
  if (!h) return fail(PEVAL_EINVAL, "null handle");
  if (mode > PEVAL_ARITH_PMERSENNE) return fail(PEVAL_EINVAL, "unknown arithmetic %u", mode);
  if (mode == PEVAL_ARITH_FP64 && (h->p < (1ull << 31) || h->p >= (1ull << 50)))
    return fail(PEVAL_EUNSUPPORTED, "the FP64 product needs 2^31 <= p < 2^50");
  if (mode == PEVAL_ARITH_PMERSENNE && !pseudo_mersenne(h->p))
    return fail(PEVAL_EUNSUPPORTED, "the pseudo-Mersenne product needs p = 2^63 - c (c < 2^20) or 2^31 - c (c < 2^12)");
  std::lock_guard<std::mutex> lk(h->mu);
  if (mode == PEVAL_ARITH_PMERSENNE) {
    h->arith = 2;
    h->arith_auto = false;
    h->mpm64 = ModPM64{h->p, (1ull << 63) - h->p, h->m64};
    if (h->w == 4) h->mpm32 = ModPM32{(uint32_t)h->p, (uint32_t)((1ull << 31) - h->p), h->m32};
    return PEVAL_OK;
  }
  h->arith = (mode == PEVAL_ARITH_FP64 || (mode == PEVAL_ARITH_AUTO && fp64_by_default(h->p))) ? 1 : 0;
  h->arith_auto = mode == PEVAL_ARITH_AUTO;
  return PEVAL_OK;
}

extern "C" int peval_get_arith(const peval_poly *h, uint32_t *mode) {
  if (!h || !mode) return fail(PEVAL_EINVAL, "null argument");
  *mode = h->arith == 1 ? PEVAL_ARITH_FP64 : h->arith == 2 ? PEVAL_ARITH_PMERSENNE : PEVAL_ARITH_INT;
  return PEVAL_OK;
}

extern "C" int peval_get_tuning(peval_poly *h, uint32_t T, uint32_t *K, uint32_t *P, uint32_t *C) {
  if (!h || !K || !P || !C) return fail(PEVAL_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(h->mu);
  Tuning t = choose_tuning(h, T);
  *K = t.L ? 0 : t.K;
  *P = t.L ? 0 : t.P;
  *C = t.L ? 0 : t.C;
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------
template <class A>
struct Dispatch {
  using EvalFn = void (*)(EvalArgs<A>);
  static EvalFn eval(uint32_t K, uint32_t P) {
#define PEVAL_CASE(k, pp) \
  if (K == k && P == pp) return eval_kernel<A, k, pp>;
#define PEVAL_CASES_K(k) PEVAL_CASE(k, 8) PEVAL_CASE(k, 16) PEVAL_CASE(k, 32)
    PEVAL_CASES_K(1)
    PEVAL_CASES_K(2)
    PEVAL_CASES_K(4)
    PEVAL_CASES_K(8)
    PEVAL_CASES_K(16)
    if constexpr (sizeof(typename A::T) == 4) {  // 32 running values of 64 bits would not fit two waves
      PEVAL_CASE(32, 8)
      PEVAL_CASE(32, 16)
    }
#undef PEVAL_CASES_K
#undef PEVAL_CASE
    return nullptr;
  }
};

template <>
struct Dispatch<WF64> {  // a thread sums at most 8 doubles exactly: K <= 8
  using EvalFn = void (*)(EvalArgs<WF64>);
  static EvalFn eval(uint32_t K, uint32_t P) {
#define PEVAL_CASE(k, pp) \
  if (K == k && P == pp) return eval_kernel<WF64, k, pp>;
#define PEVAL_CASES_K(k) PEVAL_CASE(k, 8) PEVAL_CASE(k, 16) PEVAL_CASE(k, 32)
    PEVAL_CASES_K(1)
    PEVAL_CASES_K(2)
    PEVAL_CASES_K(4)
    PEVAL_CASES_K(8)
#undef PEVAL_CASES_K
#undef PEVAL_CASE
    return nullptr;
  }
};

// Pseudo-Mersenne products: P = 16 only.
template <class A>
struct DispatchPM {
  using EvalFn = void (*)(EvalArgs<A>);
  static EvalFn eval(uint32_t K) {
    switch (K) {
      case 1: return eval_kernel<A, 1, 16>;
      case 2: return eval_kernel<A, 2, 16>;
      case 4: return eval_kernel<A, 4, 16>;
      case 8: return eval_kernel<A, 8, 16>;
      case 16: return eval_kernel<A, 16, 16>;
      default: return nullptr;
    }
  }
};
template <>
struct Dispatch<W64PM> {
  static void (*eval(uint32_t K, uint32_t))(EvalArgs<W64PM>) { return DispatchPM<W64PM>::eval(K); }
};
template <>
struct Dispatch<W32PM> {
  static void (*eval(uint32_t K, uint32_t))(EvalArgs<W32PM>) { return DispatchPM<W32PM>::eval(K); }
};

// Blocks of the evaluation kernel for (K, P) and the handle's product that
// the device holds at once (0 if unknown); queried once per variant.
namespace peval {
static uint64_t eval_block_slots(const peval_poly *h, uint32_t K, uint32_t P) {
  static std::mutex mu;
  static std::map<uint32_t, uint64_t> cache;
  const uint32_t key = (uint32_t)h->w << 24 | h->arith << 16 | K << 8 | P;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const void *fn = nullptr;
  if (h->w == 4)
    fn = h->arith == 2 ? (const void *)Dispatch<W32PM>::eval(K, 16) : (const void *)Dispatch<W32>::eval(K, P);
  else
    fn = h->arith == 1   ? (const void *)Dispatch<WF64>::eval(K, P)
         : h->arith == 2 ? (const void *)Dispatch<W64PM>::eval(K, 16)
                         : (const void *)Dispatch<W64>::eval(K, P);
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  uint64_t slots = 0;
  if (fn && hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kEvalBlock, 0) == hipSuccess)
    slots = (uint64_t)per_cu * prop.multiProcessorCount;
  else
    (void)hipGetLastError();
  cache[key] = slots;
  return slots;
}
}  // namespace peval

template <class A>
static const typename A::M &mod_of(const peval_poly *h);
template <>
const Mod64 &mod_of<W64>(const peval_poly *h) { return h->m64; }
template <>
const Mod32 &mod_of<W32>(const peval_poly *h) { return h->m32; }
template <>
const ModF64 &mod_of<WF64>(const peval_poly *h) { return h->mf; }
template <>
const ModPM64 &mod_of<W64PM>(const peval_poly *h) { return h->mpm64; }
template <>
const ModPM32 &mod_of<W32PM>(const peval_poly *h) { return h->mpm32; }

static constexpr size_t kPartialBudget = (size_t)2 << 30;  // bytes of partial sums per launch

// A: integer policy of the prologue, partial sums and output; E: policy of
// the evaluation kernel (A itself, or the FP64 product on 64-bit residues).
template <class A, class E = A>
static int run_impl(peval_poly *h, const BetaArg &beta, uint64_t t0, uint32_t T, void *dev_out,
                    hipStream_t st, const Tuning &tu, const FixedScratch *fixed) {
  using T_ = typename A::T;
  const auto &m = mod_of<A>(h);
  constexpr bool fp = std::is_same<E, WF64>::value;
  constexpr bool pm = std::is_same<E, W64PM>::value || std::is_same<E, W32PM>::value;
  const uint32_t ntail = h->n - 2;
  const uint32_t K = tu.K, P = pm ? 16 : tu.P;
  uint32_t C = tu.C;
  Plan *pl = nullptr;
  if (fixed) {
    pl = find_plan(h, K, P);
    if (!pl)
      return fail(PEVAL_EUNSUPPORTED,
                  "no thread layout for K=%u P=%u on this handle yet (a peval_run_async with this tuning makes it)",
                  K, P);
  } else {
    PEVAL_TRY(get_plan(h, K, P, &pl));
  }
  const size_t w = sizeof(T_);
  auto eval = Dispatch<E>::eval(K, P);
  if (!eval) return fail(PEVAL_EINVAL, "no kernel for K=%u P=%u", K, P);

  // Every group within one thread's K terms: the evaluation kernel writes
  // the images itself (no partial sums, no combine).
  const bool direct = (uint64_t)K >= h->max_group;
  // T is processed in chunks so that the partial sums stay within budget
  const size_t tab_bytes = (size_t)std::max<uint32_t>(h->tab_total, 1) * w;
  const size_t chain_bytes = (size_t)K * pl->NT * w;  // chain starts of one chain; also Gamma, Gamma'
  const size_t row_bytes = direct ? 1 : (size_t)pl->nslots * w;  // partial sums of one evaluation
  uint64_t tc = std::max<uint64_t>(1, kPartialBudget / std::max<size_t>(1, row_bytes));
  void *tabval, *tabquot, *lam, *gam, *gamq, *partial;
  uint64_t fit_rows = 0;  // rows of partial sums that fit the caller's region
  if (fixed) {
    // everything in the caller's region: tables, Gamma, Gamma', then as many
    // chains as fit beside at least one row of partial sums, then the rows
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t head = 2 * up(tab_bytes) + 2 * up(chain_bytes);
    if (head + up(chain_bytes) + up(row_bytes) + 256 > fixed->bytes)
      return fail(PEVAL_EUNSUPPORTED,
                  "run needs at least %zu bytes of scratch (%zu available): %llu terms are too many",
                  head + up(chain_bytes) + up(row_bytes) + 256, fixed->bytes, (unsigned long long)h->s);
    const uint64_t cfit = (fixed->bytes - head - up(row_bytes) - 256) / std::max<size_t>(chain_bytes, 1);
    C = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(C, cfit));
    unsigned char *b = fixed->base;
    tabval = b;
    tabquot = b + up(tab_bytes);
    gam = b + 2 * up(tab_bytes);
    gamq = b + 2 * up(tab_bytes) + up(chain_bytes);
    lam = b + head;
    const size_t lam_end = head + up((size_t)C * chain_bytes);
    partial = b + lam_end;
    fit_rows = (fixed->bytes - lam_end) / std::max<size_t>(row_bytes, 1);  // >= 1 by the choice of C
    tc = std::min<uint64_t>(tc, fit_rows);
  }
  tc = std::min<uint64_t>(tc, (uint64_t)C * kCombineTile * 32768);  // keeps grid.z of the combine in range
  tc = std::min<uint64_t>(tc, T);
  if (tc < T && tc > C) tc = tc / C * C;
  if (fixed) {
    // a chunk of x evaluations on min(C, x) chains fills whole rounds of rows
    const uint64_t cc = std::min<uint64_t>(C, tc), rows = (tc + cc - 1) / cc * cc;
    if (rows > fit_rows) tc = fit_rows >= C ? fit_rows / C * C : fit_rows;
  }
  if (!fixed) {
    PEVAL_TRY(ensure(h->tabval, tab_bytes, h));
    PEVAL_TRY(ensure(h->tabquot, tab_bytes, h));
    PEVAL_TRY(ensure(h->lam, (size_t)C * chain_bytes, h));
    PEVAL_TRY(ensure(h->gam, chain_bytes, h));
    PEVAL_TRY(ensure(h->gamq, chain_bytes, h));
    PEVAL_TRY(ensure(h->partial, (size_t)((tc + C - 1) / C) * C * row_bytes, h));
    tabval = h->tabval.ptr;
    tabquot = h->tabquot.ptr;
    lam = h->lam.ptr;
    gam = h->gam.ptr;
    gamq = h->gamq.ptr;
    partial = h->partial.ptr;
  }

  // A2: power tables
  if (ntail) {
    ProfScope ps(st, 0);
    uint32_t blocks = (h->tab_total + 255) / 256;
    power_table_kernel<A><<<blocks, 256, 0, st>>>(beta, h->tab, ntail, h->tab_total, (T_ *)tabval,
                                                  (T_ *)tabquot, m);
    HIP_TRY(hipGetLastError());
  }

  for (uint64_t done = 0; done < T; done += tc) {
    const uint32_t Tc = (uint32_t)std::min<uint64_t>(tc, T - done);
    const uint32_t Cc = std::min<uint32_t>(C, Tc);
    {  // A3: monomial values and chain starts
      MonoArgs<A> ma;
      ma.coeff = (const T_ *)h->d_coeff;
      ma.exps = h->d_exps;
      ma.tval = (const T_ *)tabval;
      ma.tquot = (const T_ *)tabquot;
      ma.to = h->tab;
      ma.thr_first = pl->d_thr_first;
      ma.thr_cnt = pl->d_thr_cnt;
      ma.lam = (T_ *)lam;
      ma.gam = (T_ *)gam;
      ma.gamq = (T_ *)gamq;
      ma.s = h->s;
      ma.NT = pl->NT;
      ma.t0 = t0 + done;
      ma.ntail = ntail;
      ma.K = K;
      ma.C = Cc;
      ma.as_double = fp ? 1 : 0;
      ma.m = m;
      ma.R = mono_slots_for(K, (uint64_t)K * pl->NT);
      ma.tab_total = h->tab_total;
      const uint64_t total = (uint64_t)K * pl->NT / ma.R;  // work-items
      ma.xchunk = (uint32_t)(((total + 255) / 256 + kXcds - 1) / kXcds);
      ProfScope ps(st, 1);
      monomial_kernel<A><<<kXcds * ma.xchunk, 256, 0, st>>>(ma);
      HIP_TRY(hipGetLastError());
    }
    {  // A4-A6: evaluations
      using TE = typename E::T;
      EvalArgs<E> ea;
      ea.lam = (const TE *)lam;
      ea.gam = (const TE *)gam;
      ea.gamq = (const TE *)gamq;
      ea.endmask = pl->d_endmask;
      ea.slot_base = pl->d_slot_base;
      ea.partial = (typename E::PT *)partial;
      ea.NT = pl->NT;
      ea.NW = pl->NW;
      ea.nslots = pl->nslots;
      ea.C = Cc;
      ea.T = Tc;
      ea.Lmax = (Tc + Cc - 1) / Cc;
      ea.m = mod_of<E>(h);
      ea.direct = direct ? 1 : 0;
      ea.G = h->G;
      ea.out = (typename E::PT *)dev_out + done * h->G;
      dim3 grid((unsigned)((pl->NW + 3) / 4), Cc);
      ProfScope ps(st, 2);
      eval<<<grid, kEvalBlock, 0, st>>>(ea);
      HIP_TRY(hipGetLastError());
    }
    if (!direct) {  // A7: combine
      CombineArgs<A> ca;
      ca.partial = (const T_ *)partial;
      ca.slot_off = pl->d_slot_off;
      ca.out = (T_ *)dev_out + done * h->G;
      ca.G = h->G;
      ca.C = Cc;
      ca.T = Tc;
      ca.Lmax = (Tc + Cc - 1) / Cc;
      ca.m = m;
      dim3 grid((unsigned)((h->G + kCombineTile - 1) / kCombineTile), Cc,
                (unsigned)((ca.Lmax + kCombineTile - 1) / kCombineTile));
      ProfScope ps(st, 3);
      combine_kernel<A><<<grid, kCombineBlock, 0, st>>>(ca);
      HIP_TRY(hipGetLastError());
    }
  }
  return PEVAL_OK;
}

// Single-launch path: tables, chain starts, evaluations and group sums in
// one kernel (small runs, where the four launches would dominate).
template <class A>
static int run_small(peval_poly *h, const BetaArg &beta, uint64_t t0, uint32_t T, void *dev_out, hipStream_t st,
                     uint32_t L) {
  using T_ = typename A::T;
  const uint64_t lds = (2ull * h->tab_total + (uint64_t)L * h->s) * sizeof(T_);
  if (L == 0 || lds > kSmallLds || !h->d_grp_off32)
    return fail(PEVAL_EINVAL, "single-launch path does not fit (L=%u)", L);
  SmallArgs<A> a;
  a.coeff = (const T_ *)h->d_coeff;
  a.exps = h->d_exps;
  a.grp_off = h->d_grp_off32;
  a.out = (T_ *)dev_out;
  a.beta = beta;
  a.to = h->tab;
  a.t0 = t0;
  a.s = (uint32_t)h->s;
  a.G = (uint32_t)h->G;
  a.T = T;
  a.L = L;
  a.ntail = h->n - 2;
  a.tab_total = h->tab_total;
  a.m = mod_of<A>(h);
  ProfScope ps(st, 2);
  small_run_kernel<A><<<(T + L - 1) / L, kSmallBlock, (size_t)lds, st>>>(a);
  HIP_TRY(hipGetLastError());
  return PEVAL_OK;
}

namespace peval {

int check_run_args(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T, BetaArg *ba) {
  if (!h) return fail(PEVAL_EINVAL, "null handle");
  if (h->n > 2 && !beta) return fail(PEVAL_EINVAL, "null beta");
  if (t0 < 1) return fail(PEVAL_EINVAL, "t0 must be >= 1");
  if ((uint64_t)T * h->G > (1ull << 40)) return fail(PEVAL_EUNSUPPORTED, "T*G too large");
  memset(ba, 0, sizeof *ba);
  for (uint32_t k = 0; k + 2 < h->n; ++k) ba->b[k] = beta[k] % h->p;
  return PEVAL_OK;
}

// Enqueue one run on stream st (handle lock held by the caller).
int run_locked(peval_poly *h, const BetaArg &ba, uint64_t t0, uint32_t T, void *dev_out, hipStream_t st,
               const Tuning &tu, const FixedScratch *fixed) {
  HIP_TRY(hipSetDevice(h->device));
  if (h->have_done) HIP_TRY(hipStreamWaitEvent(st, h->done, 0));
  int rc;
  if (tu.L)
    rc = (h->w == 4) ? run_small<W32>(h, ba, t0, T, dev_out, st, tu.L) : run_small<W64>(h, ba, t0, T, dev_out, st, tu.L);
  else if (h->w == 4)
    rc = (h->arith == 2) ? run_impl<W32, W32PM>(h, ba, t0, T, dev_out, st, tu, fixed)
                         : run_impl<W32>(h, ba, t0, T, dev_out, st, tu, fixed);
  else
    rc = (h->arith == 1)   ? run_impl<W64, WF64>(h, ba, t0, T, dev_out, st, tu, fixed)
         : (h->arith == 2) ? run_impl<W64, W64PM>(h, ba, t0, T, dev_out, st, tu, fixed)
                           : run_impl<W64>(h, ba, t0, T, dev_out, st, tu, fixed);
  if (rc != PEVAL_OK) return rc;
  HIP_TRY(hipEventRecord(h->done, st));
  h->have_done = true;
  return PEVAL_OK;
}

}  // namespace peval

extern "C" int peval_run_async(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T,
                               void *dev_out, void *stream) {
  BetaArg ba;
  PEVAL_TRY(check_run_args(h, beta, t0, T, &ba));
  if (T == 0 || h->G == 0) return PEVAL_OK;
  if (!dev_out) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(h->mu);
  return run_locked(h, ba, t0, T, dev_out, (hipStream_t)stream, choose_tuning(h, T));
}

// ---------------------------------------------------------------------------
// allocation-free entry point
// ---------------------------------------------------------------------------
// One fixed scratch region per GPU for peval_run_async_noalloc.  In host code
// `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;  // device -> address of its copy of `scratch`
}  // namespace

// Address of the current device's scratch (device `dev` must be current).
static int scratch_address(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PEVAL_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    it = g_scratch_addr.emplace(dev, (unsigned char *)ptr).first;
  }
  *out = it->second;
  return PEVAL_OK;
}

extern "C" int peval_run_async_noalloc(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T,
                                       void *dev_out, void *stream) {
  BetaArg ba;
  PEVAL_TRY(check_run_args(h, beta, t0, T, &ba));
  if (T == 0 || h->G == 0) return PEVAL_OK;
  if (!dev_out) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(h->mu);
  HIP_TRY(hipSetDevice(h->device));
  FixedScratch fx;
  PEVAL_TRY(scratch_address(h->device, &fx.base));
  fx.bytes = kNoAllocScratchBytes;
  ProfOff no_events;
  return run_locked(h, ba, t0, T, dev_out, (hipStream_t)stream, choose_tuning(h, T), &fx);
}

extern "C" int peval_run(peval_poly *h, const uint64_t *beta, uint32_t T, void *out) {
  BetaArg ba;
  PEVAL_TRY(check_run_args(h, beta, 1, T, &ba));
  if (T == 0 || h->G == 0) return PEVAL_OK;
  if (!out) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(h->mu);
  const size_t bytes = (size_t)T * h->G * h->w;
  PEVAL_TRY(ensure(h->outbuf, bytes, h));
  PEVAL_TRY(run_locked(h, ba, 1, T, h->outbuf.ptr, h->stream, choose_tuning(h, T)));
  HIP_TRY(hipMemcpyAsync(out, h->outbuf.ptr, bytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PEVAL_OK;
}
