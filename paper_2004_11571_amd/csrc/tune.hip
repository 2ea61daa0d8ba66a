// Autotuner for the evaluation kernel's K (terms per thread), P (evaluations
// per pass) and C (independent chains).
//
// The paper tunes its blocking (T_i, T_d, M) by sweeping every combination
// and timing it (Section 4.4, Fig. 4).  Here the analogous knobs are timed
// on the device for the polynomial at hand and the winner is cached per
// shape class, so later polynomials of a similar shape (and the batched
// launches) reuse it without timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "errors.hpp"
#include "peval_internal.hpp"

namespace peval {

namespace {

// Shape class: residue width, term count, mean group size and T, each on a
// half-octave grid.
using ShapeKey = std::tuple<uint32_t, int, int, int>;

struct TuneEntry {
  Tuning t;
  float ms;
};

std::mutex g_tune_mu;
std::map<ShapeKey, TuneEntry> g_tune;

int half_octave(double v) { return v <= 1 ? 0 : (int)std::floor(2.0 * std::log2(v)); }

ShapeKey shape_key(const peval_poly *h, uint32_t T) {
  double mean_group = h->G ? (double)h->s / (double)h->G : 1.0;
  return ShapeKey{h->w, half_octave((double)h->s), half_octave(mean_group), half_octave((double)T)};
}

}  // namespace

bool tune_cache_lookup(const peval_poly *h, uint32_t T, Tuning *out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(shape_key(h, T));
  if (it == g_tune.end()) return false;
  *out = it->second.t;
  return true;
}

static int time_run(peval_poly *h, const BetaArg &ba, uint32_t T, const Tuning &tu, int reps, float *best_ms) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  int rc = PEVAL_OK;
  for (int r = 0; r <= reps && rc == PEVAL_OK; ++r) {  // r == 0 warms up
    if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(PEVAL_EDEVICE, "event record"); break; }
    rc = run_locked(h, ba, 1, T, h->outbuf.ptr, h->stream, tu);
    if (rc != PEVAL_OK) break;
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(PEVAL_EDEVICE, "event wait");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (r > 0) best = std::min(best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return rc;
}

}  // namespace peval

using namespace peval;

extern "C" int peval_autotune(peval_poly *h, const uint64_t *beta, uint32_t T, uint32_t exhaustive,
                              uint32_t *K, uint32_t *P, uint32_t *C, float *ms) {
  BetaArg ba;
  PEVAL_TRY(check_run_args(h, beta, 1, T, &ba));
  if (T == 0) return fail(PEVAL_EINVAL, "T must be >= 1");
  if (h->G == 0) {
    if (K) *K = 1;
    if (P) *P = 16;
    if (C) *C = 1;
    if (ms) *ms = 0;
    return PEVAL_OK;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  PEVAL_TRY(ensure(h->outbuf, (size_t)T * h->G * h->w, h));

  // the FP64 product sums at most 8 doubles per thread exactly: K <= 8;
  // 32 terms per thread for 32-bit residues under the Shoup product only,
  // with at most 16 evaluations per pass
  const uint32_t kmax = (h->arith == 1) ? 8u : (h->w == 4 && h->arith == 0) ? 32u : 16u;
  std::vector<uint32_t> Ks;
  for (uint32_t k : {1u, 2u, 4u, 8u, 16u, 32u})
    if (k <= kmax && (k == 1 || padded_threads(h, k) * k * 2 <= h->s * 3)) Ks.push_back(k);
  const uint32_t Ps[] = {8, 16, 32};
  auto has_kernel = [](uint32_t k, uint32_t p) { return k < 32 || p <= 16; };
  // chain counts for about this many waves (the chip holds 3072-4096 of
  // the evaluation kernel at once, so the larger ones fill the last round
  // of a large run better)
  const uint64_t targets[] = {2048, 4096, 8192, 16384, 32768, 65536};
  auto chains = [&](uint32_t k, uint64_t target) {
    uint64_t nw = (padded_threads(h, k) + 63) / 64;
    return chains_for_waves(nw, target, T);
  };

  Tuning best = heuristic_tuning(h, T);
  best.K = std::min(best.K, kmax);
  const Tuning heur = best;
  float best_ms = 1e30f;
  // a candidate replaces the current choice only when it is faster by more
  // than the spread of repeated timings, so that ties keep the heuristic's
  // (considered first) and the choice is stable from process to process
  const float margin = 0.985f;
  auto consider = [&](Tuning t) -> int {
    float m = 0;
    PEVAL_TRY(time_run(h, ba, T, t, 2, &m));
    if (m < best_ms * margin) {
      best_ms = m;
      best = t;
    }
    return PEVAL_OK;
  };

  // a few untimed runs first: the candidate timed first would otherwise meet
  // the device still raising its clocks
  {
    float warm_ms = 0;
    PEVAL_TRY(time_run(h, ba, T, heur, 3, &warm_ms));
  }
  if (exhaustive) {
    for (uint32_t k : Ks)
      for (uint32_t p : Ps) {
        if (!has_kernel(k, p)) continue;
        std::vector<uint32_t> seen;
        for (uint64_t tg : targets) {
          uint32_t c = chains(k, tg);
          if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
          seen.push_back(c);
          PEVAL_TRY(consider(Tuning{k, p, c}));
        }
      }
  } else {  // coordinate search from the heuristic's choice: K, then P, then C
    PEVAL_TRY(consider(heur));
    Tuning t0 = best;
    for (uint32_t k : Ks) PEVAL_TRY(consider(Tuning{k, t0.P, chains(k, 8192)}));
    Tuning t1 = best;
    for (uint32_t p : Ps)
      if (p != t1.P && has_kernel(t1.K, p)) PEVAL_TRY(consider(Tuning{t1.K, p, t1.C}));
    Tuning t2 = best;
    std::vector<uint32_t> tried{t2.C};
    for (uint64_t tg : targets) {
      uint32_t c = chains(t2.K, tg);
      if (std::find(tried.begin(), tried.end(), c) != tried.end()) continue;
      tried.push_back(c);
      PEVAL_TRY(consider(Tuning{t2.K, t2.P, c}));
    }
  }
  // the single-launch path, where the run fits it
  const uint32_t L = h->arith_auto ? single_launch_L(h, T) : 0;
  if (L) {
    Tuning t = best;
    t.L = L;
    PEVAL_TRY(consider(t));
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[shape_key(h, T)] = TuneEntry{best, best_ms};
  }
  if (K) *K = best.L ? 0 : best.K;
  if (P) *P = best.L ? 0 : best.P;
  if (C) *C = best.L ? 0 : best.C;
  if (ms) *ms = best_ms;
  return PEVAL_OK;
}

extern "C" int peval_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  return PEVAL_OK;
}

extern "C" int peval_tune_save(const char *path) {
  if (!path) return fail(PEVAL_EINVAL, "null path");
  std::lock_guard<std::mutex> g(g_tune_mu);
  FILE *f = fopen(path, "w");
  if (!f) return fail(PEVAL_EINVAL, "cannot open %s", path);
  fprintf(f, "# peval tuning cache: width s_class group_class T_class K P C ms (K P C = 0 0 0: single launch)\n");
  for (auto &kv : g_tune) {
    const Tuning &t = kv.second.t;
    fprintf(f, "%u %d %d %d %u %u %u %.6f\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
            std::get<3>(kv.first), t.L ? 0 : t.K, t.L ? 0 : t.P, t.L ? 0 : t.C, kv.second.ms);
  }
  fclose(f);
  return PEVAL_OK;
}

extern "C" int peval_tune_load(const char *path) {
  if (!path) return fail(PEVAL_EINVAL, "null path");
  FILE *f = fopen(path, "r");
  if (!f) return fail(PEVAL_EINVAL, "cannot open %s", path);
  char line[256];
  std::map<ShapeKey, TuneEntry> add;
  int rc = PEVAL_OK;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    unsigned w, k, p, c;
    int sb, gb, tb;
    float ms;
    const int got = sscanf(line, "%u %d %d %d %u %u %u %f", &w, &sb, &gb, &tb, &k, &p, &c, &ms);
    const bool single = got == 8 && k == 0 && p == 0 && c == 0;
    if (got != 8 || (w != 4 && w != 8) || (!single && (!valid_K(k) || !valid_P(p) || c == 0 || c > 65535))) {
      rc = fail(PEVAL_EINVAL, "bad tuning line: %s", line);
      break;
    }
    Tuning t{k, p, c};
    if (single) t.L = 1;  // recomputed for each polynomial when used
    add[ShapeKey{w, sb, gb, tb}] = TuneEntry{t, ms};
  }
  fclose(f);
  if (rc != PEVAL_OK) return rc;
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto &kv : add) g_tune[kv.first] = kv.second;
  return PEVAL_OK;
}
