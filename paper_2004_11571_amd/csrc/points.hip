// Point mode: images at T arbitrary points (paper, Section 2.1: the random
// points of Zippel's method; Section 2.3 puts their cost at O(nT(d+s))).
// Kernels in points_kernels.hpp; the thread layout, partial sums and combine
// are the power path's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <type_traits>

#include "errors.hpp"
#include "peval.h"
#include "peval_testing.h"
#include "peval_internal.hpp"

using namespace peval;

namespace peval {

// Digits: a tail variable of degree bound D becomes one digit of radix D+1,
// or two base-256 digits when D >= 256; variables that never occur are
// dropped.  Digits are then spread over nf factors (smallest nf first),
// largest radix first, each into the factor whose table grows least; a plan
// is accepted when all tables of one point fit in kPointsTableBytes.
int build_factor_plan(uint32_t w, uint32_t ntail, const uint32_t *maxdeg, FactorPlan *fp) {
  FactorPlan f{};
  struct Dig {
    uint8_t var, shift;
    uint16_t mask, radix;
  };
  std::vector<Dig> dig;
  for (uint32_t v = 0; v < ntail; ++v) {
    const uint32_t D = maxdeg[v];
    if (D == 0) continue;
    if (D + 1 <= 256) {
      dig.push_back({(uint8_t)v, 0, 0xffff, (uint16_t)(D + 1)});
    } else {
      dig.push_back({(uint8_t)v, 0, 0xff, 256});
      dig.push_back({(uint8_t)v, 8, 0xff, (uint16_t)((D >> 8) + 1)});
    }
  }
  std::stable_sort(dig.begin(), dig.end(), [](const Dig &a, const Dig &b) { return a.radix > b.radix; });
  const uint64_t emax = kPointsTableBytes / (2 * w);
  if (dig.empty()) {  // the tail monomial is 1 for every term
    f.nf = 1;
    f.f_off[0] = 0;
    f.f_off[1] = 1;
    f.E = w == 4 ? 4 : 2;
    *fp = f;
    return PEVAL_OK;
  }
  for (uint32_t nf = 1; nf <= (uint32_t)kMaxFactors; ++nf) {
    uint64_t size[kMaxFactors] = {1, 1, 1, 1};
    std::vector<uint32_t> fac(dig.size());
    for (size_t d = 0; d < dig.size(); ++d) {
      uint32_t best = 0;
      for (uint32_t b = 1; b < nf; ++b)
        if (size[b] < size[best]) best = b;  // smallest table grows least
      fac[d] = best;
      size[best] *= dig[d].radix;
    }
    uint64_t total = 0;
    uint32_t used = 0;
    for (uint32_t b = 0; b < nf; ++b)
      if (size[b] > 1) total += size[b], ++used;
    if (used < nf || total > emax) continue;
    // strides inside each factor, in digit order
    uint64_t place[kMaxFactors] = {1, 1, 1, 1};
    f.ndig = (uint32_t)dig.size();
    f.nf = nf;
    for (size_t d = 0; d < dig.size(); ++d) {
      f.var[d] = dig[d].var;
      f.fac[d] = (uint8_t)fac[d];
      f.shift[d] = dig[d].shift;
      f.mask[d] = dig[d].mask;
      f.radix[d] = dig[d].radix;
      f.stride[d] = (uint32_t)place[fac[d]];
      place[fac[d]] *= dig[d].radix;
    }
    f.f_off[0] = 0;
    for (uint32_t b = 0; b < nf; ++b) f.f_off[b + 1] = f.f_off[b] + (uint32_t)size[b];
    // whole 16-byte pieces: 4-byte entries (32-bit residues) in fours, 16-byte ones in twos
    f.E = w == 4 ? (f.f_off[nf] + 3) & ~3u : (f.f_off[nf] + 1) & ~1u;
    *fp = f;
    return PEVAL_OK;
  }
  return fail(PEVAL_EUNSUPPORTED,
              "point mode: the tail degrees need more than %d factor tables of %u entries per point",
              kMaxFactors, (unsigned)emax);
}

}  // namespace peval

extern "C" int peval_points_factors(uint32_t w, uint32_t ntail, const uint32_t *maxdeg, uint32_t *nf,
                                    uint32_t *E) {
  if ((w != 4 && w != 8) || ntail > (uint32_t)kMaxTail || (ntail && !maxdeg) || !nf || !E)
    return fail(PEVAL_EINVAL, "bad argument");
  for (uint32_t v = 0; v < ntail; ++v)
    if (maxdeg[v] > 65535) return fail(PEVAL_EINVAL, "tail degree above 65535");
  FactorPlan fp;
  PEVAL_TRY(build_factor_plan(w, ntail, maxdeg, &fp));
  *nf = fp.nf;
  *E = fp.E;
  return PEVAL_OK;
}

namespace {

template <class A>
const typename A::M &mod_for(const peval_poly *h);
template <>
const Mod64 &mod_for<W64>(const peval_poly *h) { return h->m64; }
template <>
const Mod32 &mod_for<W32>(const peval_poly *h) { return h->m32; }
template <>
const ModF64 &mod_for<WF64>(const peval_poly *h) { return h->mf; }

template <class A>
using PointsFn = void (*)(PointsArgs<A>);

// Which term fills each thread slot (k, j), [K][NT]: the threads of a group
// keep the group (the segmented walk relies on it) and slot (k, t) of the
// group's t-th thread is filled for k nt + t < m (k-major; the kernel adds
// all K slots, padding ones with coefficient 0), but which of the group's
// terms takes which slot is free.
// The lookups of one k are one LDS gather per factor across the wave, and
// lanes whose entries differ but share a bank serialise.  As measured on
// gfx950, a 4- or 8-byte gather is served per 32 lanes, its banks the 4-byte
// words modulo 32 (4 bytes) or the 8-byte words modulo 32 (8 bytes); a
// 16-byte one per 16 lanes, 16-byte words modulo 16.  With 4-byte entries
// (32-bit residues) every gather has 32 banks per 32 lanes; with 16-byte
// (value, quotient) entries the first factor's 8-byte value has 16 per 32
// lanes, the last factor's whole entry 16 per 16 lanes, its value alone (the
// FP64 product's 8-byte gather) 16 per 32 lanes.  The slots are filled wave by wave, k by k, in lane
// order: each lane takes, among its group's remaining terms with the
// smallest first-factor entries (a few per bank of the last factor), the
// one that adds the fewest conflicts to the gathers of its pass (whatever
// group the other lanes belong to); among those, one whose first-factor
// entry a lane of the pass already reads (a shared entry costs no bank),
// then one from the bank with the most terms left (the rare banks stay
// available for later lanes), then the smallest first-factor entry, so that
// a group moves through the first factor's table in a narrow window.  On
// the 1e6-term, 1024-point workload this leaves about 0.7 conflict cycles
// per wave and k, against 4.5 when each group's terms are dealt sorted by
// their entries.  0xffffffff marks padding.
// (host only) ex: the tail exponents, variable-major ((n - 2) x s); eb: bytes
// per table entry; r0, r1: bytes the kernel gathers per entry of the first
// and of the last factor.
int deal_slots_host(const std::vector<uint64_t> &grp_off, uint64_t s, const uint16_t *ex, uint32_t eb, uint32_t r0,
                    uint32_t r1, uint32_t K, uint64_t NT, const FactorPlan &fp, std::vector<uint32_t> *out) {
  const uint64_t G = grp_off.size() - 1;
  const uint32_t last = fp.nf ? fp.nf - 1 : 0;
  const bool two = fp.nf > 1;                      // a last factor distinct from the first
  // each gather: banks (in its read width), which are also its lanes per
  // pass, and bank words per entry
  const uint32_t nb = r1 == 16 ? 16 : 32, lanes1 = nb, scale1 = eb / r1;
  const uint32_t kBanks0 = r0 == 16 ? 16 : 32, kLanes0 = kBanks0, scale0 = eb / r0;
  constexpr uint32_t kLook = 8;                    // candidates per bank (smallest first-factor entries)
  constexpr uint32_t kNone = 0xffffffffu;
  HostPlan hp = build_host_plan(grp_off, K, kPointsP, true);
  if (hp.NT != NT) return fail(PEVAL_EINVAL, "thread layout mismatch");
  out->assign((size_t)K * NT, kNone);
  // threads of each group
  std::vector<uint64_t> tj0(G), tnt(G);
  std::vector<uint32_t> tg(NT, kNone);
  {
    uint64_t j = 0;
    for (uint64_t g = 0; g < G; ++g) {
      const uint64_t e = grp_off[g + 1];
      tj0[g] = j;
      while (j < NT && hp.thr_cnt[j] && hp.thr_first[j] < e) tg[j++] = (uint32_t)g;
      tnt[g] = j - tj0[g];
      if (!tnt[g]) return fail(PEVAL_EINVAL, "group without threads");
    }
  }
  struct Term {
    uint32_t e0, e1, i;  // first and last factor's entries, term
  };
  // a group's remaining terms: by bank of the last factor's entry, each bank
  // sorted by the first factor's entry
  struct Pool {
    std::vector<Term> t;
    std::vector<uint32_t> base, head;
    std::vector<uint8_t> taken;
  };
  std::map<uint64_t, Pool> pools;
  auto make_pool = [&](uint64_t g) {
    Pool &pl = pools[g];
    const uint64_t b = grp_off[g], e = grp_off[g + 1];
    std::vector<Term> all;
    all.reserve(e - b);
    for (uint64_t i = b; i < e; ++i) {
      uint32_t local[kMaxFactors] = {0, 0, 0, 0};
      for (uint32_t d = 0; d < fp.ndig; ++d) {
        const uint32_t x = ex[(size_t)fp.var[d] * s + i];
        local[fp.fac[d]] += ((x >> fp.shift[d]) & fp.mask[d]) * fp.stride[d];
      }
      all.push_back(Term{fp.f_off[0] + local[0], fp.f_off[last] + local[last], (uint32_t)i});
    }
    auto bank = [&](const Term &x) { return two ? (x.e1 * scale1) % nb : 0u; };
    std::sort(all.begin(), all.end(), [&](const Term &x, const Term &y) {
      const uint32_t bx = bank(x), by = bank(y);
      if (bx != by) return bx < by;
      return x.e0 != y.e0 ? x.e0 < y.e0 : x.e1 < y.e1;
    });
    pl.base.assign(nb + 1, 0);
    for (const Term &x : all) pl.base[bank(x) + 1]++;
    for (uint32_t c = 0; c < nb; ++c) pl.base[c + 1] += pl.base[c];
    pl.head.assign(pl.base.begin(), pl.base.end() - 1);
    pl.taken.assign(all.size(), 0);
    pl.t.swap(all);
  };
  std::vector<uint32_t> owner0(kBanks0);
  std::vector<uint8_t> held0(kBanks0);
  std::vector<std::vector<uint32_t>> ent1(nb);  // distinct last-factor entries per bank in the pass
  for (uint64_t w = 0; w < NT / 64; ++w) {
    for (uint32_t l = 0; l < 64; ++l) {
      const uint32_t g = tg[w * 64 + l];
      if (g != kNone && !pools.count(g)) make_pool(g);
    }
    for (uint32_t k = 0; k < K; ++k) {
      for (uint32_t l = 0; l < 64; ++l) {
        if (l % kLanes0 == 0) std::fill(held0.begin(), held0.end(), 0);
        if (l % lanes1 == 0)
          for (auto &v : ent1) v.clear();
        const uint64_t j = w * 64 + l;
        const uint32_t g = tg[j];
        if (g == kNone) continue;
        const uint64_t t = j - tj0[g];
        if (k * tnt[g] + t >= grp_off[g + 1] - grp_off[g]) continue;  // no slot (k, t)
        Pool &pl = pools[g];
        uint64_t best = ~0ull;
        uint32_t bpos = kNone, bc = 0;
        for (uint32_t c = 0; c < nb; ++c) {
          uint32_t u = pl.head[c];
          while (u < pl.base[c + 1] && pl.taken[u]) ++u;
          pl.head[c] = u;
          for (uint32_t seen = 0; u < pl.base[c + 1] && seen < kLook; ++u) {
            if (pl.taken[u]) continue;
            ++seen;
            const Term &x = pl.t[u];
            const uint32_t b0 = (x.e0 * scale0) % kBanks0;
            uint64_t conf = (held0[b0] && owner0[b0] != x.e0) ? 1 : 0;
            if (two)
              for (uint32_t y : ent1[c]) conf += (y != x.e1);
            const uint64_t shared = (held0[b0] && owner0[b0] == x.e0) ? 0 : 1;
            const uint64_t left = std::min<uint64_t>(pl.base[c + 1] - pl.head[c], 0xffff);
            const uint64_t cost = (conf << 48) | (shared << 40) | ((0xffff - left) << 16) | x.e0;  // e0 < 2^16
            if (cost < best) {
              best = cost;
              bpos = u;
              bc = c;
            }
          }
        }
        if (bpos == kNone) return fail(PEVAL_EINVAL, "slot dealing ran out of terms");
        const Term &x = pl.t[bpos];
        pl.taken[bpos] = 1;
        (*out)[(uint64_t)k * NT + j] = x.i;
        const uint32_t b0 = (x.e0 * scale0) % kBanks0;
        held0[b0] = 1;
        owner0[b0] = x.e0;
        if (std::find(ent1[bc].begin(), ent1[bc].end(), x.e1) == ent1[bc].end()) ent1[bc].push_back(x.e1);
      }
    }
    // groups that end in this wave are dealt completely
    for (auto it = pools.begin(); it != pools.end();) {
      if (tj0[it->first] + tnt[it->first] <= (w + 1) * 64)
        it = pools.erase(it);
      else
        ++it;
    }
  }
  return PEVAL_OK;
}

int deal_slots(peval_poly *h, uint32_t eb, uint32_t r0, uint32_t r1, uint32_t K, uint64_t NT, const FactorPlan &fp,
               std::vector<uint32_t> *out) {
  std::vector<uint16_t> ex((size_t)(h->n - 2) * h->s);
  if (!ex.empty()) HIP_TRY(hipMemcpy(ex.data(), h->d_exps, ex.size() * 2, hipMemcpyDeviceToHost));
  return deal_slots_host(h->grp_off, h->s, ex.data(), eb, r0, r1, K, NT, fp, out);
}

template <class A>
PointsFn<A> points_kernel_for(uint32_t K, uint32_t NF) {
#define PEVAL_PCASE(k, f) \
  if (K == k && NF == f) return points_eval_kernel<A, k, f>;
#define PEVAL_PCASES(k) PEVAL_PCASE(k, 1) PEVAL_PCASE(k, 2) PEVAL_PCASE(k, 3) PEVAL_PCASE(k, 4)
  PEVAL_PCASES(1)
  PEVAL_PCASES(2)
  PEVAL_PCASES(4)
  PEVAL_PCASES(8)
  if constexpr (!std::is_same<A, WF64>::value) {  // FP64: a thread sums at most 8 doubles exactly
    PEVAL_PCASES(16)
  }
#undef PEVAL_PCASES
#undef PEVAL_PCASE
  return nullptr;
}

constexpr size_t kPointsPartialBudget = (size_t)2 << 30;  // partial sums per launch
constexpr size_t kPointsTablesBudget = (size_t)256 << 20;  // factor tables per launch

// A: integer policy of the tables, slot arrays, partial sums and output;
// E: policy of the evaluation kernel (A itself, or the FP64 product on
// 64-bit residues, whose tables and coefficients are written as doubles).
template <class A, class E = A>
int run_points_impl(peval_poly *h, const uint64_t *points, uint32_t T, void *dev_out, hipStream_t st,
                    uint32_t K, uint32_t C) {
  using T_ = typename A::T;
  using TE = typename E::T;
  constexpr bool fp64 = std::is_same<E, WF64>::value;
  static_assert(sizeof(TE) == sizeof(T_), "the FP64 product runs on 64-bit residues");
  const auto &m = mod_for<A>(h);
  const size_t w = sizeof(T_);
  const uint32_t ntail = h->n - 2;
  const FactorPlan &fp = h->fplan;
  Plan *pl = nullptr;
  PEVAL_TRY(get_plan(h, K, kPointsP, &pl, true));
  auto eval = points_kernel_for<E>(K, fp.nf);
  if (!eval) return fail(PEVAL_EINVAL, "no point kernel for K=%u with %u factors", K, fp.nf);

  const uint32_t prep_key = K | (fp64 ? 0x100u : 0u);  // slot arrays differ by product
  auto it = h->pprep.find(prep_key);
  if (it == h->pprep.end()) {  // per-slot coefficients, quotients and entry indices
    std::vector<uint32_t> slot_term;
    // gathers: 32-bit residues read 4-byte entries; 64-bit ones the 8-byte
    // value of the first factor and the whole 16-byte entry of the others
    // (the FP64 product: their 8-byte value)
    const uint32_t eb = points_entry_bytes<T_>(), r0 = (uint32_t)w, r1 = (w == 4 || fp64) ? (uint32_t)w : eb;
    PEVAL_TRY(deal_slots(h, eb, r0, r1, K, pl->NT, fp, &slot_term));
    PointsPrep pp;
    const uint64_t total = (uint64_t)K * pl->NT;
    const bool ok = hipMalloc(&pp.pa, total * w) == hipSuccess && hipMalloc(&pp.paq, total * w) == hipSuccess &&
                    hipMalloc((void **)&pp.pidx, total * sizeof(uint64_t)) == hipSuccess &&
                    hipMalloc((void **)&pp.slot_term, total * sizeof(uint32_t)) == hipSuccess &&
                    hipMemcpy(pp.slot_term, slot_term.data(), total * sizeof(uint32_t), hipMemcpyHostToDevice) ==
                        hipSuccess;
    if (!ok) {  // nothing half-built stays behind
      (void)hipFree(pp.pa);
      (void)hipFree(pp.paq);
      (void)hipFree(pp.pidx);
      (void)hipFree(pp.slot_term);
      (void)hipGetLastError();
      return fail(PEVAL_ENOMEM, "point-mode slot arrays of %llu slots", (unsigned long long)total);
    }
    it = h->pprep.emplace(prep_key, pp).first;
    ProfScope ps(st, 1);
    points_prep_kernel<A><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(
        (const T_ *)h->d_coeff, h->d_exps, pp.slot_term, h->s, pl->NT, K, fp, (T_ *)pp.pa, (T_ *)pp.paq, pp.pidx,
        m, fp64 ? 1u : 0u);
    HIP_TRY(hipGetLastError());
  }
  const PointsPrep &pp = it->second;

  uint64_t tc = std::max<uint64_t>(1, kPointsPartialBudget / std::max<uint64_t>(1, pl->nslots * w));
  const size_t eb = points_entry_bytes<T_>();
  tc = std::min<uint64_t>(tc, std::max<uint64_t>(1, kPointsTablesBudget / ((uint64_t)fp.E * eb)));
  tc = std::min<uint64_t>(tc, (uint64_t)C * kCombineTile * 32768);
  tc = std::min<uint64_t>(tc, T);
  if (tc < T && tc > C) tc = tc / C * C;
  PEVAL_TRY(ensure(h->ptab, (size_t)tc * fp.E * eb, h));
  PEVAL_TRY(ensure(h->partial, (size_t)((tc + C - 1) / C) * C * pl->nslots * w, h));
  const size_t shmem = (kEvalBlock / 64) * sizeof(Stage<E, kPointsP>) + (size_t)fp.E * eb;

  for (uint64_t done = 0; done < T; done += tc) {
    const uint32_t Tc = (uint32_t)std::min<uint64_t>(tc, T - done);
    const uint32_t Cc = std::min<uint32_t>(C, Tc);
    const uint32_t Lmax = (Tc + Cc - 1) / Cc;
    {
      const uint64_t total = (uint64_t)Tc * fp.E;
      ProfScope ps(st, 0);
      points_table_kernel<A><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(
          points + done * ntail, ntail, Tc, fp, (T_ *)h->ptab.ptr, m, fp64 ? 1u : 0u);
      HIP_TRY(hipGetLastError());
    }
    {
      PointsArgs<E> a;
      a.pa = (const TE *)pp.pa;
      a.paq = (const TE *)pp.paq;
      a.pidx = pp.pidx;
      a.tables = (const TE *)h->ptab.ptr;
      a.endmask = pl->d_endmask;
      a.slot_base = pl->d_slot_base;
      a.partial = (typename E::PT *)h->partial.ptr;
      a.NT = pl->NT;
      a.NW = pl->NW;
      a.C = Cc;
      a.T = Tc;
      a.Lmax = Lmax;
      a.E = fp.E;
      a.m = mod_for<E>(h);
      dim3 grid((unsigned)((pl->NW + 3) / 4), Cc);
      ProfScope ps(st, 2);
      eval<<<grid, kEvalBlock, shmem, st>>>(a);
      HIP_TRY(hipGetLastError());
    }
    {
      CombineArgs<A> ca;
      ca.partial = (const T_ *)h->partial.ptr;
      ca.slot_off = pl->d_slot_off;
      ca.out = (T_ *)dev_out + done * h->G;
      ca.G = h->G;
      ca.C = Cc;
      ca.T = Tc;
      ca.Lmax = Lmax;
      ca.m = m;
      dim3 grid((unsigned)((h->G + kCombineTile - 1) / kCombineTile), Cc,
                (unsigned)((Lmax + kCombineTile - 1) / kCombineTile));
      ProfScope ps(st, 3);
      combine_kernel<A><<<grid, kCombineBlock, 0, st>>>(ca);
      HIP_TRY(hipGetLastError());
    }
  }
  return PEVAL_OK;
}

// Layout for the point mode: K as chosen for the power mode (explicit
// setting, else the padding heuristic), P fixed, chains for ~8192 waves.
Tuning points_tuning(peval_poly *h, uint32_t T) {
  Tuning t = heuristic_tuning(h, T);
  if (h->tune_K) t.K = h->tune_K;
  if (h->arith == 1) t.K = std::min<uint32_t>(t.K, 8);  // FP64 product: exact sums of at most 8 doubles
  t.K = std::min<uint32_t>(t.K, 16);                    // the point kernels hold at most 16 terms
  t.P = kPointsP;
  const uint64_t nw = (padded_threads(h, t.K) + 63) / 64;
  t.C = h->tune_C ? h->tune_C : chains_for_waves(nw, 8192, T);
  t.C = std::max<uint32_t>(1, std::min<uint32_t>(t.C, T));
  return t;
}

int points_locked(peval_poly *h, const uint64_t *points_dev, uint32_t T, void *dev_out, hipStream_t st) {
  HIP_TRY(hipSetDevice(h->device));
  if (h->fplan_rc == 1) {
    uint32_t maxdeg[kMaxTail] = {0};
    for (uint32_t v = 0; v + 2 < h->n; ++v) maxdeg[v] = h->max_exp[v + 2];
    h->fplan_rc = build_factor_plan(h->w, h->n - 2, maxdeg, &h->fplan);
  }
  if (h->fplan_rc != PEVAL_OK)
    return fail(PEVAL_EUNSUPPORTED, "point mode: the tail degrees need too many factor tables");
  if (h->have_done) HIP_TRY(hipStreamWaitEvent(st, h->done, 0));
  const Tuning tu = points_tuning(h, T);
  int rc = (h->w == 4)       ? run_points_impl<W32>(h, points_dev, T, dev_out, st, tu.K, tu.C)
           : (h->arith == 1) ? run_points_impl<W64, WF64>(h, points_dev, T, dev_out, st, tu.K, tu.C)
                             : run_points_impl<W64>(h, points_dev, T, dev_out, st, tu.K, tu.C);
  if (rc != PEVAL_OK) return rc;
  HIP_TRY(hipEventRecord(h->done, st));
  h->have_done = true;
  return PEVAL_OK;
}

int check_points_args(peval_poly *h, const uint64_t *points, uint32_t T) {
  if (!h) return fail(PEVAL_EINVAL, "null handle");
  if (h->n > 2 && T && !points) return fail(PEVAL_EINVAL, "null points");
  if ((uint64_t)T * h->G > (1ull << 40)) return fail(PEVAL_EUNSUPPORTED, "T*G too large");
  return PEVAL_OK;
}

}  // namespace

extern "C" int peval_test_deal_points(uint32_t w, uint32_t ntail, uint64_t s, const uint16_t *tail_exps, uint64_t G,
                                      const uint64_t *group_sizes, uint32_t K, uint32_t *slot_term,
                                      uint64_t slot_count) {
  if ((w != 4 && w != 8) || ntail > (uint32_t)kMaxTail || (s && ntail && !tail_exps) || (G && !group_sizes) ||
      !slot_term || !(K == 1 || K == 2 || K == 4 || K == 8 || K == 16))
    return fail(PEVAL_EINVAL, "bad argument");
  std::vector<uint64_t> off(G + 1, 0);
  for (uint64_t g = 0; g < G; ++g) {
    if (!group_sizes[g]) return fail(PEVAL_EINVAL, "empty group");
    off[g + 1] = off[g] + group_sizes[g];
  }
  if (off[G] != s) return fail(PEVAL_EINVAL, "group sizes do not add up to s");
  uint32_t maxdeg[kMaxTail] = {0};
  for (uint32_t v = 0; v < ntail; ++v)
    for (uint64_t i = 0; i < s; ++i) maxdeg[v] = std::max<uint32_t>(maxdeg[v], tail_exps[(size_t)v * s + i]);
  FactorPlan fp;
  PEVAL_TRY(build_factor_plan(w, ntail, maxdeg, &fp));
  const uint64_t NT = build_host_plan(off, K, kPointsP, true).NT;
  if (slot_count != (uint64_t)K * NT) return fail(PEVAL_EINVAL, "slot_count must be K x NT = %llu", (unsigned long long)(K * NT));
  std::vector<uint32_t> out;
  PEVAL_TRY(deal_slots_host(off, s, tail_exps, w == 4 ? 4 : 16, w, w == 4 ? 4 : 16, K, NT, fp, &out));
  std::copy(out.begin(), out.end(), slot_term);
  return PEVAL_OK;
}

extern "C" int peval_run_points_async(peval_poly *h, const uint64_t *points_dev, uint32_t T, void *dev_out,
                                      void *stream) {
  PEVAL_TRY(check_points_args(h, points_dev, T));
  if (T == 0 || h->G == 0) return PEVAL_OK;
  if (!dev_out) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(h->mu);
  return points_locked(h, points_dev, T, dev_out, (hipStream_t)stream);
}

extern "C" int peval_points_tuning(peval_poly *h, uint32_t T, uint32_t *K, uint32_t *P, uint32_t *C) {
  if (!h || !K || !P || !C) return fail(PEVAL_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(h->mu);
  const Tuning t = points_tuning(h, T);
  *K = t.K;
  *P = t.P;
  *C = t.C;
  return PEVAL_OK;
}

extern "C" int peval_run_points(peval_poly *h, const uint64_t *points_host, uint32_t T, void *out) {
  PEVAL_TRY(check_points_args(h, points_host, T));
  if (T == 0 || h->G == 0) return PEVAL_OK;
  if (!out) return fail(PEVAL_EINVAL, "null output");
  std::lock_guard<std::mutex> lk(h->mu);
  const size_t pbytes = (size_t)T * std::max<uint32_t>(h->n - 2, 1) * sizeof(uint64_t);
  const size_t obytes = (size_t)T * h->G * h->w;
  PEVAL_TRY(ensure(h->ptsbuf, pbytes, h));
  PEVAL_TRY(ensure(h->outbuf, obytes, h));
  if (h->n > 2)
    HIP_TRY(hipMemcpyAsync(h->ptsbuf.ptr, points_host, pbytes, hipMemcpyHostToDevice, h->stream));
  PEVAL_TRY(points_locked(h, (const uint64_t *)h->ptsbuf.ptr, T, h->outbuf.ptr, h->stream));
  HIP_TRY(hipMemcpyAsync(out, h->outbuf.ptr, obytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PEVAL_OK;
}
