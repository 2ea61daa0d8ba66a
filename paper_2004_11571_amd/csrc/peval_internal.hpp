// Internal state of a resident polynomial and its evaluation plans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "modarith.hpp"
#include "points_kernels.hpp"

namespace peval {

// Thread layout of one (K, P) choice (see kernels.hpp).
struct Plan {
  uint32_t K = 0, P = 0;
  uint64_t NT = 0;      // threads, multiple of 64
  uint64_t NW = 0;      // waves
  uint64_t nslots = 0;  // segment slots (partial coefficients per evaluation)
  uint32_t *d_thr_first = nullptr;
  uint8_t *d_thr_cnt = nullptr;
  uint64_t *d_endmask = nullptr;
  uint32_t *d_slot_base = nullptr;
  uint32_t *d_slot_off = nullptr;  // G + 1
  uint64_t device_bytes = 0;
};

// Device scratch that grows on demand and is reused across runs.
struct Scratch {
  void *ptr = nullptr;
  size_t bytes = 0;
};

// A caller-provided region that a run carves all of its scratch from (power
// tables, chain starts, Gamma and its quotients, partial sums) instead of
// the handle's grow-on-demand buffers; nothing is allocated.
struct FixedScratch {
  unsigned char *base = nullptr;
  size_t bytes = 0;
};

// Host-side layout computation (pure C++; also used by the CPU tests through
// peval_debug_plan).
struct HostPlan {
  uint64_t NT = 0, NW = 0, nslots = 0;
  std::vector<uint32_t> thr_first;
  std::vector<uint8_t> thr_cnt;
  std::vector<uint64_t> endmask;
  std::vector<uint32_t> slot_base;
  std::vector<uint32_t> slot_off;
};
HostPlan build_host_plan(const std::vector<uint64_t> &grp_off, uint32_t K, uint32_t P, bool subtile_ends);

struct Tuning {
  uint32_t K, P, C;
  uint32_t L = 0;  // > 0: the single-launch path with L evaluations per block (K, P, C unused)
};

// Per-thread-slot inputs of the point mode for one thread layout (K).
struct PointsPrep {
  void *pa = nullptr, *paq = nullptr;
  uint64_t *pidx = nullptr;
  uint32_t *slot_term = nullptr;
};

// HIP-event timing of one kernel launch (active while profiling is enabled).
// kind: 0 tables, 1 monomials / point prologue, 2 evaluation, 3 combine.
struct ProfScope {
  hipStream_t st;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(hipStream_t s, int k);
  ~ProfScope();
};
// Timing is off for the calling thread while a ProfOff is alive (the
// allocation-free entry point creates no events).
struct ProfOff {
  ProfOff();
  ~ProfOff();
};

// Factor tables of the point mode from the per-variable degree bounds of the
// tail (host only).  Returns PEVAL_OK or PEVAL_EUNSUPPORTED.
int build_factor_plan(uint32_t w, uint32_t ntail, const uint32_t *maxdeg, FactorPlan *fp);

}  // namespace peval

struct peval_poly {
  uint64_t p = 0;
  uint32_t n = 0;
  uint64_t s = 0;
  uint64_t G = 0;
  uint32_t w = 8;  // bytes per residue
  peval::Mod64 m64{};
  peval::Mod32 m32{};
  peval::ModF64 mf{};
  peval::ModPM64 mpm64{};
  peval::ModPM32 mpm32{};
  uint32_t arith = 0;  // 0: Shoup products; 1: FP64 product (Alg. 2), 2^31 <= p < 2^50; 2: pseudo-Mersenne
  bool arith_auto = true;  // product chosen automatically (not set explicitly)
  int device = 0;

  std::vector<uint32_t> gd, ge;        // output columns
  std::vector<uint64_t> grp_off;       // CSR of groups over the sorted terms (G + 1)
  uint64_t max_group = 0;              // terms of the largest group
  uint32_t max_exp[32] = {0};
  peval::TableOffsets tab{};           // power-table offsets per tail variable
  uint32_t tab_total = 0;

  void *d_coeff = nullptr;             // s residues (w bytes)
  uint16_t *d_exps = nullptr;          // (n - 2) * s tail exponents
  uint64_t resident_bytes = 0;

  std::map<uint32_t, peval::Plan> plans;  // key (sub-tile ends) << 16 | K << 8 | P
  peval::Scratch tabval, tabquot, lam, gam, gamq, partial, outbuf;

  uint32_t tune_K = 0, tune_P = 0, tune_C = 0;  // 0 = automatic

  // point mode (built on first use)
  peval::FactorPlan fplan{};
  int fplan_rc = 1;                          // 1: not built yet
  std::map<uint32_t, peval::PointsPrep> pprep;  // key K
  peval::Scratch ptab, ptsbuf;

  // interpolation (built on first use)
  std::vector<uint32_t> order;         // sorted position -> caller's term index
  // (d_grp_off32 is uploaded at create for polynomials small enough for the
  // single-launch path, which reads it too)
  uint32_t *d_order = nullptr, *d_grp_off32 = nullptr, *d_gorder = nullptr;
  bool interp_ready = false;           // every interpolation array below is in place
  uint32_t *d_task_group = nullptr, *d_task_first = nullptr;
  uint64_t ntasks = 0;
  uint32_t interp_H = 1;                       // sub-products per group for Q
  uint32_t *d_mt[3][3] = {};                   // merge tasks per level: group, pair, first
  uint64_t mt_n[3] = {0, 0, 0};
  peval::Scratch iscr;

  hipStream_t stream = nullptr;  // for peval_run
  hipEvent_t done = nullptr;     // end of the last enqueued call
  bool have_done = false;
  std::mutex mu;
};

namespace peval {

// Per-modulus constants of the integer products (host, exact 128-bit
// arithmetic): p^{-1} mod 2^w, 2^w mod p and the Shoup quotients.
Mod64 make_mod64(uint64_t p);
Mod32 make_mod32(uint32_t p);

bool valid_K(uint32_t K);
bool valid_P(uint32_t P);
uint64_t padded_threads(const peval_poly *h, uint32_t K);
uint32_t chains_for_waves(uint64_t nw, uint64_t target_waves, uint32_t T);
Tuning heuristic_tuning(const peval_poly *h, uint32_t T);
Tuning choose_tuning(const peval_poly *h, uint32_t T);
// Evaluations per block of the single-launch path for T evaluations, 0 if
// the run does not fit it.
uint32_t single_launch_L(const peval_poly *h, uint32_t T);
bool tune_cache_lookup(const peval_poly *h, uint32_t T, Tuning *out);

int ensure(Scratch &sc, size_t bytes, peval_poly *h);
// subtile_ends: every P-lane sub-tile also ends a segment (layout of the walk
// that does not merge sub-tiles, used by the point mode)
int get_plan(peval_poly *h, uint32_t K, uint32_t P, Plan **out, bool subtile_ends = false);
// The existing layout of (K, P), or null (never builds one).
Plan *find_plan(peval_poly *h, uint32_t K, uint32_t P, bool subtile_ends = false);
int check_run_args(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T, BetaArg *ba);
// fixed: carve the run's scratch from this region (no allocation; the chains
// C of tu are lowered and T is split into chunks as needed to fit), else the
// handle's own buffers, grown on demand.
int run_locked(peval_poly *h, const BetaArg &ba, uint64_t t0, uint32_t T, void *dev_out, hipStream_t st,
               const Tuning &tu, const FixedScratch *fixed = nullptr);

}  // namespace peval
