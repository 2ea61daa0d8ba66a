/*
 * peval — partial modular evaluation of sparse multivariate polynomials on
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (paper, Section 2.1 and Section 2.3, Eq. (1)).  For a prime p, a
 * polynomial f = sum_i a_i x1^{d_i} x2^{e_i} M_i(x3..xn) over F_p and a base
 * point beta = (beta_3..beta_n), compute the T bivariate images
 *
 *     b_t(x1, x2) = f(x1, x2, beta_3^t, ..., beta_n^t)      t = t0 .. t0+T-1
 *
 * by the matrix method (Section 2.3): m_i = M_i(beta) once, then
 * a_i m_i^t by one modular product per term and per evaluation, and the
 * coefficient of x1^d x2^e in b_t as the modular sum over the terms whose
 * (x1, x2) exponents equal (d, e) ("coefficient reduction").
 *
 * Output layout (dense).  The columns are the G distinct (d, e) pairs of the
 * input in descending lexicographic order (x1 before x2), as returned by
 * peval_groups.  Row r holds b_{t0+r}; entry (r, g) is at index r*G + g.
 * Every entry is the canonical residue in [0, p), zeros included.  Elements
 * are uint32 when p < 2^31 and uint64 otherwise (peval_info.elem_bytes).
 *
 * Conventions.  Coefficients and base-point entries are reduced modulo p on
 * entry.  0^0 = 1.  Exponent rows may repeat (their terms add) and
 * coefficients may be zero (their group is still listed).
 *
 * Errors.  Every call returns PEVAL_OK (0) or a negative code; nothing is
 * thrown across this interface.  Argument checks happen before any device
 * call, so PEVAL_EINVAL / PEVAL_EUNSUPPORTED never leave device state behind.
 * A failing HIP call maps to PEVAL_EDEVICE, an allocation failure to
 * PEVAL_ENOMEM.  peval_strerror() names a code; peval_last_error() gives a
 * message for the calling thread's most recent failure.
 *
 * Threads.  Distinct handles are independent.  Calls on one handle are
 * serialised by the handle; device work of consecutive calls on one handle
 * is ordered even across streams (each call waits for the previous one).
 */
#ifndef PEVAL_H
#define PEVAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PEVAL_OK = 0,
    PEVAL_EINVAL = -1,        /* bad argument (null pointer, size, range) */
    PEVAL_ENOMEM = -2,        /* host or device allocation failed */
    PEVAL_EDEVICE = -3,       /* HIP runtime or kernel error */
    PEVAL_EUNSUPPORTED = -4,  /* valid input outside what the library supports */
    PEVAL_EBUSY = -5,         /* resource temporarily unavailable (server) */
    PEVAL_ETIMEOUT = -6,      /* wait ended before completion */
    PEVAL_ESINGULAR = -7      /* interpolation: a group's system has no unique solution */
};

typedef struct peval_poly peval_poly;

typedef struct peval_info_t {
    uint64_t p;               /* modulus */
    uint32_t n;               /* number of variables */
    uint32_t elem_bytes;      /* 4 if p < 2^31, else 8 */
    uint64_t s;               /* number of terms */
    uint64_t G;               /* number of distinct (x1, x2) exponent pairs = output columns */
    uint64_t device_bytes;    /* device memory held by the handle now */
    uint32_t max_exp[32];     /* largest exponent of x_{k+1} over all terms, k < n */
} peval_info_t;

/*
 * Ingest a polynomial (Section 2.3, Eq. (1)) and keep it resident on the
 * current HIP device.
 *
 * p          modulus, odd, 3 <= p < 2^63 (EINVAL otherwise).  Primality is
 *            not required by the arithmetic used here.
 * n          number of variables, 2 <= n <= 32.
 * s          number of terms (0 allowed: every image is empty).
 * exponents  host, s*n uint32, row-major: exponents[i*n + k] is the
 *            exponent of x_{k+1} in term i.  Exponents of x3..xn must be
 *            <= 65535 (EUNSUPPORTED otherwise); x1, x2 exponents are free.
 * coeffs     host, s uint64, any value (reduced modulo p).
 * out        receives the handle.
 *
 * The inputs are copied; the caller may free them on return.  The handle
 * owns its device memory until peval_destroy.
 */
int peval_create(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exponents,
                 const uint64_t *coeffs, peval_poly **out);

/* Sizes and modulus of a handle (host struct filled by the call). */
int peval_info(const peval_poly *h, peval_info_t *info);

/*
 * The G output columns: d[g], e[g] (host arrays of G uint32 each) are the
 * x1 and x2 exponents of column g, in descending lexicographic order.
 */
int peval_groups(const peval_poly *h, uint32_t *d, uint32_t *e);

/*
 * Evaluate b_t for t = 1..T (Section 2.1: t starts at 1, since beta^0 may be
 * an unlucky point) and copy the T*G images to host memory.
 *
 * beta  host, n-2 uint64 (beta_3..beta_n), reduced modulo p; zero allowed.
 * T     number of evaluations; 0 is a no-op.
 * out   host buffer of T*G elements of elem_bytes each.
 * Blocks until the result is in out.
 */
int peval_run(peval_poly *h, const uint64_t *beta, uint32_t T, void *out);

/*
 * Evaluate b_t for t = t0..t0+T-1 into device memory, asynchronously on
 * `stream` (a hipStream_t; NULL means the null stream).
 *
 * t0       first evaluation index, t0 >= 1.
 * dev_out  device buffer of T*G elements of elem_bytes (caller-owned, may
 *          be a torch allocation); must stay valid until the stream has
 *          passed this call.
 * Returns once the work is enqueued.  Resuming or splitting a long run:
 * rows t0.. of a run equal a run started at t0.
 *
 * Small runs (s <= 8192 terms for p < 2^31, s <= 4096 otherwise, s*T <= 2^20,
 * no group above 256 terms, power tables and one evaluation's term values
 * within 64 KiB) take a
 * single-launch path: one kernel builds the tables, the chain starts
 * (Alg. 7) and every image, with one chain of consecutive evaluations per
 * block, instead of the four kernels of the general path (Section 2.3).  It
 * is used unless a tuning is set (peval_set_tuning), the autotuner chose a
 * multi-kernel tuning for the shape, or the product was set explicitly
 * (peval_set_arith with a mode other than AUTO).  Results are identical.
 */
int peval_run_async(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T,
                    void *dev_out, void *stream);

/*
 * peval_run_async without any device allocation, for callers that cannot
 * allocate device memory while they run (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc after setup).
 *
 * Same arguments, results and ordering as peval_run_async.  The run's
 * scratch (power tables, chain starts, Gamma and its quotients, partial
 * sums) is carved from one fixed region of 128 MiB per GPU, held by the
 * library from its first use on that GPU until the process ends; fewer
 * chains, or more launches over shorter stretches of T, are used when the
 * tuning's scratch would not fit (results are the same).  It calls no
 * hipMalloc, hipFree or other allocating routine, and records no timing
 * events (peval_prof_enable does not see its kernels).
 *
 * Limits and errors:
 *   - PEVAL_EUNSUPPORTED when even one chain does not fit the region
 *     (about 3 s residues of elem_bytes plus the tables and one row of
 *     partial sums: roughly s <= 5e6 terms for p >= 2^31, 1e7 below);
 *   - PEVAL_EUNSUPPORTED when the handle has no thread layout yet for the
 *     run's tuning (K, P): a layout is device memory of the handle, made
 *     once by the first peval_run or peval_run_async with that tuning (the
 *     single-launch path of small runs needs none).
 * Sharing: every call on one GPU uses that GPU's one region.  Calls on the
 * same handle are ordered on the device as with peval_run_async; calls on
 * different handles whose device work overlaps (other streams, no ordering
 * by the caller) race on the region and give wrong results.  Nothing in the
 * region needs clearing between calls (every entry is written before it is
 * read within a call).
 */
int peval_run_async_noalloc(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T,
                            void *dev_out, void *stream);

/*
 * Images at T arbitrary points instead of the powers of one base point
 * (paper, Section 2.1: the random points of Zippel's method; the cost of
 * evaluating at unrelated points is O(nT(d+s)), Section 2.3):
 *
 *   row t of out = f(x1, x2, points[t][0], ..., points[t][n-3]),  0 <= t < T,
 *
 * in the same dense T x G layout and column order as peval_run.
 *
 * points  T rows of n-2 uint64 values (x3..xn), row-major; any values,
 *         reduced mod p on the device.  Host memory for peval_run_points,
 *         device memory for peval_run_points_async (valid until the stream
 *         has passed the call).  May be NULL when n == 2.
 * Each term's monomial is formed from per-point tables of products of its
 * tail variables' powers; a polynomial whose tail degrees need more than
 * four such tables of 32 KiB per point gives PEVAL_EUNSUPPORTED.
 */
int peval_run_points(peval_poly *h, const uint64_t *points, uint32_t T, void *out);
int peval_run_points_async(peval_poly *h, const uint64_t *points, uint32_t T, void *dev_out,
                           void *stream);

/* The tiles the next point-mode run with T points would use: terms per
 * thread K (at most 16; 8 under the FP64 product), points per pass P and
 * chains C.  Outputs must not be NULL. */
int peval_points_tuning(peval_poly *h, uint32_t T, uint32_t *K, uint32_t *P, uint32_t *C);

/*
 * Host-only planner of the point mode's tables (for tests): residue width
 * w (4 or 8), ntail = n-2 tail degree bounds -> number of factor tables nf
 * and table entries per point E.  PEVAL_EUNSUPPORTED if no plan fits.
 */
int peval_points_factors(uint32_t w, uint32_t ntail, const uint32_t *maxdeg, uint32_t *nf, uint32_t *E);

/*
 * Coefficients back from the images: the sparse interpolation step that
 * follows the evaluations in Zippel's method (paper, Section 2.1).  Because
 * the images are taken at the powers beta^t, each (d, e) group's linear
 * system is a transposed Vandermonde system, solved here in O(m^2)
 * operations for a group of m terms.
 *
 * h       a handle whose exponent rows are the support of the polynomial to
 *         recover (its coefficients are not used; zeros are fine).  The
 *         rows must be distinct and p prime.
 * beta    the base point the images were taken at (n-2 values).
 * images  b_1..b_T in the dense layout of peval_run (T rows of G residues
 *         of elem_bytes); T must be at least the largest group's term
 *         count, and only that many rows are read.  Host memory for
 *         peval_interpolate, device memory for peval_interpolate_async.
 * coeffs  s uint64 coefficients, canonical, in the order of the rows given
 *         to peval_create (host / device).
 * Groups of more than 8191 terms give PEVAL_EUNSUPPORTED.  A group whose
 * system is singular (two of its terms with equal monomial values at beta,
 * a zero monomial value, or p not prime) gives PEVAL_ESINGULAR from
 * peval_interpolate; peval_interpolate_async writes 0 or 1 to *dev_status
 * (a device int32) instead, and 0 to the affected coefficients.
 */
int peval_interpolate(peval_poly *h, const uint64_t *beta, uint32_t T, const void *images, uint64_t *coeffs);
int peval_interpolate_async(peval_poly *h, const uint64_t *beta, uint32_t T, const void *dev_images,
                            uint64_t *dev_coeffs, int32_t *dev_status, void *stream);

/* Release the handle and its device memory (waits for its pending work).
 * NULL is accepted. */
int peval_destroy(peval_poly *h);

/*
 * Tuning knobs of the evaluation kernel for one handle (0 = automatic):
 *   K      terms held per thread (1, 2, 4, 8, 16; 32 for p < 2^31 under the
 *          integer product, with P <= 16; EINVAL otherwise)
 *   P      evaluations per pass before each coefficient reduction (8, 16, 32;
 *          the role of the paper's dependent evaluations T_d, Section 4.2)
 *   C      independent evaluation chains (>= 1; chain c does t = t0+c,
 *          t0+c+C, ...: the independent evaluations T_i of Section 4.2 and
 *          Alg. 7, with Lambda_c = a_i m_i^{t0+c} and the common multiplier
 *          m_i^C as in Fig. 3)
 * The results never depend on these; only speed does.
 */
int peval_set_tuning(peval_poly *h, uint32_t K, uint32_t P, uint32_t C);

/*
 * Modular product of the evaluation kernel.  PEVAL_ARITH_INT: Shoup's
 * precomputed-quotient product on 32-bit limbs, for every p.
 * PEVAL_ARITH_FP64: the paper's FP64-FMA product (Alg. 2) on signed running
 * values with its quotient estimate rounded to nearest (no correction step)
 * and sums folded the same way, allowed for 2^31 <= p < 2^50; terms per
 * thread are capped at 8 (exact double sums).  PEVAL_ARITH_AUTO (the
 * default at create): FP64 for 2^31 <= p < 2^50, where it is faster on
 * gfx950, integer otherwise.  The choice applies to the power mode, the
 * point mode, interpolation's b_l sums and Horner steps, and batches
 * created afterwards (peval_batch_create, the server); the single-launch
 * path of small runs and interpolation's product of (z - v) factors use the
 * integer product.
 * Results are identical; only speed differs.
 */
#define PEVAL_ARITH_AUTO 0u
#define PEVAL_ARITH_INT 1u
#define PEVAL_ARITH_FP64 2u
#define PEVAL_ARITH_PMERSENNE 3u
int peval_set_arith(peval_poly *h, uint32_t mode);

/* PEVAL_ARITH_PMERSENNE: for p = 2^63 - c (c < 2^20) or p = 2^31 - c
 * (c < 2^12), the full product folded twice with 2^k = c (mod p), with no
 * precomputed quotient (not in the paper; measured slower than Shoup's
 * product on gfx950, so never chosen by AUTO).  Evaluations per pass are
 * fixed at 16 with it. */

/* The product the power-mode evaluation kernel of this handle uses now:
 * *mode = PEVAL_ARITH_INT, PEVAL_ARITH_FP64 or PEVAL_ARITH_PMERSENNE
 * (AUTO resolved). */
int peval_get_arith(const peval_poly *h, uint32_t *mode);

/* The tuning the next run with T evaluations would use; K = P = C = 0 when
 * it takes the single-launch path (see peval_run_async). */
int peval_get_tuning(peval_poly *h, uint32_t T, uint32_t *K, uint32_t *P, uint32_t *C);

/*
 * Autotuner (the analogue of the paper's (T_i, T_d, M) sweep, Section 4.4).
 * Times candidate (K, P, C) on the device for this polynomial and T
 * evaluations at base point beta, and records the fastest for the handle's
 * shape class (residue width, term count, mean group size and T, each on a
 * half-octave grid) in a process-wide cache that every later run of a
 * matching shape uses (explicit peval_set_tuning values take precedence).
 * exhaustive = 0: the heuristic's own choice, then a coordinate search
 * over K, then P, then C (chains for 2048 .. 65536 waves; about fifteen
 * timed runs); 1: the full grid.  Where the run fits the single-launch path
 * (with the product on AUTO) that path is timed too.  A candidate replaces
 * the one chosen so far only when it is more than 1.5% faster (the best of
 * two timed runs each), so near-ties keep the earlier one.  Outputs (any may be
 * NULL): the chosen K, P, C (all 0 if the single-launch path won) and its
 * time in ms.  Blocks until the timing runs are done.
 */
int peval_autotune(peval_poly *h, const uint64_t *beta, uint32_t T, uint32_t exhaustive,
                   uint32_t *K, uint32_t *P, uint32_t *C, float *ms);

/* Tuning cache: forget everything, or save to / merge from a text file
 * (one line per shape class: width s_class group_class T_class K P C ms;
 * K P C = 0 0 0 records the single-launch path). */
int peval_tune_clear(void);
int peval_tune_save(const char *path);
int peval_tune_load(const char *path);

/*
 * Batched evaluation (many polynomials, uneven sizes, mixed moduli): the
 * images of Section 2.1 / Eq. (1) by the matrix method of Section 2.3, for
 * every member, in one pass.
 *
 * peval_batch_create plans one pass over `count` resident polynomials,
 * polys[j] evaluated Ts[j] times: it fixes every member's thread layout
 * (K from the tuning cache or the heuristic) and its
 * chains so that the work items (one wave of one chain of one polynomial)
 * have similar costs, allocates all device scratch, and captures the pass
 * (power tables, monomials, persistent evaluation kernels fed by work
 * queues in decreasing item cost, one for each kind of member: 64-bit
 * residues with the integer product and K = 16 (16 evaluations per pass by
 * default), the same with K <= 8 (8 per pass), 64-bit residues with the
 * FP64 product (members whose arithmetic resolves to it when the batch is
 * created), 32-bit residues with K = 32, and with K <= 16; combine) into a
 * hipGraph unless flags has PEVAL_BATCH_NO_GRAPH.  Each kind's kernels run
 * on a stream of their own inside the pass, the kinds side by side.  The
 * handles must outlive the batch; a later peval_set_arith on a member does
 * not change the batch.
 *
 * peval_batch_run evaluates polys[j] at betas[j] (n_j - 2 values each) for
 * t = t0s[j] .. t0s[j]+Ts[j]-1 (t0s may be NULL: all 1) into dev_outs[j]
 * (device, Ts[j] x G_j residues of that polynomial's width), on `stream`.
 * Results equal those of peval_run_async member by member.  Consecutive
 * runs of one batch are ordered on the device (also across streams); the
 * call returns after enqueueing and blocks only when the run table it stages
 * (four staging buffers in rotation) still awaits its upload.
 *
 * peval_batch_info fills info[5]: members, work items, persistent blocks
 * (all evaluation kernels), scratch bytes, term-evaluations per run.
 *
 * flags PEVAL_BATCH_TUNE: before planning, time candidate plans of this
 * batch on the device (the analogue of the paper's tile sweep, Section 4.4)
 * and keep the fastest: members are grouped by product and width and by
 * whether their K is the largest allowed, each group's K is moved one
 * doubling either way in turn (coordinate search), then the work items'
 * target cost is halved and doubled, then each kind's evaluations per pass
 * switched between 8 and 16.  Candidates run with base point 2 into
 * scratch outputs of sum(T_j G_j elem_bytes) bytes allocated for the search
 * (each timed as the median of five passes after a warm-up); a choice is
 * kept only when it is at least 1% faster.  Results never
 * depend on the plan.
 * peval_batch_members reports, per member j, its terms per thread K[j],
 * chains C[j] and kernel kind[j] (0: 64-bit Shoup with K = 16; 1: 64-bit
 * Shoup, K <= 8; 2: FP64 product; 3: 32-bit, K = 32; 4: 32-bit, K <= 16),
 * and the tuner's pass time and number of timed candidates (0 if the batch
 * was not tuned).  Any output pointer may be NULL.
 * flags PEVAL_BATCH_PASS8: every kind stages 8 evaluations per pass (without
 * PEVAL_BATCH_TUNE; for comparisons and tests).
 * peval_batch_kinds fills P[5] and blocks[5]: per kind (numbered as above)
 * its evaluations per pass and its kernel's persistent blocks, 0 for a kind
 * with no member.  Neither pointer may be NULL.
 */
typedef struct peval_batch peval_batch;
#define PEVAL_BATCH_NO_GRAPH 1u
#define PEVAL_BATCH_TUNE 2u
#define PEVAL_BATCH_PASS8 4u
int peval_batch_create(uint32_t count, peval_poly *const *polys, const uint32_t *Ts, uint32_t flags,
                       peval_batch **out);
int peval_batch_run(peval_batch *b, const uint64_t *const *betas, const uint64_t *t0s,
                    void *const *dev_outs, void *stream);
int peval_batch_info(const peval_batch *b, uint64_t *info);
int peval_batch_members(const peval_batch *b, uint32_t *K, uint32_t *C, uint32_t *kind, float *tuned_ms,
                        uint32_t *tune_trials);
int peval_batch_kinds(const peval_batch *b, uint32_t *P, uint32_t *blocks);
int peval_batch_destroy(peval_batch *b);

/*
 * Serving: a request loop over resident polynomials; every request asks for
 * the images b_1..b_T of Section 2.1 / Eq. (1) at its own base point.
 *
 * peval_server_create starts a scheduler thread on the current device.  The
 * server keeps polynomials resident within hbm_budget_bytes (resident term
 * data + request outputs + per-pass scratch), evicting the least recently
 * used polynomial with no request in flight when room is needed (its host
 * copy is kept, so a later request re-uploads it).  Requests are admitted in
 * arrival order when their memory fits; each is cut into slices of
 * consecutive evaluations and every pass batches one slice of each admitted
 * request into one batched launch; two passes run at a time on two streams,
 * so arrivals join the next pass (continuous batching).  Finished results
 * are copied to host memory by four copy threads (directly when host_out is
 * page-locked, through pinned staging otherwise).  A request's result
 * is identical to a plain peval_run of it.  flags: PEVAL_SERVER_SIMULATE
 * runs the same scheduler without any device call (passes take
 * term-evaluations / sim_rate seconds and produce no output), for testing
 * the policy on machines without a GPU.
 *
 * add_poly copies the polynomial (same rules as peval_create) and returns its
 * id; it becomes resident at its first admitted request.  submit queues
 * b_1..b_T at beta into host_out (T x G residues of the polynomial's width;
 * G = number of distinct (x1, x2) exponent pairs), which must stay valid
 * until the request is done; a request that could not fit in the budget
 * even alone is refused with PEVAL_ENOMEM (under a tight budget a request
 * first gets shorter slices).  poll sets *done; wait blocks
 * (timeout_ms < 0: forever; PEVAL_ETIMEOUT when it expires); both return the
 * request's error if it failed.  next_done hands out finished requests in
 * completion order.  release forgets a finished request.
 * Latency = submit to result in host memory.
 */
typedef struct peval_server peval_server;
#define PEVAL_SERVER_SIMULATE 1u
typedef struct peval_server_stats_t {
    uint64_t submitted, completed, rejected, queued, active, passes;
    uint64_t term_evals;        /* of completed requests */
    uint64_t uploads, evictions;  /* polynomials made resident / evicted */
    uint64_t slices;            /* request slices launched (members over all passes) */
    uint64_t hbm_in_use, hbm_peak;
    double wall_s;              /* from create (or reset) to the last completion */
    double p50_ms, p99_ms, max_ms, mean_ms;  /* request latency */
    double host_pass_s;         /* scheduler time spent planning and launching passes */
    double gpu_pass_s;          /* device time of the passes (start to end, summed) */
} peval_server_stats_t;
int peval_server_create(uint64_t hbm_budget_bytes, uint32_t flags, peval_server **out);
/* slice_work: target term-evaluations per request slice (default 2e9);
 * pass_work: term-evaluations gathered into one pass before launching it
 * (default 1.5e10; the oldest request always gets a slice, the others are
 * taken shortest remaining work first); max_members: slices per pass
 * (default 512); sim_rate: term-evaluations per second of the simulated
 * executor. */
int peval_server_configure(peval_server *srv, double slice_work, double pass_work, uint32_t max_members,
                           double sim_rate);
int peval_server_add_poly(peval_server *srv, uint64_t p, uint32_t n, uint64_t s, const uint32_t *exponents,
                          const uint64_t *coeffs, uint64_t *poly_id);
/* The registered polynomial's modulus, sizes and output shape (G columns of
 * elem_bytes, the layout submit writes); device_bytes is its resident size,
 * 0 while it is not resident. */
int peval_server_poly_info(peval_server *srv, uint64_t poly_id, peval_info_t *info);
int peval_server_remove_poly(peval_server *srv, uint64_t poly_id);
int peval_server_submit(peval_server *srv, uint64_t poly_id, const uint64_t *beta, uint32_t T, void *host_out,
                        uint64_t *req_id);
int peval_server_poll(peval_server *srv, uint64_t req_id, int *done);
int peval_server_wait(peval_server *srv, uint64_t req_id, int64_t timeout_ms);
/* Completion queue: the id of the next finished (or failed) request, in
 * completion order; waits up to timeout_ms (< 0: forever). */
int peval_server_next_done(peval_server *srv, int64_t timeout_ms, uint64_t *req_id);
int peval_server_release(peval_server *srv, uint64_t req_id);
int peval_server_stats(peval_server *srv, peval_server_stats_t *stats);
int peval_server_reset_stats(peval_server *srv);
int peval_server_destroy(peval_server *srv);

/*
 * Kernel timing (HIP events around each kernel on the launch stream).
 * enable != 0 starts recording for every handle; peval_prof_read returns
 * cumulative milliseconds and launch counts per kernel kind and resets them:
 * kind 0 power tables, 1 monomials and chain starts, 2 evaluation
 * (Hadamard product + coefficient reduction), 3 combine.
 * ms and launches are host arrays of 4 entries.  Reading synchronises with
 * the recorded events.
 */
int peval_prof_enable(int enable);
int peval_prof_read(double *ms, uint64_t *launches);

/*
 * Host-only layout planner (no device call; used by the tests on machines
 * without a GPU).  Given G group sizes (terms per distinct (x1, x2) pair, in
 * output-column order, each >= 1), K terms per thread and P evaluations per
 * pass, it computes the thread layout of the evaluation kernel:
 *   sizes[0] = NT threads (multiple of 64), sizes[1] = NW = NT/64 waves,
 *   sizes[2] = number of segment slots;
 *   thr_first[NT], thr_cnt[NT]  first term (offset in the sorted order) and
 *                               number of real terms (0..K) of each thread;
 *   endmask[NW]    bit l: lane l of the wave closes a segment (its group ends
 *                  there, or it is the wave's last lane: the evaluation
 *                  kernel merges a group's sub-tiles inside the wave);
 *   slot_base[NW]  index of the wave's first slot;
 *   slot_off[G+1]  slots of group g are slot_off[g] .. slot_off[g+1]-1.
 * Any of the array arguments may be NULL to skip it; otherwise they must hold
 * the sizes above (call once with NULL arrays to learn them).
 */
int peval_layout(const uint64_t *group_sizes, uint64_t G, uint32_t K, uint32_t P,
                 uint64_t *sizes, uint32_t *thr_first, uint8_t *thr_cnt,
                 uint64_t *endmask, uint32_t *slot_base, uint32_t *slot_off);

/* Error code name and the calling thread's last error message. */
const char *peval_strerror(int code);
const char *peval_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PEVAL_H */
