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
    PEVAL_EUNSUPPORTED = -4,  /* valid input outside what this build supports */
    PEVAL_EBUSY = -5,         /* resource temporarily unavailable (server) */
    PEVAL_ETIMEOUT = -6       /* wait ended before completion */
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
 */
int peval_run_async(peval_poly *h, const uint64_t *beta, uint64_t t0, uint32_t T,
                    void *dev_out, void *stream);

/* Release the handle and its device memory (waits for its pending work).
 * NULL is accepted. */
int peval_destroy(peval_poly *h);

/*
 * Tuning knobs of the evaluation kernel for one handle (0 = automatic):
 *   K      terms held per thread (1, 2, 4, 8, 16)
 *   P      evaluations per pass before each coefficient reduction (8, 16, 32)
 *   C      independent evaluation chains (>= 1; chain c does t = t0+c, t0+c+C, ...)
 * The results never depend on these; only speed does.
 */
int peval_set_tuning(peval_poly *h, uint32_t K, uint32_t P, uint32_t C);

/* The tuning the next run with T evaluations would use. */
int peval_get_tuning(peval_poly *h, uint32_t T, uint32_t *K, uint32_t *P, uint32_t *C);

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
 *                  there or its sub-tile of P lanes ends there);
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
