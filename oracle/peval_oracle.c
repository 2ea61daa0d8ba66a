/*
 * CPU oracle for partial modular polynomial evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark may use it.  It shares no code with the HIP path.
 *
 * What it computes (paper, Section 2.1 and Section 2.3, Eq. (1)):
 *
 *   f = sum_i a_i x1^{d_i} x2^{e_i} x3^{g_i3} ... xn^{g_in}  over F_p,
 *   b_t(x1, x2) = f(x1, x2, beta_3^t, ..., beta_n^t),   1 <= t <= T,
 *
 * and b_t is returned densely: the coefficient of x1^d x2^e in b_t is
 *
 *   out[t][(d,e)] = sum_{i : (d_i, e_i) = (d, e)} a_i * prod_{k=3..n} (beta_k^t)^{g_ik}  mod p.
 *
 * The columns are the distinct (d, e) pairs present in the input, sorted in
 * descending lexicographic order with x1 > x2 (the monomial order named in
 * Section 2.3 for the coefficient reductions).  Zero coefficients are kept.
 *
 * This is the plain definition written out: for every t the point beta^t is
 * formed first, then every term is evaluated at it by square-and-multiply.
 * It does NOT use the matrix method's recurrence M_i(beta^t) = m_i^t: the
 * oracle must stay independent of the method it checks.  Every product is a
 * 128-bit integer product reduced with the % operator, so every result is the
 * canonical residue in [0, p).
 *
 * Inputs are taken as integers and reduced modulo p on entry (coefficients
 * and base point), matching the convention that elements of F_p are residues.
 * 0^0 is 1 (an exponent of zero contributes the factor 1 for any base).
 *
 * Any modulus p >= 2 is accepted here (primality is not needed for the
 * definition); the product library restricts p further.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)(((u128)a * (u128)b) % p);
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)(((u128)a + (u128)b) % p);
}

/* base^e mod p by square-and-multiply; powmod(x, 0) = 1 mod p. */
static uint64_t powmod(uint64_t base, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    base %= p;
    while (e) {
        if (e & 1) r = mulmod(r, base, p);
        base = mulmod(base, base, p);
        e >>= 1;
    }
    return r;
}

/* descending lexicographic order on (d, e): x1 first, then x2 */
static int key_cmp_desc(uint64_t a, uint64_t b)
{
    return (a > b) ? -1 : (a < b) ? 1 : 0;
}

static int cmp_u64_desc(const void *x, const void *y)
{
    return key_cmp_desc(*(const uint64_t *)x, *(const uint64_t *)y);
}

static uint64_t group_key(const uint32_t *row)
{
    return ((uint64_t)row[0] << 32) | (uint64_t)row[1];
}

/*
 * Distinct (d, e) pairs of the s terms (row i of exps holds the exponents of
 * x1..xn of term i), descending lexicographic order.  Writes up to s keys to
 * gd/ge and the count to *G.  Returns 0, or -1 on allocation failure.
 */
int oracle_groups(uint64_t s, uint32_t n, const uint32_t *exps,
                  uint32_t *gd, uint32_t *ge, uint64_t *G)
{
    *G = 0;
    if (s == 0) return 0;
    uint64_t *keys = (uint64_t *)malloc(s * sizeof(uint64_t));
    if (!keys) return -1;
    for (uint64_t i = 0; i < s; ++i) keys[i] = group_key(exps + i * n);
    qsort(keys, s, sizeof(uint64_t), cmp_u64_desc);
    uint64_t g = 0;
    for (uint64_t i = 0; i < s; ++i) {
        if (i == 0 || keys[i] != keys[i - 1]) {
            gd[g] = (uint32_t)(keys[i] >> 32);
            ge[g] = (uint32_t)(keys[i] & 0xffffffffu);
            ++g;
        }
    }
    *G = g;
    free(keys);
    return 0;
}

/* position of key in the descending list gk[0..G-1] (binary search) */
static uint64_t find_group(const uint64_t *gk, uint64_t G, uint64_t key)
{
    uint64_t lo = 0, hi = G;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (gk[mid] > key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/*
 * The coefficient of every group at one point x = (x_3, ..., x_n) of
 * F_p^{n-2}: row[g] = sum_{i in g} a_i prod_k x_k^{g_ik} mod p.
 */
static void eval_at_point(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                          const uint64_t *coeffs, const uint64_t *x,
                          const uint64_t *gk, uint64_t G, uint64_t *row)
{
    memset(row, 0, G * sizeof(uint64_t));
    for (uint64_t i = 0; i < s; ++i) {
        const uint32_t *r = exps + i * n;
        uint64_t v = coeffs[i] % p;                       /* a_i */
        for (uint32_t k = 2; k < n; ++k)                  /* * x_k^{g_ik} */
            v = mulmod(v, powmod(x[k - 2], r[k], p), p);
        uint64_t g = find_group(gk, G, group_key(r));
        row[g] = addmod(row[g], v, p);
    }
}

/* One evaluation b_t: the coefficient of every group at the point beta^t. */
static void eval_one_t(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                       const uint64_t *coeffs, const uint64_t *beta, uint64_t t,
                       const uint64_t *gk, uint64_t G, uint64_t *row, uint64_t *bt)
{
    /* the point beta^t = (beta_3^t, ..., beta_n^t) */
    for (uint32_t k = 0; k + 2 < n; ++k) bt[k] = powmod(beta[k] % p, t, p);
    eval_at_point(p, n, s, exps, coeffs, bt, gk, G, row);
}

struct job {
    uint64_t p; uint32_t n; uint64_t s;
    const uint32_t *exps; const uint64_t *coeffs; const uint64_t *beta;
    const uint64_t *gk; uint64_t G;
    const uint64_t *points;     /* NULL: the powers beta^t; else T rows of n-2 values */
    uint64_t t_first, t_count, t0;
    uint64_t *out;
    int rc;
};

static void *run_job(void *arg)
{
    struct job *j = (struct job *)arg;
    uint64_t *bt = (uint64_t *)malloc((j->n > 2 ? j->n - 2 : 1) * sizeof(uint64_t));
    if (!bt) { j->rc = -1; return NULL; }
    uint32_t m = j->n - 2;
    for (uint64_t q = 0; q < j->t_count; ++q) {
        uint64_t t = j->t_first + q;
        uint64_t *row = j->out + (t - j->t0) * j->G;
        if (j->points) {
            for (uint32_t k = 0; k < m; ++k) bt[k] = j->points[(t - j->t0) * m + k] % j->p;
            eval_at_point(j->p, j->n, j->s, j->exps, j->coeffs, bt, j->gk, j->G, row);
        } else {
            eval_one_t(j->p, j->n, j->s, j->exps, j->coeffs, j->beta, t, j->gk, j->G, row, bt);
        }
    }
    free(bt);
    j->rc = 0;
    return NULL;
}

/* shared driver: t ranges split over threads; points == NULL selects beta^t */
static int eval_images(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                       const uint64_t *coeffs, const uint64_t *beta, const uint64_t *points,
                       uint64_t t0, uint64_t T, uint64_t *out, uint32_t nthreads)
{
    if (p < 2 || n < 2 || nthreads == 0) return -2;
    if (T == 0) return 0;
    uint32_t *gd = (uint32_t *)malloc((s ? s : 1) * sizeof(uint32_t));
    uint32_t *ge = (uint32_t *)malloc((s ? s : 1) * sizeof(uint32_t));
    uint64_t *gk = (uint64_t *)malloc((s ? s : 1) * sizeof(uint64_t));
    uint64_t G = 0;
    int rc = -1;
    if (!gd || !ge || !gk) goto done;
    if (oracle_groups(s, n, exps, gd, ge, &G) != 0) goto done;
    for (uint64_t g = 0; g < G; ++g) gk[g] = ((uint64_t)gd[g] << 32) | ge[g];
    if (G == 0) { rc = 0; goto done; }
    {
        if (nthreads > T) nthreads = (uint32_t)T;
        struct job *jobs = (struct job *)calloc(nthreads, sizeof(struct job));
        pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
        if (!jobs || !th) { free(jobs); free(th); goto done; }
        uint64_t base = T / nthreads, extra = T % nthreads, next = t0;
        for (uint32_t w = 0; w < nthreads; ++w) {
            uint64_t cnt = base + (w < extra ? 1 : 0);
            jobs[w] = (struct job){p, n, s, exps, coeffs, beta, gk, G, points, next, cnt, t0, out, -1};
            next += cnt;
        }
        rc = 0;
        if (nthreads == 1) {
            run_job(&jobs[0]);
            rc = jobs[0].rc;
        } else {
            uint32_t started = 0;
            for (; started < nthreads; ++started)
                if (pthread_create(&th[started], NULL, run_job, &jobs[started]) != 0) break;
            for (uint32_t w = 0; w < started; ++w) pthread_join(th[w], NULL);
            if (started < nthreads) rc = -1;
            for (uint32_t w = 0; w < started; ++w) if (jobs[w].rc) rc = jobs[w].rc;
        }
        free(jobs);
        free(th);
    }
done:
    free(gd); free(ge); free(gk);
    return rc;
}

/*
 * Dense bivariate images b_t for t = t0 .. t0+T-1.
 *
 * p >= 2; n >= 2; exps: s rows of n uint32 exponents; coeffs: s values;
 * beta: n-2 values (beta_3..beta_n).  out: T*G values, row (t - t0) holds
 * b_t in the column order of oracle_groups.  nthreads >= 1 splits the t range
 * into contiguous chunks, one per thread; the result does not depend on it.
 * Returns 0, -1 on allocation failure, -2 on invalid arguments.
 */
int oracle_eval(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                const uint64_t *coeffs, const uint64_t *beta, uint64_t t0, uint64_t T,
                uint64_t *out, uint32_t nthreads)
{
    return eval_images(p, n, s, exps, coeffs, beta, NULL, t0, T, out, nthreads);
}

/*
 * Images at T arbitrary points instead of the powers of one base point (the
 * random evaluation points of Zippel's original method, Section 2.1; cost
 * O(nT(d+s)), Section 2.3):
 *
 *   out[t][(d,e)] = sum_{i : (d_i, e_i) = (d, e)} a_i prod_{k=3..n} x_{t,k}^{g_ik}  mod p
 *
 * points: T rows of n-2 values (x_{t,3} .. x_{t,n}), reduced mod p on entry.
 * Same column order, threading and return codes as oracle_eval.
 */
int oracle_eval_points(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                       const uint64_t *coeffs, const uint64_t *points, uint64_t T,
                       uint64_t *out, uint32_t nthreads)
{
    return eval_images(p, n, s, exps, coeffs, NULL, points, 0, T, out, nthreads);
}

/*
 * One coefficient: the coefficient of x1^d x2^e in b_t, straight from the
 * definition (for spot checks at sizes where the full table is too large).
 * Returns the canonical residue; a (d, e) absent from the input gives 0.
 */
uint64_t oracle_entry(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                      const uint64_t *coeffs, const uint64_t *beta, uint64_t t,
                      uint32_t d, uint32_t e)
{
    uint64_t acc = 0;
    for (uint64_t i = 0; i < s; ++i) {
        const uint32_t *r = exps + i * n;
        if (r[0] != d || r[1] != e) continue;
        uint64_t v = coeffs[i] % p;
        for (uint32_t k = 2; k < n; ++k)
            v = mulmod(v, powmod(powmod(beta[k - 2] % p, t, p), r[k], p), p);
        acc = addmod(acc, v, p);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Sparse interpolation from the images (the step that follows the          */
/* evaluations in Zippel's method, Section 2.1)                             */
/* ------------------------------------------------------------------------ */

/* inverse of a modulo p by the extended Euclidean algorithm; 0 if none */
static uint64_t invmod(uint64_t a, uint64_t p)
{
    __int128 r0 = (__int128)p, r1 = (__int128)(a % p), s0 = 0, s1 = 1;
    while (r1 != 0) {
        __int128 q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    if (r0 != 1) return 0;
    s0 %= (__int128)p;
    if (s0 < 0) s0 += p;
    return (uint64_t)s0;
}

/*
 * Solve V a = c over F_p by Gauss-Jordan elimination with row pivoting,
 * where V is the m x m matrix (row-major) and c has m entries; the solution
 * overwrites c.  Returns 0, or -3 if V is singular modulo p.
 */
static int gauss_solve(uint64_t *V, uint64_t *c, uint64_t m, uint64_t p)
{
    for (uint64_t col = 0; col < m; ++col) {
        uint64_t piv = col;
        while (piv < m && V[piv * m + col] == 0) ++piv;
        if (piv == m) return -3;
        if (piv != col) {
            for (uint64_t j = 0; j < m; ++j) {
                uint64_t t = V[col * m + j]; V[col * m + j] = V[piv * m + j]; V[piv * m + j] = t;
            }
            uint64_t t = c[col]; c[col] = c[piv]; c[piv] = t;
        }
        uint64_t inv = invmod(V[col * m + col], p);
        if (inv == 0) return -3;
        for (uint64_t j = 0; j < m; ++j) V[col * m + j] = mulmod(V[col * m + j], inv, p);
        c[col] = mulmod(c[col], inv, p);
        for (uint64_t r = 0; r < m; ++r) {
            if (r == col || V[r * m + col] == 0) continue;
            uint64_t f = V[r * m + col];
            for (uint64_t j = 0; j < m; ++j)
                V[r * m + j] = addmod(V[r * m + j], p - mulmod(f, V[col * m + j], p), p);
            c[r] = addmod(c[r], p - mulmod(f, c[col], p), p);
        }
    }
    return 0;
}

/*
 * Coefficients from the images.  Given the support of f (exponent rows), the
 * base point beta and the images b_1..b_T in the dense layout of oracle_eval
 * (T rows of G columns), find the coefficients a_i: for every group (d, e)
 * with terms i_1..i_m, the coefficient of x1^d x2^e in b_t is
 *
 *   c_t = sum_j a_{i_j} m_{i_j}^t,   m_i = prod_{k=3..n} beta_k^{g_ik},
 *
 * so the a's of the group solve the m x m system V a = c with
 * V[t-1][j] = m_{i_j}^t, t = 1..m (a transposed Vandermonde system scaled by
 * the m's; Section 2.1).  This is the plain definition solved by elimination,
 * O(m^3) per group; only the first m rows of the group's column are used.
 *
 * coeffs_out: s values, in the order of the input rows (duplicate rows of
 * the support are not allowed: their monomial values coincide).  Returns 0;
 * -1 on allocation failure; -2 on invalid arguments or T smaller than the
 * largest group; -3 if some group's system is singular (two of its terms
 * share a monomial value, or a monomial value is 0 or not invertible).
 */
int oracle_interpolate(uint64_t p, uint32_t n, uint64_t s, const uint32_t *exps,
                       const uint64_t *beta, uint64_t T, const uint64_t *images,
                       uint64_t *coeffs_out)
{
    if (p < 2 || n < 2) return -2;
    int rc = -1;
    uint32_t *gd = (uint32_t *)malloc((s ? s : 1) * sizeof(uint32_t));
    uint32_t *ge = (uint32_t *)malloc((s ? s : 1) * sizeof(uint32_t));
    uint64_t *gk = (uint64_t *)malloc((s ? s : 1) * sizeof(uint64_t));
    uint64_t *gid = (uint64_t *)malloc((s ? s : 1) * sizeof(uint64_t));
    uint64_t *mono = (uint64_t *)malloc((s ? s : 1) * sizeof(uint64_t));
    uint64_t *members = (uint64_t *)malloc((s ? s : 1) * sizeof(uint64_t));
    uint64_t *V = NULL, *c = NULL;
    uint64_t G = 0;
    if (!gd || !ge || !gk || !gid || !mono || !members) goto done;
    if (oracle_groups(s, n, exps, gd, ge, &G) != 0) goto done;
    for (uint64_t g = 0; g < G; ++g) gk[g] = ((uint64_t)gd[g] << 32) | ge[g];
    for (uint64_t i = 0; i < s; ++i) {
        const uint32_t *r = exps + i * n;
        gid[i] = find_group(gk, G, group_key(r));
        uint64_t v = 1 % p;
        for (uint32_t k = 2; k < n; ++k) v = mulmod(v, powmod(beta[k - 2] % p, r[k], p), p);
        mono[i] = v;
    }
    rc = 0;
    for (uint64_t g = 0; g < G && rc == 0; ++g) {
        uint64_t m = 0;
        for (uint64_t i = 0; i < s; ++i) if (gid[i] == g) members[m++] = i;
        if (m > T) { rc = -2; break; }
        V = (uint64_t *)malloc(m * m * sizeof(uint64_t));
        c = (uint64_t *)malloc(m * sizeof(uint64_t));
        if (!V || !c) { rc = -1; break; }
        for (uint64_t t = 1; t <= m; ++t) {
            for (uint64_t j = 0; j < m; ++j) V[(t - 1) * m + j] = powmod(mono[members[j]], t, p);
            c[t - 1] = images[(t - 1) * G + g] % p;
        }
        rc = gauss_solve(V, c, m, p);
        if (rc == 0)
            for (uint64_t j = 0; j < m; ++j) coeffs_out[members[j]] = c[j];
        free(V); free(c); V = NULL; c = NULL;
    }
done:
    free(V); free(c);
    free(gd); free(ge); free(gk); free(gid); free(mono); free(members);
    return rc;
}
