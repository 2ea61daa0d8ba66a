/*
 * peval test and measurement entry points: the device modular arithmetic of
 * the evaluation kernels run element by element, and a microbenchmark of the
 * modular products and of the gfx950 instructions they are made of.  Not
 * part of the evaluation path; same error conventions as peval.h.
 */
#ifndef PEVAL_TESTING_H
#define PEVAL_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Device arithmetic, one element per thread (paper, Section 3.1: the
 * modular product of Alg. 2 and the sums of Alg. 3, and their integer
 * counterparts used here).  For i < count, out[i] = op(a[i], b[i]) with
 * a, b, out device arrays of uint64 (signed values as two's complement).
 * Operand conditions are the caller's; the kernel applies the operation as
 * the evaluation kernels do.
 *
 * 64-bit residues (odd 3 <= p < 2^63):
 *   PEVAL_TOP_MUL64     a, b canonical -> a b mod p, canonical
 *   PEVAL_TOP_QUOT64    a canonical -> floor(a 2^64 / p) (Shoup quotient)
 *   PEVAL_TOP_SHOUP64   a any 64-bit word, b canonical -> the lazy Shoup
 *                       product of a by b with b's quotient, in [0, 2p)
 *   PEVAL_TOP_REDUCE96  (b mod 2^32) 2^64 + a -> canonical residue
 *   PEVAL_TOP_FOLD96    (b mod 2^32) 2^64 + a -> a 64-bit word congruent
 *                       to it (the segmented sums' partial coefficients)
 *   PEVAL_TOP_POW64     a canonical, b exponent -> a^b mod p (0^0 = 1)
 *   PEVAL_TOP_SUM64     count sums: out[i] = sum of a[16 i .. 16 i + 15]
 *                       (any 64-bit words) reduced mod p through the
 *                       evaluation kernel's half sums, their 96-bit fold
 *                       and its reduction
 * The FP64 product (2^31 <= p < 2^50):
 *   PEVAL_TOP_ALG2      a signed with |a| < p, b canonical -> the
 *                       rounded-quotient product of Alg. 2, signed, exact,
 *                       |result| < p
 *   PEVAL_TOP_FOLD      a signed with |a| < 2^53 -> a - rint(a / p) p
 *   PEVAL_TOP_CANON_F64 a signed with |a| < p -> its canonical residue as
 *                       uint64 (the conversion partial sums leave by)
 * Pseudo-Mersenne products:
 *   PEVAL_TOP_PM63      p = 2^63 - c (c < 2^20); a any 64-bit word, b < 2^63
 *                       -> a b mod p, lazy, in [0, 2p)
 *   PEVAL_TOP_PM31      p = 2^31 - c (c < 2^12); a, b < 2^32 -> lazy, < 2p
 * 32-bit residues (odd 3 <= p < 2^31), values in the low 32 bits:
 *   PEVAL_TOP_MUL32, PEVAL_TOP_QUOT32 (floor(a 2^32 / p)),
 *   PEVAL_TOP_SHOUP32 (a any 32-bit word), PEVAL_TOP_REDUCE64_32 (a any
 *   64-bit word -> canonical), PEVAL_TOP_POW32, PEVAL_TOP_SUM32 (16 values
 *   below 2^32 per sum) as for 64-bit residues.
 *   PEVAL_TOP_MONT32    a < 2p, b < p -> Montgomery's product a b 2^-32 mod
 *                       p, lazy in [0, 2p) (the point mode's factor tables)
 *
 * Returns PEVAL_EINVAL for an unknown op, a modulus outside the op's range
 * or null arrays with count > 0; enqueues on `stream` and returns.
 */
enum {
    PEVAL_TOP_MUL64 = 0, PEVAL_TOP_QUOT64 = 1, PEVAL_TOP_SHOUP64 = 2, PEVAL_TOP_REDUCE96 = 3,
    PEVAL_TOP_POW64 = 4, PEVAL_TOP_SUM64 = 5, PEVAL_TOP_FOLD96 = 6,
    PEVAL_TOP_ALG2 = 8, PEVAL_TOP_FOLD = 9, PEVAL_TOP_CANON_F64 = 10,
    PEVAL_TOP_PM63 = 12, PEVAL_TOP_PM31 = 13,
    PEVAL_TOP_MUL32 = 16, PEVAL_TOP_QUOT32 = 17, PEVAL_TOP_SHOUP32 = 18, PEVAL_TOP_REDUCE64_32 = 19,
    PEVAL_TOP_POW32 = 20, PEVAL_TOP_SUM32 = 21, PEVAL_TOP_MONT32 = 22
};
int peval_test_arith(uint32_t op, uint64_t p, uint64_t count, const uint64_t *dev_a, const uint64_t *dev_b,
                     uint64_t *dev_out, void *stream);

/*
 * Microbenchmark (the analogue of the paper's comparison of modular products,
 * Section 3.4, Fig. 1).  Runs `blocks` workgroups of 256 threads for `iters`
 * iterations of one kernel and returns its device time (HIP events) in *ms
 * and the work done in *work.  Blocks until done.
 *
 * Product kinds: every thread keeps 16 running values (8 for the FP64
 * product) with fixed multipliers, and each iteration adds each value into
 * the thread's sum and multiplies it by its multiplier (the loop of the
 * evaluation kernel without its stage and walk); *work = products
 * (each with its addition).  p must suit the product (as in
 * peval_test_arith); multipliers are drawn below p.
 *   PEVAL_MB_SHOUP64, PEVAL_MB_SHOUP32, PEVAL_MB_FP64, PEVAL_MB_PM63,
 *   PEVAL_MB_PM31
 * Instruction kinds (p ignored): eight independent dependency chains per
 * thread of one instruction; *work = lane-instructions.
 *   PEVAL_MB_ADD_U32 (v_add_u32), PEVAL_MB_MUL_LO_U32, PEVAL_MB_MUL_HI_U32,
 *   PEVAL_MB_MAD_U64_U32, PEVAL_MB_FMA_F64
 */
enum {
    PEVAL_MB_SHOUP64 = 0, PEVAL_MB_SHOUP32 = 1, PEVAL_MB_FP64 = 2, PEVAL_MB_PM63 = 3, PEVAL_MB_PM31 = 4,
    PEVAL_MB_ADD_U32 = 16, PEVAL_MB_MUL_LO_U32 = 17, PEVAL_MB_MUL_HI_U32 = 18, PEVAL_MB_MAD_U64_U32 = 19,
    PEVAL_MB_FMA_F64 = 20
};
int peval_bench_product(uint32_t kind, uint64_t p, uint32_t iters, uint32_t blocks, double *ms, double *work);

/*
 * Point mode (paper, Section 2.1, random points): which term takes each
 * thread slot of the point evaluation kernel, as the library deals them
 * (host only, no device needed).  w: bytes per residue (4 or 8); the terms
 * are given already sorted into G groups of group_sizes[g] >= 1 terms
 * (group g owns the next group_sizes[g] term indices); tail_exps: their
 * n - 2 tail exponents, variable-major (tail_exps[v * s + i], v < ntail);
 * K: terms per thread (1, 2, 4, 8 or 16).  slot_term receives K x NT term
 * indices (slot (k, j) at k * NT + j, 0xffffffff for padding), where NT is
 * the thread count of the layout (peval_layout's sizes[0] for this K);
 * slot_count must equal K * NT.  Every term lands in exactly one slot of
 * one of its own group's threads.  Returns PEVAL_EINVAL for bad arguments,
 * PEVAL_EUNSUPPORTED where the point mode's factor tables do not fit.
 */
int peval_test_deal_points(uint32_t w, uint32_t ntail, uint64_t s, const uint16_t *tail_exps, uint64_t G,
                           const uint64_t *group_sizes, uint32_t K, uint32_t *slot_term, uint64_t slot_count);

#ifdef __cplusplus
}
#endif

#endif /* PEVAL_TESTING_H */
