/*
 * dqt.h -- C ABI of libdqt, the MI355X (gfx950) packed-DQT / REDQ library.
 *
 * Method: Dumas, Fousse, Salvy, "Simultaneous Modular Reduction and Kronecker
 * Substitution for Small Finite Fields".  Polynomials over F_p are packed into
 * machine words by evaluation at q = 2^log2q (the DQT map, equation eq:dqt),
 * multiplied and accumulated as integers while every q-adic digit stays below
 * q (the a priori bounds eq:bounds / eq:lower / eq:upper), and recovered with
 * REDQ (section 3): one floating-point floor for the whole word (section 4,
 * algorithm AFDIV), field-parallel integer operations, and a correction read
 * from tables held in LDS.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a dqt_status; none aborts, throws or prints.
 * - Residues are uint8 values in [0, p), 2 <= p <= 255.  Inputs with an entry
 *   >= p give unspecified (but memory-safe) results; debug mode
 *   (dqt_debug_enable) reports them as DQT_E_INPUT instead.
 * - Coefficient i of a polynomial is the coefficient of X^i (low degree first).
 * - Pointers named d_* are device pointers (HIP global memory) owned by the
 *   caller; the library allocates no device memory and keeps no pointer after
 *   the call returns.  `stream` is a hipStream_t (NULL = the null stream);
 *   all device work is enqueued asynchronously on it.
 * - Argument and bound checks run on the host, synchronously, before anything
 *   is enqueued.  On an error nothing is enqueued.  DQT_E_DEVICE reports a HIP
 *   runtime error; dqt_last_error() gives its text (thread-local).
 * - Calls on distinct streams with distinct output buffers may run
 *   concurrently.
 * - The first call that enqueues work on a device runs a one-thread check on
 *   the null stream and waits for it: REDQ's floor by one binary64 multiply
 *   (section 4, case 2 of the FDIV table) needs round-to-nearest, and a device
 *   in another rounding mode gets DQT_E_UNSUPPORTED from every later call.
 *   Make that first call before capturing a stream into a graph.
 */
#ifndef DQT_H
#define DQT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dqt_status {
    DQT_OK = 0,
    DQT_E_INVALID = -1,     /* null pointer, p outside [2,255], zero or overflowing sizes */
    DQT_E_BOUND = -2,       /* parameters violate the paper's a priori bounds */
    DQT_E_UNSUPPORTED = -3, /* valid, but outside what the kernels implement */
    DQT_E_DEVICE = -4,      /* HIP runtime error (see dqt_last_error) */
    DQT_E_WORKSPACE = -5,   /* workspace null or smaller than required */
    DQT_E_INPUT = -6        /* a device-side check failed: an entry not a residue in [0, p), a packed
                               operand or REDQ word outside its bounds (debug mode, dqt_sync_status,
                               dqt_check_input_u8) */
} dqt_status;

/* Text of a status code (static storage). */
const char *dqt_status_str(dqt_status s);
/* Text of the last HIP error seen by this thread ("" if none). */
const char *dqt_last_error(void);
/* Library version string. */
const char *dqt_version(void);

/*
 * REDQ correction tables (section 3.5, the time-memory trade-off): the
 * correction mu_i = (u_i - (q mod p) u_{i+1}) mod p is read from an LDS table
 * indexed by a window of j consecutive residues (2^(j ceil(log2 p)) entries,
 * j-1 corrected residues per lookup) or computed arithmetically.
 * dqt_set_table_window(j) applies to the calls that follow, process-wide:
 * 0 = automatic (the largest of 3, 2 whose table has at most 4096 entries),
 * 1 = no table, 2 = windows of two residues at most, 3 = three at most
 * (each falls back to a smaller window when its table would not fit).
 * DQT_E_INVALID for j > 3.  Results are identical for every j.
 */
dqt_status dqt_set_table_window(uint32_t j);
uint32_t dqt_get_table_window(void);

/*
 * Debug mode: device-side checks with a status word.
 * The a priori bounds (eq:bounds, eq:lower) hold only for entries that are
 * residues in [0, p), and REDQ (algorithm REDQ, section 3.2) only for words
 * whose lower digits are below q and that are exact in binary64 (AFDIV,
 * section 4).  The host cannot see the data, so with debug mode on every
 * entry point, after its host checks and before it enqueues its own work,
 * checks on its stream the data it is given: uint8 entries < p (status bit
 * 1); the packed operand words of dqt_polymul have k_coeffs fields below p
 * and nothing above (bit 2: by eq:bounds every digit of their product is
 * then below q); the words given to redq_unpack are below 2^beta (bit 4).
 * It then waits for the stream, reads and clears the status word and returns
 * DQT_E_INPUT (nothing else enqueued, dqt_last_error names the check) if a
 * bit was set.  dqt_fgemm_packed and dqt_fgemm_compute take packed operands
 * that were checked when they were packed.
 *
 * dqt_debug_enable(d_status): turns debug mode on (process-wide) with the
 * caller's 4-byte device word d_status on the current device (zeroed here,
 * synchronously), or off with NULL.  The word must stay valid while debug
 * mode is on; calls on another device return DQT_E_INVALID, and calls on a
 * stream under graph capture DQT_E_UNSUPPORTED (the checks wait).
 * dqt_sync_status(stream): waits for `stream`, then reads and clears the
 * status word: DQT_E_INPUT if a check failed since the last read, DQT_OK
 * otherwise (and DQT_OK after the wait when debug mode is off).
 */
dqt_status dqt_debug_enable(uint32_t *d_status);
dqt_status dqt_sync_status(void *stream);

/*
 * Input validation on demand.  The packed paths assume every entry is a
 * residue in [0, p): the a priori bounds (eq:bounds, eq:lower) are stated for
 * entries at most p-1, and a larger entry silently breaks them.  This call
 * checks `count` bytes at d_x on `stream`, using the caller's 4-byte device
 * word d_flag (no allocation), waits for the stream, and returns DQT_E_INPUT
 * if some entry is >= p, DQT_OK otherwise.  Blocking; meant for debugging and
 * tests, not for the timed paths.
 */
dqt_status dqt_check_input_u8(const uint8_t *d_x, uint64_t count, uint32_t p, uint32_t *d_flag, void *stream);

/*
 * q-adic packing parameters (section 2.3, theorem eq:bounds).
 *   p        the prime.
 *   log2q    q = 2^log2q, the evaluation point.
 *   k_coeffs coefficients per packed operand (polynomials of degree < k_coeffs).
 *   nres     digits of a packed result, 2*k_coeffs - 1 for a product (REDQ_nres).
 *   n_accum  number of products summed into one result word before REDQ
 *            (the n of eq:bounds); 1 for a single product.
 *   word_bits beta, the width of the words REDQ reduces: packed results are
 *            below 2^word_bits.  0 means 53 (the binary64 mantissa, so that
 *            REDQ's one division is one FP64 multiply and floor, section 4);
 *            values above 53 give DQT_E_UNSUPPORTED.
 * Every packed word is a uint64 holding nres fields of log2q bits.
 */
typedef struct dqt_qadic {
    uint32_t p;
    uint32_t log2q;
    uint32_t k_coeffs;
    uint32_t nres;
    uint64_t n_accum;
    uint32_t word_bits;
} dqt_qadic;

/*
 * Host-only check of a parameter set.  DQT_OK iff
 *   q > n_accum * k_coeffs * (p-1)^2     (eq:bounds, digits never carry),
 *   nres * log2q <= beta                 (eq:bounds: the word is below
 *                                         2^beta, beta = word_bits or 53),
 *   log2q <= 32, 1 <= k_coeffs, 1 <= nres <= 32.
 * Returns DQT_E_INVALID for null or malformed input, DQT_E_UNSUPPORTED for
 * beta > 53, DQT_E_BOUND otherwise.
 */
dqt_status dqt_qadic_check(const dqt_qadic *a);

/*
 * Host-only: the smallest log2q satisfying dqt_qadic_check for (p, k_coeffs,
 * n_accum, word_bits) with nres = 2*k_coeffs - 1.  Writes *out on success;
 * DQT_E_BOUND when no q fits in beta bits.
 */
dqt_status dqt_qadic_choose(uint32_t p, uint32_t k_coeffs, uint64_t n_accum, uint32_t word_bits, dqt_qadic *out);

/*
 * DQT map (equation eq:dqt; section 2.1 with q = 2^log2q a shift).
 * d_coeffs: uint8 [count][a->k_coeffs]; d_words: uint64 [count].
 * reverse = 0: word = sum_i c_i q^i.  reverse != 0: word = sum_i c_i q^(k-1-i)
 * (the reversed row packing of the compressed matrix product, section 7.1).
 * count == 0 is a no-op.
 */
dqt_status dqt_pack(const uint8_t *d_coeffs, uint64_t count, const dqt_qadic *a, int reverse,
                    uint64_t *d_words, void *stream);

/*
 * Packed product (equation eq:mult): d_r[t] = d_a[t] * d_b[t] as integers,
 * i.e. the Kronecker product of two packed polynomials, left unreduced.
 * Requires dqt_qadic_check(a) == DQT_OK with n_accum >= 1 and
 * nres == 2*k_coeffs - 1.  Word layout as dqt_pack.
 */
dqt_status dqt_polymul(const uint64_t *d_a, const uint64_t *d_b, uint64_t count, const dqt_qadic *a,
                       uint64_t *d_r, void *stream);

/*
 * REDQ (algorithm REDQ, section 3.2, with the binary-case compression of
 * section 3.3, the tabulated correction of section 3.5 and the FP64 floor of
 * algorithm AFDIV, section 4.6).
 * d_r: uint64 [count] packed words r = sum_{i<nres} m_i q^i whose lower
 * digits m_0..m_{nres-2} are < q (the REQUIRE of algorithm REDQ, section
 * 3.2: guaranteed by eq:bounds when the words come from products of packed
 * residues, the caller's guarantee otherwise; the top digit may exceed q)
 * and r < 2^beta, beta = a->word_bits or 53 (AFDIV's domain).  Checked on
 * the host: nres * log2q <= 53 (DQT_E_BOUND otherwise) and log2q >=
 * ceil(log2 p) (DQT_E_UNSUPPORTED otherwise); n_accum and the first part of
 * eq:bounds are not used.  In debug mode (dqt_debug_enable) the words are
 * checked to be below 2^beta on the device first (DQT_E_INPUT otherwise);
 * the digit condition is asserted where it can fail, on the packed operands
 * of dqt_polymul and the uint8 inputs of the packing and fused calls.
 * modulus == NULL: d_out uint8 [count][nres], d_out[t][i] = m_i mod p.
 * modulus != NULL (GF(p^k) reduction by two tables, algorithm FGDP, theorem
 * thm:fgdp): host pointer to k_coeffs+1 coefficients of a monic polynomial P
 * (modulus[k_coeffs] == 1), nres must be 2*k_coeffs-1, k_coeffs <= 6, and
 * d_out is uint8 [count][k_coeffs] = (sum_i m_i X^i mod p) mod P.
 */
dqt_status redq_unpack(const uint64_t *d_r, uint64_t count, const dqt_qadic *a, const uint8_t *modulus,
                       uint8_t *d_out, void *stream);

/*
 * Fused one-word polynomial product: pack + product + REDQ + store, in one
 * kernel.  d_a, d_b: uint8 [count][k]; d_out: uint8 [count][2k-1], the
 * product mod p (zeros included).  log2q = 0 takes the smallest q allowed by
 * eq:bounds (dqt_qadic_choose(p, k, 1)); a given log2q must satisfy
 * dqt_qadic_check with n_accum = 1 (DQT_E_BOUND otherwise).
 * DQT_E_UNSUPPORTED if no q fits in one 53-bit word (k too large for p) or
 * k > 9.
 */
dqt_status dqt_polymul_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t k, uint32_t p,
                          uint32_t log2q, uint8_t *d_out, void *stream);

/*
 * Fused GF(p^k) product (section 6, algorithm FGDP, its two-table reduction on single
 * products): d_a, d_b, d_out uint8 [count][k], modulus a host pointer to the
 * k+1 coefficients of a monic P (not checked for irreducibility: the result
 * is the product in F_p[X]/(P)).  2 <= k <= 6, k*ceil(log2 p) <= 12 (the two
 * tables of 2^(k ceil(log2 p)) entries live in LDS).  log2q as for
 * dqt_polymul_u8.
 */
dqt_status dqt_gf_mul_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t k, uint32_t p,
                         uint32_t log2q, const uint8_t *modulus, uint8_t *d_out, void *stream);

/*
 * Dot products over GF(p^k) (algorithm FGDP, section 6, theorem thm:fgdp):
 * d_out[t] = sum_{l<n} a[t][l] * b[t][l] in F_p[X]/(P).  d_a, d_b: uint8
 * [count][n][k], d_out: uint8 [count][k]; modulus as for dqt_gf_mul_u8.
 * Products are accumulated in packed words, n_q at a time, with q the
 * largest power of two such that (2k-1) log2 q <= 53 and n_q the largest
 * count with q > n_q k (p-1)^2 (eq:bounds); each word costs one REDQ
 * compression, two table lookups and one field addition.  p <= 127,
 * 2 <= k <= 6, k ceil(log2 p) <= 12; DQT_E_UNSUPPORTED when not even one
 * product fits such a word.
 */
dqt_status dqt_gf_dot_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t n, uint32_t k, uint32_t p,
                         const uint8_t *modulus, uint8_t *d_out, void *stream);

/*
 * Matrix products over GF(p^k) by algorithm FGDP (section 6): C[i][j] =
 * sum_l A[i][l] B[l][j], every entry a dot product of field elements summed
 * n_q products at a time in packed form (the same q, n_q, REDQ and two tables
 * as dqt_gf_dot_u8).  d_a: uint8 [m][kd][k], d_b: uint8 [kd][n][k], d_out:
 * uint8 [m][n][k], all row-major and dense; modulus as for dqt_gf_mul_u8.
 * kd = 0 gives zeros; m or n = 0 is a no-op.  p <= 127, 2 <= k <= 6, k w <= 11
 * (w = bits of p - 1: the two tables of 2^(k w) entries share a workgroup's
 * 64 KiB of LDS with the tiles), m <= 4,194,240; DQT_E_UNSUPPORTED otherwise.
 */
dqt_status dqt_gf_matmul_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t m, uint64_t n, uint64_t kd, uint32_t k,
                            uint32_t p, const uint8_t *modulus, uint8_t *d_out, void *stream);

/*
 * Plain per-entry comparators (the paper's "delayed" baseline, section 5.1):
 * one coefficient per machine multiply-add, integer accumulation, one
 * reduction (REDC) per output coefficient.  Same layouts and results as the
 * packed entry points.  dqt_polymul_plain_u8 accepts any k <= 4096 (above 64
 * coefficients a workgroup, or for short products a group of lanes of one
 * wave, computes a product, eight output coefficients per lane, operands in
 * LDS).
 */
dqt_status dqt_polymul_plain_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t k, uint32_t p,
                                uint8_t *d_out, void *stream);
dqt_status dqt_gf_mul_plain_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t k, uint32_t p,
                               const uint8_t *modulus, uint8_t *d_out, void *stream);

/*
 * Long polynomial products by the FQT (section 5.2): P = sum_i P_i Y^i with
 * Y = X^(d+1) and each block P_i of d+1 coefficients packed in one word; block
 * products are summed in packed form (delayed, at most the n_q of section 5.3
 * per word) and each output block is recovered by one REDQ_{2d+1}; the d
 * overlapping coefficients of consecutive blocks are added mod p.
 * d_a: uint8 [count][na], d_b: uint8 [count][nb], d_out: uint8 [count][na+nb-1].
 * block = d+1 coefficients per word (0 = choose).  na, nb <= 4096.  Up to 64
 * coefficients each, a thread computes a product and every output block holds
 * all its block products in one word.  Above that, and at up to 64 where no
 * block size keeps such a sum in one word and block = 0 (p <= 127, block
 * 2..4), one workgroup (or, for products of up to 64 pairs of chunks, a
 * group of lanes of one wave, four waves sharing a workgroup) computes a
 * product: the block words of both operands sit in LDS,
 * each output block is summed n_q block products at a time
 * (q > n_q (d+1)(p-1)^2, eq:bounds, with (2d+1) log2 q <= 51), with one
 * REDQ_{2d+1} per such sum and the sums' residues added mod p; the block size
 * minimizes section 5.3's counts (block products, reductions) weighted by
 * their cost in the kernel.  DQT_E_UNSUPPORTED for p > 127 there.
 */
dqt_status dqt_polymul_fqt_u8(const uint8_t *d_a, uint32_t na, const uint8_t *d_b, uint32_t nb, uint64_t count,
                              uint32_t p, uint32_t block, uint8_t *d_out, void *stream);

/*
 * Long products by Karatsuba's recursion over F_p with the packed FQT at its
 * base (section 5.3, figure fig:pmkara): `levels` (1..3) levels each turn a
 * product of two n-coefficient polynomials into three products of
 * h = ceil(n/2) coefficients (a0 b0, a1 b1, (a0 + a1)(b0 + b1), the sums
 * reduced mod p), the 3^levels base products run through dqt_polymul_fqt_u8,
 * and the results are combined back, a b = P0 + x^h (P1 - P0 - P2) + x^2h P2
 * mod p.  d_a, d_b: uint8 [count][n]; d_out: uint8 [count][2n-1]; same bytes
 * as dqt_polymul_fqt_u8.  d_work: device workspace of at least
 * dqt_polymul_kara_long_workspace(count, n, levels) bytes (the split operands
 * and the products of every level), owned by the caller, not retained.
 * DQT_E_INVALID for levels outside 1..3, n outside 2..4096 or a base size
 * below 2; DQT_E_WORKSPACE for a short workspace; the base products' own
 * errors (DQT_E_UNSUPPORTED for p > 127 when they exceed 64 coefficients).
 * dqt_polymul_kara_long_workspace returns 0 for invalid arguments.
 */
size_t dqt_polymul_kara_long_workspace(uint64_t count, uint32_t n, uint32_t levels);
dqt_status dqt_polymul_kara_long_u8(const uint8_t *d_a, const uint8_t *d_b, uint64_t count, uint32_t n, uint32_t p,
                                    uint32_t levels, uint8_t *d_out, void *d_work, size_t work_bytes, void *stream);

/*
 * dqt_polymul_fqt_u8 with the block products by Karatsuba's recursion
 * (`levels` = 1 or 2 levels, schoolbook below; the subquadratic FQT of
 * section 5.3, figure fig:pmkara).  The recursion runs on the packed block
 * words as integers modulo 2^64 (the evaluation at q is a ring morphism), so
 * the output blocks, their REDQ and the bytes are those of
 * dqt_polymul_fqt_u8.  Same arguments and errors; DQT_E_INVALID for another
 * `levels`.
 */
dqt_status dqt_polymul_fqt_kara_u8(const uint8_t *d_a, uint32_t na, const uint8_t *d_b, uint32_t nb, uint64_t count,
                                   uint32_t p, uint32_t block, uint32_t levels, uint8_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * F_p matrix product C = A.B mod p (section 7).
 * A: uint8 m x kdim, row-major, leading dimension lda >= kdim.
 * B: uint8 kdim x n, row-major, ldb >= n.  C: uint8 m x n, ldc >= n.
 * m or n may be 0 (no-op); kdim == 0 gives C = 0 (empty sums) without
 * reading A, B or the workspace; none needs to be a multiple of any tile.
 * ------------------------------------------------------------------------ */

typedef enum dqt_gemm_algo {
    DQT_GEMM_AUTO = 0,      /* CMM when the packing bounds allow it, else PLAIN */
    DQT_GEMM_CMM = 1,       /* compressed (middle product, section 7.1) on packed words */
    DQT_GEMM_PLAIN = 2,     /* one entry per multiply-add, delayed REDC */
    DQT_GEMM_DOT4 = 3,      /* plain, four u8 entries per hardware dot instruction */
    DQT_GEMM_MFMA = 4,      /* plain, INT8 matrix cores, exact int32 accumulation */
    DQT_GEMM_RIGHT = 5,     /* right compressed (section 7.4): e columns of B per binary64 word, A
                               uncompressed, product on the FP64 matrix cores, one REDQ_e per word */
    DQT_GEMM_LEFT = 6,      /* left compressed (section 7.4, the transpose): e rows of A per word */
    DQT_GEMM_FULL = 7,      /* full compression (section 7.5): 2 rows of A in powers of Q times e_c
                               columns of B in powers of Theta = Q^2, 2 e_c digits per word */
    DQT_GEMM_BY_SHAPE = 8,  /* the rule of section 7.6.2: CMM (as AUTO) when kdim is the largest
                               dimension, RIGHT when n is, LEFT when m is */
    DQT_GEMM_DOT8 = 9       /* plain, p <= 16: eight 4-bit entries per word, one hardware dot
                               instruction per eight multiply-adds (DQT_E_UNSUPPORTED for p > 16) */
} dqt_gemm_algo;

typedef enum dqt_gemm_epilogue {
    DQT_EPI_REDC = 0,       /* one reduction per output (section 7.2) */
    DQT_EPI_REDQ = 1        /* middle digits gathered e per word and reduced by one REDQ_e */
} dqt_gemm_epilogue;

typedef struct dqt_gemm_plan {
    uint32_t algo;          /* dqt_gemm_algo */
    uint32_t log2Q;         /* 0 = smallest allowed by eq:lower for the interval */
    uint32_t interval;      /* delayed-reduction interval in k (0 = whole kdim); multiple of 4 */
    uint32_t tile_rows;     /* rows per wave (CMM/PLAIN/DOT4: 8, 16 or 32; 0 = default 8) */
    uint32_t ksplit;        /* waves splitting kdim inside a workgroup (1, 2, 4, 8; 0 = default) */
    uint32_t epilogue;      /* dqt_gemm_epilogue */
    uint32_t tile_cols;     /* columns per lane of a wave (CMM/PLAIN/DOT4: 2 or 4; 0 = default 4; 4 needs
                               tile_rows 8 or 16) */
} dqt_gemm_plan;

/*
 * Bytes of device workspace dqt_fgemm needs for (m, n, kdim, plan); 0 when
 * none.  plan == NULL means the default plan for (p, kdim).
 */
size_t dqt_fgemm_workspace_size(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan *plan);

/*
 * F_p matrix product.  plan == NULL: DQT_GEMM_AUTO with defaults.
 * RIGHT / LEFT / FULL: Q is the smallest power of two above kdim (p-1)^2
 * (eq:lower) unless log2Q asks for a larger one, and a word holds
 * floor(52 / log2 Q) digits (at most 8; eq:upper with one spare bit), so
 * every product and partial sum is an integer below 2^52, exact in binary64;
 * DQT_E_UNSUPPORTED when fewer than two digits fit (four for FULL).  ksplit
 * applies; tile_rows, tile_cols, interval and epilogue are ignored.
 * CMM bounds (eq:lower with the interval in place of kdim): interval*(p-1)^2
 * < Q, and (p-1)(Q+1) < 2^16 so that a Kronecker pair fits a 16-bit lane of
 * the packed word.  CMM, PLAIN and DOT4 add whole dot products in uint32, so
 * they need kdim*(p-1)^2 < 2^32 (DQT_E_UNSUPPORTED otherwise, AUTO included);
 * MFMA needs kdim*(p-1)^2 < 2^31 and p <= 128.  d_work: device workspace of at least
 * dqt_fgemm_workspace_size(...) bytes (packed operands), 16-byte aligned
 * (DQT_E_INVALID otherwise); its contents on entry are ignored.
 */
dqt_status dqt_fgemm(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t *d_A, uint64_t lda,
                     const uint8_t *d_B, uint64_t ldb, uint8_t *d_C, uint64_t ldc, const dqt_gemm_plan *plan,
                     void *d_work, size_t work_bytes, void *stream);

/*
 * dqt_fgemm for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it): same arguments and results as dqt_fgemm, without the workspace.
 * The packed operands go to a static device array inside the library, one
 * per GPU, held until the process ends; the call allocates nothing.  Its
 * size is dqt_fgemm_noalloc_max_bytes() (32 MiB): a product whose
 * dqt_fgemm_workspace_size exceeds it gets DQT_E_WORKSPACE, before anything
 * is enqueued.  All calls on one GPU share that array: calls that overlap on
 * one GPU (concurrent streams or threads) race and give undefined results;
 * calls ordered on one stream are safe (nothing needs clearing in between).
 */
dqt_status dqt_fgemm_noalloc(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t *d_A, uint64_t lda,
                             const uint8_t *d_B, uint64_t ldb, uint8_t *d_C, uint64_t ldc, const dqt_gemm_plan *plan,
                             void *stream);
size_t dqt_fgemm_noalloc_max_bytes(void);

/*
 * The two phases of dqt_fgemm on their own (section 7.1: compression,
 * multiplication and extraction; compressed matrices are often reused).
 * dqt_fgemm_pack writes the packed operands of (p, m, n, kdim, plan) into
 * d_work; either d_A or d_B may be NULL to keep the packed copy already in the
 * workspace.  dqt_fgemm_compute multiplies the packed operands in d_work and
 * writes C; it must be given the same (p, m, n, kdim, plan) as the pack call
 * that filled d_work.  dqt_fgemm is the two calls in sequence.
 */
dqt_status dqt_fgemm_pack(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t *d_A, uint64_t lda,
                          const uint8_t *d_B, uint64_t ldb, const dqt_gemm_plan *plan, void *d_work,
                          size_t work_bytes, void *stream);
dqt_status dqt_fgemm_compute(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t *d_C, uint64_t ldc,
                             const dqt_gemm_plan *plan, const void *d_work, size_t work_bytes, void *stream);

/*
 * dqt_fgemm_compute, with the multiply kernel's own start and end recorded
 * into two caller-created hipEvent_t (either may be NULL): the elapsed time
 * between them is that kernel's execution, without the launch gaps around
 * it (measurement).
 */
dqt_status dqt_fgemm_compute_timed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t *d_C, uint64_t ldc,
                                   const dqt_gemm_plan *plan, const void *d_work, size_t work_bytes,
                                   void *start_event, void *stop_event, void *stream);
/* dqt_fgemm (both phases in one call) with the multiply kernel's start and end recorded the same way. */
dqt_status dqt_fgemm_timed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t *d_A, uint64_t lda,
                           const uint8_t *d_B, uint64_t ldb, uint8_t *d_C, uint64_t ldc, const dqt_gemm_plan *plan,
                           void *d_work, size_t work_bytes, void *start_event, void *stop_event, void *stream);

/*
 * One packed operand in a buffer of its own, so that it can stay resident
 * and be multiplied many times (section 7.1: compressed matrices are often
 * reused).  side 0 packs the rows of A (rows_or_cols = m, d_X = A, ldx = lda
 * >= kdim); side 1 packs the columns of B (rows_or_cols = n, d_X = B, ldx =
 * ldb >= n).  The packed layout depends only on (p, kdim, plan) and on the
 * packed dimension, so an A packed with m rows can be multiplied by any packed
 * B with the same (p, kdim, plan).  dqt_fgemm_packed_bytes gives the size of
 * the packed copy (0 for invalid arguments or an unsupported plan); d_packed
 * must be 16-byte aligned and hold that many bytes.  dqt_fgemm_packed
 * multiplies a packed A (m rows) by a packed B (n columns) and writes C; both
 * must come from dqt_fgemm_pack_side with the same p, kdim and plan.
 * DQT_GEMM_BY_SHAPE is refused by these three calls (0 bytes, DQT_E_INVALID):
 * it picks the algorithm from all three dimensions, which one side alone
 * does not know.
 */
size_t dqt_fgemm_packed_bytes(uint32_t p, uint64_t rows_or_cols, uint64_t kdim, int side, const dqt_gemm_plan *plan);
dqt_status dqt_fgemm_pack_side(uint32_t p, uint64_t rows_or_cols, uint64_t kdim, const uint8_t *d_X, uint64_t ldx,
                               int side, const dqt_gemm_plan *plan, void *d_packed, void *stream);
dqt_status dqt_fgemm_packed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const void *d_CA, const void *d_CB,
                            uint8_t *d_C, uint64_t ldc, const dqt_gemm_plan *plan, void *stream);

/*
 * Batched F_p matrix products in one persistent launch.
 *
 * Each descriptor names its own device operands (row-major uint8, as for
 * dqt_fgemm) and its packing choices: algo (DQT_GEMM_AUTO, _CMM, _PLAIN,
 * _DOT4 or _DOT8), interval and log2Q (0 = smallest allowed), epilogue.  These are the
 * knobs the tuner picks per (size, p) bucket.
 *
 * dqt_fgemm_batched_prepare builds the device-resident plan in d_work
 * (descriptors, packed-operand slices, the work-item list sorted by
 * decreasing cost) with one host-to-device copy on `stream`, waits for it,
 * and returns a host handle.  dqt_fgemm_batched_run enqueues the batch:
 * one packing launch over all products, then one persistent launch whose
 * workgroups take (product, tile) items from an atomic counter until none is
 * left.  run reads only d_work and may be called again (or captured in a
 * graph and replayed) as long as the operands and d_work stay valid; calls
 * that share a d_work must not overlap.  dqt_fgemm_batched = prepare + run +
 * free.
 *
 * Resident packed operands (section 7.1: compressed matrices are often
 * reused): run = pack + compute.  dqt_fgemm_batched_pack enqueues only the
 * packing launch, which writes every product's packed copies of A and B into
 * d_work; dqt_fgemm_batched_compute enqueues only the persistent launch (after
 * a one-thread kernel that clears the item counter), which reads the packed
 * copies left in d_work by the last run or pack of this batch.  The caller
 * calls pack (or run) again after changing any operand; compute alone on
 * operands changed since then gives the products of the old operands.  Both
 * may be captured in a graph; DQT_E_INVALID for a null handle.
 */
typedef struct dqt_gemm_desc {
    const uint8_t *A;
    const uint8_t *B;
    uint8_t *C;
    uint32_t m, n, kdim;
    uint32_t lda, ldb, ldc;
    uint32_t p;
    uint32_t algo;          /* DQT_GEMM_AUTO, DQT_GEMM_CMM, DQT_GEMM_PLAIN, DQT_GEMM_DOT4 or DQT_GEMM_DOT8 */
    uint32_t interval;      /* delayed-reduction interval in k (0 = largest allowed) */
    uint32_t log2Q;         /* 0 = smallest allowed */
    uint32_t epilogue;      /* dqt_gemm_epilogue */
} dqt_gemm_desc;

typedef struct dqt_batch_opts {
    uint32_t tile_rows;     /* 8 or 16 (0 = 16) */
    uint32_t ksplit;        /* 2, 4 or 8 waves per workgroup (0 = 4); 8 not with 16 rows and 4 columns */
    uint32_t tile_cols;     /* columns per lane, 2 or 4 (0 = 2) */
} dqt_batch_opts;

typedef struct dqt_batch dqt_batch;   /* opaque host handle */

size_t dqt_fgemm_batched_workspace_size(const dqt_gemm_desc *descs, uint32_t count, const dqt_batch_opts *opts);
dqt_status dqt_fgemm_batched_prepare(const dqt_gemm_desc *descs, uint32_t count, const dqt_batch_opts *opts,
                                     void *d_work, size_t work_bytes, void *stream, dqt_batch **out);
dqt_status dqt_fgemm_batched_run(const dqt_batch *batch, void *stream);
dqt_status dqt_fgemm_batched_pack(const dqt_batch *batch, void *stream);
dqt_status dqt_fgemm_batched_compute(const dqt_batch *batch, void *stream);
void dqt_batch_free(dqt_batch *batch);
dqt_status dqt_fgemm_batched(const dqt_gemm_desc *descs, uint32_t count, const dqt_batch_opts *opts,
                             void *d_work, size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DQT_H */
