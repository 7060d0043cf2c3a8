/*
 * Plain CPU oracle for the packed-DQT / REDQ hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library and never calls into it.
 *
 * Every function below is the plain definition of what the packed path
 * computes, written out with a reduction modulo p after every multiply and
 * every add (the "reduce after every operation" schoolbook).  Nothing is
 * blocked, fused, packed or reordered.  Values are canonical residues in
 * [0, p); every result is unique, so comparisons against it are bit-exact.
 *
 * Paper: Dumas, Fousse, Salvy, "Simultaneous Modular Reduction and Kronecker
 * Substitution for Small Finite Fields".
 */
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint32_t add_mod(uint32_t x, uint32_t y, uint32_t p) { return (x + y) % p; }
static inline uint32_t mul_mod(uint32_t x, uint32_t y, uint32_t p) { return (x * y) % p; }
static inline uint32_t sub_mod(uint32_t x, uint32_t y, uint32_t p) { return (x + p - (y % p)) % p; }

/* nthreads > 0: that many threads for this call; 0: the process default (the
   OpenMP maximum seen at the first call), also after a call that asked for
   fewer. */
static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    static int32_t default_threads = 0;
    if (default_threads == 0) default_threads = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : default_threads);
#else
    (void)nthreads;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Polynomial product over F_p (section 2.1, equation eq:mult, with the
 * final "mod p" of the DQT dot-product algorithm, section 2.3):
 *   c_j = sum_{i} a_i * b_{j-i}  mod p,   j = 0 .. ka+kb-2.
 * a: [count][ka], b: [count][kb], out: [count][ka+kb-1]; coefficient i of a
 * polynomial is its X^i coefficient (low degree first).  All output
 * coefficients are written, zeros included.
 */
void orc_polymul(const uint8_t *a, int32_t ka, const uint8_t *b, int32_t kb,
                 int64_t count, int32_t p, uint8_t *out, int32_t nthreads)
{
    const int32_t kc = ka + kb - 1;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        const uint8_t *x = a + t * ka;
        const uint8_t *y = b + t * kb;
        uint8_t *z = out + t * kc;
        for (int32_t j = 0; j < kc; ++j) {
            uint32_t c = 0;
            for (int32_t i = 0; i < ka; ++i) {
                int32_t l = j - i;
                if (l < 0 || l >= kb) continue;
                c = add_mod(c, mul_mod(x[i] % p, y[l] % p, p), p);
            }
            z[j] = (uint8_t)c;
        }
    }
}

/*
 * Matrix product over F_p (section 7.1): C_ij = sum_l A_il * B_lj mod p.
 * Row-major with leading dimensions lda, ldb, ldc (in elements).
 */
void orc_fgemm(const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
               uint8_t *C, int64_t ldc, int64_t m, int64_t n, int64_t kdim,
               int32_t p, int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            uint32_t c = 0;
            for (int64_t l = 0; l < kdim; ++l)
                c = add_mod(c, mul_mod(A[i * lda + l] % p, B[l * ldb + j] % p, p), p);
            C[i * ldc + j] = (uint8_t)c;
        }
    }
}

/*
 * Selected entries of the same product, one by one: out[s] = C[rows[s], cols[s]].
 * Used to check outputs at sizes where the full product is too slow.
 */
void orc_fgemm_entries(const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                       int64_t kdim, int32_t p, const int64_t *rows, const int64_t *cols,
                       int64_t nsamp, uint8_t *out, int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsamp; ++s) {
        uint32_t c = 0;
        for (int64_t l = 0; l < kdim; ++l)
            c = add_mod(c, mul_mod(A[rows[s] * lda + l] % p, B[l * ldb + cols[s]] % p, p), p);
        out[s] = (uint8_t)c;
    }
}

/*
 * Multiplication in GF(p^k) = F_p[X]/(P) (section 6): the polynomial product
 * of two elements of degree < k, then long division by the monic modulus P
 * of degree k, from the top coefficient down, reducing mod p after every
 * operation.  modulus: k+1 coefficients, low degree first, modulus[k] == 1.
 * a, b: [count][k]; out: [count][k].
 */
void orc_gf_mul(const uint8_t *a, const uint8_t *b, int64_t count, int32_t k,
                int32_t p, const uint8_t *modulus, uint8_t *out, int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        uint32_t r[2 * 16];
        const uint8_t *x = a + t * k;
        const uint8_t *y = b + t * k;
        for (int32_t j = 0; j < 2 * k - 1; ++j) {
            uint32_t c = 0;
            for (int32_t i = 0; i < k; ++i) {
                int32_t l = j - i;
                if (l < 0 || l >= k) continue;
                c = add_mod(c, mul_mod(x[i] % p, y[l] % p, p), p);
            }
            r[j] = c;
        }
        /* Long division: eliminate X^j for j = 2k-2 down to k. */
        for (int32_t j = 2 * k - 2; j >= k; --j) {
            uint32_t lead = r[j];
            if (lead == 0) continue;
            for (int32_t i = 0; i <= k; ++i)
                r[j - k + i] = sub_mod(r[j - k + i], mul_mod(lead, modulus[i] % p, p), p);
        }
        for (int32_t i = 0; i < k; ++i) out[t * k + i] = (uint8_t)r[i];
    }
}

/*
 * Inverse DQT of one machine word (REDQ's specification, section 3.2): with
 * q = 2^logq and r = sum_{i=0}^{nres-1} m_i q^i where every m_i < q except
 * possibly the top one, return m_i mod p.  The digits are read by plain
 * radix conversion (division and remainder by q), the top digit is
 * everything above the nres-1 lower ones.  out: [count][nres].
 */
void orc_radix_mod(const uint64_t *r, int64_t count, int32_t p, int32_t logq,
                   int32_t nres, uint8_t *out, int32_t nthreads)
{
    const uint64_t q = (uint64_t)1 << logq;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        uint64_t v = r[t];
        for (int32_t i = 0; i < nres - 1; ++i) {
            out[t * nres + i] = (uint8_t)((v % q) % (uint64_t)p);
            v /= q;
        }
        out[t * nres + nres - 1] = (uint8_t)(v % (uint64_t)p);
    }
}

/* Euclidean quotient floor(r / p) (section 4.2, the value FDIV approximates). */
void orc_floor_div(const uint64_t *r, int64_t count, uint64_t p, uint64_t *out)
{
    for (int64_t t = 0; t < count; ++t) out[t] = r[t] / p;
}

/* Evaluation at q = 2^logq (equation eq:dqt), Horner from the top:
 * words[t] = sum_i c[t][i] q^i, or, when reverse != 0, sum_i c[t][i] q^(k-1-i).
 * Overflow beyond 64 bits is the caller's responsibility (wraps mod 2^64). */
void orc_dqt_eval(const uint8_t *c, int64_t count, int32_t k, int32_t logq,
                  int32_t reverse, uint64_t *words)
{
    const uint64_t q = (uint64_t)1 << logq;
    for (int64_t t = 0; t < count; ++t) {
        uint64_t v = 0;
        for (int32_t i = 0; i < k; ++i) {
            int32_t idx = reverse ? i : (k - 1 - i);
            v = v * q + c[t * k + idx];
        }
        words[t] = v;
    }
}
