// Dot products over GF(p^k) by algorithm FGDP (section 6 of the paper).
//
// R = sum_l a_l b_l in GF(p^k) = F_p[X]/(P).  The products of up to n_q pairs
// are summed in packed form (one 64-bit word, the "floating point
// computation" of FGDP done here with exact integers): with
// q > n_q k (p-1)^2 no digit of the sum reaches q (eq:bounds) and
// (2k-1) log2 q <= 53 keeps the word exact for REDQ's binary64 floor.  Each
// word is then compressed once (REDQ compression), its residues u_0..u_{k-1}
// and u_{k-1}..u_{2k-2} index the two tables T_L and T_H (theorem thm:fgdp,
// built per workgroup in LDS), and H + L is added to the running result in
// the field, coefficient-wise mod p.

#include <string.h>

#include "dqt_internal.h"

namespace dqt {

template <int K>
__device__ void build_gf_tables_dot(uint64_t* tl, uint64_t* th, const RedqArgs& ra, const GfArgs& ga) {
    const uint32_t wm = (1u << ra.w) - 1u;
    const uint32_t n = 1u << (K * ra.w);
    for (uint32_t idx = threadIdx.x; idx < n; idx += blockDim.x) {
        uint32_t u[K];
#pragma unroll
        for (int j = 0; j < K; ++j) u[j] = (idx >> (j * ra.w)) & wm;
        uint64_t lo = 0;
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
            const uint32_t mu = ra.c ? correct_arith(u[i], u[i + 1], ra) : mod_small(u[i], ra.p, ra.pmagic);
            lo |= (uint64_t)mu << (8 * i);
        }
        tl[idx] = lo;
        uint32_t mu[K];
#pragma unroll
        for (int j = 0; j < K; ++j)
            mu[j] = (j + 1 < K && ra.c) ? correct_arith(u[j], u[j + 1], ra) : mod_small(u[j], ra.p, ra.pmagic);
        uint64_t hi = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            uint32_t acc = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) acc += mu[j] * (uint32_t)((ga.xpow[j] >> (8 * i)) & 0xFF);
            hi |= (uint64_t)mod_small(acc, ra.p, ra.pmagic) << (8 * i);
        }
        th[idx] = hi;
    }
}

// a + b coefficient-wise mod p on K byte lanes (each lane < p).
__device__ __forceinline__ uint64_t add_mod_bytes(uint64_t a, uint64_t b, uint32_t p, uint64_t ones) {
    const uint64_t s = a + b;
    const uint64_t t = s + (uint64_t)(128 - p) * ones;
    const uint64_t ge = (t >> 7) & ones;
    return s - (uint64_t)p * ge;
}

// Eight consecutive records (8 K bytes) of an operand at any byte address:
// K unaligned 8-byte loads (global memory takes them), or, for a chunk cut by
// the end of the dot product, byte loads of its first `bytes` bytes only.
template <int K>
__device__ __forceinline__ void load_chunk(const uint8_t* src, uint32_t bytes, uint64_t (&w)[K]) {
    if (bytes == 8 * K) {
#pragma unroll
        for (int i = 0; i < K; ++i) __builtin_memcpy(&w[i], src + 8 * i, 8);
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) w[i] = 0;
        for (uint32_t x = 0; x < bytes; ++x) w[x >> 3] |= (uint64_t)src[x] << (8 * (x & 7));
    }
}

// Record r of a chunk (bytes r K .. r K + K - 1) spread into fields of B bits:
// sum_i e_i 2^(B i), below 2^32 for every K here (B (K-1) + 7 <= 28).
template <int K, int B, int R>
__device__ __forceinline__ uint32_t record_word(const uint64_t (&w)[K]) {
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int byte = R * K + i;
        const uint64_t word = w[byte >> 3];
        const uint32_t half = (byte & 7) < 4 ? (uint32_t)word : (uint32_t)(word >> 32);
        v |= ((half >> (8 * (byte & 3))) & 0xFFu) << (B * i);
    }
    return v;
}

// The K residues mod p of a running sum held in 16-bit lanes (RE: coefficients
// 0, 2, 4; RO: 1, 3, 5), as K bytes.
template <int K>
__device__ __forceinline__ uint64_t fold16(uint64_t RE, uint64_t RO, uint32_t p, uint32_t pmagic) {
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t v = (uint32_t)(((i & 1) ? RO : RE) >> (16 * (i >> 1))) & 0xFFFFu;
        r |= (uint64_t)mod_small(v, p, pmagic) << (8 * i);
    }
    return r;
}

// G lanes share one dot product.  The n pairs are taken in chunks of eight
// consecutive records; lane g of a group takes chunks g, g + G, ..., so the G
// lanes of a group read G consecutive runs of 8 K bytes of each operand (8-byte
// loads, coalesced across the group).  Each lane keeps its own packed sums of
// n_q products (q = 2^B, B = floor(53 / (2K - 1)), so a record packs into one
// 32-bit word and a product of two is one 32 x 32 -> 64-bit multiply-add).
// After each REDQ the two table values (each coefficient below p) are added
// without reduction into 16-bit lanes, folded mod p every fold_at reductions
// and at the end; the G lane results are added in the field across the group
// by shuffles.  NQ1: n_q = 1 (every product is reduced on its own).
template <int K, int G, bool NQ1>
__global__ __launch_bounds__(256) void k_gf_dot(const uint8_t* __restrict__ A, const uint8_t* __restrict__ Bop,
                                                uint8_t* __restrict__ OUT, uint64_t count, uint32_t n, uint32_t nq,
                                                RedqArgs ra, GfArgs ga) {
    constexpr int B = 53 / (2 * K - 1);
    extern __shared__ uint64_t gfd_smem[];
    const uint32_t tn = 1u << (K * ra.w);
    uint64_t* tl = gfd_smem;
    uint64_t* th = gfd_smem + tn;
    build_gf_tables_dot<K>(tl, th, ra, ga);
    __syncthreads();
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    constexpr uint64_t kEven = 0x00FF00FF00FF00FFull;
    const uint32_t wm = (1u << ra.w) - 1u;
    const uint32_t fold_at = 65535u / (2u * (ra.p - 1u));   // table sums per 16-bit lane before a fold
    const uint32_t g = threadIdx.x % G;
    const uint64_t groups = (uint64_t)gridDim.x * (256 / G);
    const uint32_t nch = (n + 7) / 8;
    // every lane of a group runs the same number of outer iterations (the
    // shuffles below need the whole wave), so the loop runs to the padded count
    const uint64_t padded = (count + groups - 1) / groups * groups;
    for (uint64_t t = (uint64_t)blockIdx.x * (256 / G) + threadIdx.x / G; t < padded; t += groups) {
        const bool live = t < count;
        const uint8_t* x = A + (live ? t : 0) * (uint64_t)n * K;
        const uint8_t* y = Bop + (live ? t : 0) * (uint64_t)n * K;
        uint64_t R = 0, RE = 0, RO = 0, acc = 0;
        uint32_t cnt = 0, nred = 0;
        auto reduce = [&]() {
            const uint64_t U = redq_compress(acc, ra);
            const uint32_t xl = (uint32_t)U;
            const uint64_t xh64 = U >> (B * (K - 1));
            const uint32_t xh = (uint32_t)xh64;   // B K <= 32 bits hold the top K fields
            uint32_t il = 0, ih = 0;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                il |= __builtin_amdgcn_ubfe(xl, B * jj, ra.w) << (ra.w * jj);
                ih |= __builtin_amdgcn_ubfe(xh, B * jj, ra.w) << (ra.w * jj);
            }
            const uint64_t sum = th[ih] + tl[il];   // bytes below 2p - 1
            RE += sum & kEven;
            RO += (sum >> 8) & kEven;
            acc = 0;
            cnt = 0;
            if (++nred == fold_at) {
                R = add_mod_bytes(R, fold16<K>(RE, RO, ra.p, ra.pmagic), ra.p, ones);
                RE = RO = 0;
                nred = 0;
            }
        };
        auto pair = [&](uint32_t xa, uint32_t yb) {
            acc += (uint64_t)xa * yb;
            if (NQ1) reduce();
            else if (++cnt == nq) reduce();
        };
        // whole chunks of eight records
        const uint32_t nfull = n / 8;
        for (uint32_t c = live ? g : nfull; c < nfull; c += G) {
            uint64_t wa[K], wb[K];
            load_chunk<K>(x + (uint64_t)c * 8 * K, 8 * K, wa);
            load_chunk<K>(y + (uint64_t)c * 8 * K, 8 * K, wb);
            pair(record_word<K, B, 0>(wa), record_word<K, B, 0>(wb));
            pair(record_word<K, B, 1>(wa), record_word<K, B, 1>(wb));
            pair(record_word<K, B, 2>(wa), record_word<K, B, 2>(wb));
            pair(record_word<K, B, 3>(wa), record_word<K, B, 3>(wb));
            pair(record_word<K, B, 4>(wa), record_word<K, B, 4>(wb));
            pair(record_word<K, B, 5>(wa), record_word<K, B, 5>(wb));
            pair(record_word<K, B, 6>(wa), record_word<K, B, 6>(wb));
            pair(record_word<K, B, 7>(wa), record_word<K, B, 7>(wb));
        }
        // the last n mod 8 records (chunk nfull), on the lane that chunk falls to
        const uint32_t nrec = n - 8 * nfull;
        if (live && nrec && nfull % G == g) {
            uint64_t wa[K], wb[K];
            load_chunk<K>(x + (uint64_t)nfull * 8 * K, nrec * K, wa);
            load_chunk<K>(y + (uint64_t)nfull * 8 * K, nrec * K, wb);
            for (uint32_t r = 0; r < nrec; ++r) {
                // record r from the chunk, shifted down by r K bytes
                uint32_t xa = 0, yb = 0;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const uint32_t byte = r * K + i;
                    xa |= (uint32_t)((wa[byte >> 3] >> (8 * (byte & 7))) & 0xFFu) << (B * i);
                    yb |= (uint32_t)((wb[byte >> 3] >> (8 * (byte & 7))) & 0xFFu) << (B * i);
                }
                pair(xa, yb);
            }
        }
        if (!NQ1 && cnt) reduce();
        R = add_mod_bytes(R, fold16<K>(RE, RO, ra.p, ra.pmagic), ra.p, ones);
#pragma unroll
        for (int off = G / 2; off >= 1; off /= 2) {
            const uint32_t lo = __shfl_xor((uint32_t)R, off, G);
            const uint32_t hi = __shfl_xor((uint32_t)(R >> 32), off, G);
            R = add_mod_bytes(R, ((uint64_t)hi << 32) | lo, ra.p, ones);
        }
        if (live && g == 0) {
#pragma unroll
            for (int i = 0; i < K; ++i) OUT[t * K + i] = (uint8_t)(R >> (8 * i));
        }
    }
}

template <int K, int G>
static void launch_gf_dot_g(const uint8_t* A, const uint8_t* B, uint8_t* out, uint64_t count, uint32_t n,
                            uint32_t nq, const RedqArgs& ra, const GfArgs& ga, hipStream_t s) {
    const size_t smem = 2ull * (1ull << (K * ra.w)) * sizeof(uint64_t);
    const unsigned grid = stream_grid(count * G, 256, 4);
    if (nq == 1)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_dot<K, G, true>), dim3(grid), dim3(256), smem, s, A, B, out, count, n,
                           nq, ra, ga);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_dot<K, G, false>), dim3(grid), dim3(256), smem, s, A, B, out, count,
                           n, nq, ra, ga);
}

// Lanes per dot product: about one per four chunks of eight records, at most a wave (with one
// chunk per lane, the combining of the lanes' sums and the fold cost more than they spread:
// 65,536 dot products of 128 elements over GF(3^5) took 33 us on 16 lanes each, 30 us on 4).
template <int K>
static dqt_status launch_gf_dot(const uint8_t* A, const uint8_t* B, uint8_t* out, uint64_t count, uint32_t n,
                                uint32_t nq, const RedqArgs& ra, const GfArgs& ga, hipStream_t s) {
    const uint32_t nch = (n + 7) / 8;
    if (nch > 64) launch_gf_dot_g<K, 64>(A, B, out, count, n, nq, ra, ga, s);
    else if (nch > 16) launch_gf_dot_g<K, 16>(A, B, out, count, n, nq, ra, ga, s);
    else if (nch > 2) launch_gf_dot_g<K, 4>(A, B, out, count, n, nq, ra, ga, s);
    else launch_gf_dot_g<K, 1>(A, B, out, count, n, nq, ra, ga, s);
    DQT_LAUNCH_CHECK("dqt_gf_dot_u8");
    return DQT_OK;
}

// Matrix products over GF(p^k) by FGDP: C[i][j] = sum_l A[i][l] B[l][j], each
// entry a dot product of packed field elements (section 6).  A workgroup of 256
// threads takes a 16 TR x 16 TC tile of C, a thread TR rows x TC columns of it
// (4 x 2 where the grid has enough tiles, down to 1 x 1 for small products, so
// that every SIMD gets waves: each product costs a reduction, there is little to
// share between the outputs of a thread); A and B pass through LDS in steps of
// 16 along l, each element packed once into a 32-bit word with fields of B bits
// (the same q = 2^B as the dot products).  Every output of a thread receives
// one product per step of l, so the packed sums of all of them reach n_q
// together and are reduced together (REDQ, the two tables, the sums in 16-bit
// lanes as in k_gf_dot).
constexpr int kGmRows = 64, kGmCols = 32, kGmK = 16;   // the largest tile

template <int K>
__device__ __forceinline__ uint32_t element_word(const uint8_t* e) {
    constexpr int B = 53 / (2 * K - 1);
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) v |= (uint32_t)e[i] << (B * i);
    return v;
}

template <int K, bool NQ1, int TR, int TC>
__global__ __launch_bounds__(256) void k_gf_matmul(const uint8_t* __restrict__ A, const uint8_t* __restrict__ Bm,
                                                   uint8_t* __restrict__ OUT, uint32_t m, uint32_t n, uint32_t kd,
                                                   uint32_t nq, RedqArgs ra, GfArgs ga) {
    constexpr int B = 53 / (2 * K - 1);
    constexpr int ROWS = 16 * TR, COLS = 16 * TC;
    extern __shared__ uint64_t gfm_smem[];
    const uint32_t tn = 1u << (K * ra.w);
    uint64_t* tl = gfm_smem;
    uint64_t* th = gfm_smem + tn;
    uint32_t* la = reinterpret_cast<uint32_t*>(gfm_smem + 2 * tn);   // [kGmK][ROWS]
    uint32_t* lb = la + kGmK * ROWS;                                   // [kGmK][COLS]
    build_gf_tables_dot<K>(tl, th, ra, ga);
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    constexpr uint64_t kEven = 0x00FF00FF00FF00FFull;
    const uint32_t wm = (1u << ra.w) - 1u;
    const uint32_t fold_at = 65535u / (2u * (ra.p - 1u));
    const uint32_t tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    const uint32_t row0 = blockIdx.y * ROWS, col0 = blockIdx.x * COLS;
    uint64_t acc[TR][TC], RE[TR][TC], RO[TR][TC], R[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = RE[i][j] = RO[i][j] = R[i][j] = 0;
    uint32_t cnt = 0, nred = 0;
    auto reduce = [&]() {
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                const uint64_t U = redq_compress(acc[i][j], ra);
                const uint32_t xl = (uint32_t)U, xh = (uint32_t)(U >> (B * (K - 1)));
                uint32_t il = 0, ih = 0;
#pragma unroll
                for (int jj = 0; jj < K; ++jj) {
                    il |= __builtin_amdgcn_ubfe(xl, B * jj, ra.w) << (ra.w * jj);
                    ih |= __builtin_amdgcn_ubfe(xh, B * jj, ra.w) << (ra.w * jj);
                }
                const uint64_t sum = th[ih] + tl[il];   // bytes below 2p - 1
                RE[i][j] += sum & kEven;
                RO[i][j] += (sum >> 8) & kEven;
                acc[i][j] = 0;
            }
        cnt = 0;
        if (++nred == fold_at) {
#pragma unroll
            for (int i = 0; i < TR; ++i)
#pragma unroll
                for (int j = 0; j < TC; ++j) {
                    R[i][j] = add_mod_bytes(R[i][j], fold16<K>(RE[i][j], RO[i][j], ra.p, ra.pmagic), ra.p, ones);
                    RE[i][j] = RO[i][j] = 0;
                }
            nred = 0;
        }
    };
    for (uint32_t k0 = 0; k0 < kd; k0 += kGmK) {
        __syncthreads();   // the tables are built / the previous step's words are used
        for (uint32_t e = tid; e < ROWS * kGmK; e += 256) {
            const uint32_t r = e / kGmK, kk = e % kGmK;
            const uint32_t row = row0 + r, l = k0 + kk;
            la[kk * ROWS + r] = row < m && l < kd ? element_word<K>(A + ((uint64_t)row * kd + l) * K) : 0u;
        }
        for (uint32_t e = tid; e < COLS * kGmK; e += 256) {
            const uint32_t kk = e / COLS, c = e % COLS;
            const uint32_t col = col0 + c, l = k0 + kk;
            lb[kk * COLS + c] = col < n && l < kd ? element_word<K>(Bm + ((uint64_t)l * n + col) * K) : 0u;
        }
        __syncthreads();
        const uint32_t steps = min((uint32_t)kGmK, kd - k0);
        for (uint32_t kk = 0; kk < steps; ++kk) {
            uint32_t av[TR], bv[TC];
#pragma unroll
            for (int i = 0; i < TR; ++i) av[i] = la[kk * ROWS + ty * TR + i];
#pragma unroll
            for (int j = 0; j < TC; ++j) bv[j] = lb[kk * COLS + tx * TC + j];
#pragma unroll
            for (int i = 0; i < TR; ++i)
#pragma unroll
                for (int j = 0; j < TC; ++j) acc[i][j] += (uint64_t)av[i] * bv[j];
            if (NQ1 || ++cnt == nq) reduce();
        }
    }
    if (!NQ1 && cnt) reduce();
#pragma unroll
    for (int i = 0; i < TR; ++i) {
        const uint32_t row = row0 + ty * TR + i;
        if (row >= m) continue;
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            const uint32_t col = col0 + tx * TC + j;
            if (col >= n) continue;
            const uint64_t r = add_mod_bytes(R[i][j], fold16<K>(RE[i][j], RO[i][j], ra.p, ra.pmagic), ra.p, ones);
            uint8_t* o = OUT + ((uint64_t)row * n + col) * K;
#pragma unroll
            for (int t = 0; t < K; ++t) o[t] = (uint8_t)(r >> (8 * t));
        }
    }
}

template <int K, int TR, int TC>
static void launch_gf_matmul_tile(const uint8_t* A, const uint8_t* B, uint8_t* out, uint32_t m, uint32_t n,
                                  uint32_t kd, uint32_t nq, const RedqArgs& ra, const GfArgs& ga, hipStream_t s) {
    const size_t smem = 2ull * (1ull << (K * ra.w)) * sizeof(uint64_t) + (size_t)kGmK * 16 * (TR + TC) * 4;
    const dim3 grid((n + 16 * TC - 1) / (16 * TC), (m + 16 * TR - 1) / (16 * TR));
    if (nq == 1)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_matmul<K, true, TR, TC>), grid, dim3(256), smem, s, A, B, out, m, n,
                           kd, nq, ra, ga);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_matmul<K, false, TR, TC>), grid, dim3(256), smem, s, A, B, out, m, n,
                           kd, nq, ra, ga);
}

template <int K>
static dqt_status launch_gf_matmul(const uint8_t* A, const uint8_t* B, uint8_t* out, uint32_t m, uint32_t n,
                                   uint32_t kd, uint32_t nq, const RedqArgs& ra, const GfArgs& ga, hipStream_t s) {
    // the largest tile per thread whose grid still has kGmWantTiles workgroups (about four
    // waves per SIMD); the smaller tiles only where the larger ones leave SIMDs idle, so
    // their grids stay below the largest tile's row limit times four
    constexpr uint64_t kGmWantTiles = 1024;
    auto tiles = [&](uint32_t rows, uint32_t cols) {
        return (uint64_t)((n + cols - 1) / cols) * ((m + rows - 1) / rows);
    };
    if (tiles(64, 32) >= kGmWantTiles) launch_gf_matmul_tile<K, 4, 2>(A, B, out, m, n, kd, nq, ra, ga, s);
    else if (tiles(32, 32) >= kGmWantTiles) launch_gf_matmul_tile<K, 2, 2>(A, B, out, m, n, kd, nq, ra, ga, s);
    else if (tiles(32, 16) >= kGmWantTiles) launch_gf_matmul_tile<K, 2, 1>(A, B, out, m, n, kd, nq, ra, ga, s);
    else launch_gf_matmul_tile<K, 1, 1>(A, B, out, m, n, kd, nq, ra, ga, s);
    DQT_LAUNCH_CHECK("dqt_gf_matmul_u8");
    return DQT_OK;
}

// FGDP's parameters for sums of up to `len` products: q = 2^b with b = 53 / (2k - 1)
// (the kernels' compile-time B), n_q = floor((q - 1) / (k (p - 1)^2)) capped at len.
static dqt_status fgdp_setup(uint32_t k, uint32_t p, const uint8_t* modulus, uint64_t len, GfArgs* ga, RedqArgs* ra,
                             uint32_t* nq) {
    if (p < 2 || p > 127 || k < 2 || k > 6 || !modulus) return DQT_E_INVALID;
    DQT_TRY(gf_setup_args(k, p, modulus, ga));
    const uint32_t w = residue_bits(p);
    if (k * w > 12) return DQT_E_UNSUPPORTED;
    const uint32_t b = 53 / (2 * k - 1);
    if (b < w) return DQT_E_UNSUPPORTED;
    const uint64_t per = (uint64_t)k * (p - 1) * (p - 1);
    const uint64_t nq64 = per ? (((1ull << b) - 1) / per) : len;
    if (nq64 < 1) return DQT_E_UNSUPPORTED;   // not even one product fits a word
    *nq = (uint32_t)(nq64 > len ? (len ? len : 1) : nq64);
    if (b * (k - 1) + w > 32) return DQT_E_UNSUPPORTED;  // table indices gathered from 32-bit windows
    return make_redq_args(p, b, 2 * k - 1, (2 * k - 1) * b, ra);
}

}  // namespace dqt

using namespace dqt;

extern "C" dqt_status dqt_gf_dot_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t n, uint32_t k,
                                    uint32_t p, const uint8_t* modulus, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 127 || k < 2 || k > 6 || n < 1 || !modulus) return DQT_E_INVALID;
    GfArgs ga;
    DQT_TRY(gf_setup_args(k, p, modulus, &ga));
    const uint32_t w = residue_bits(p);
    if (k * w > 12) return DQT_E_UNSUPPORTED;
    // the largest q with (2k-1) log2 q <= 53 (and each residue field within a digit)
    // (the kernels take b as the compile-time 53 / (2k - 1): 17, 10, 7, 5, 4 for k = 2..6)
    const uint32_t b = 53 / (2 * k - 1);
    if (b < w) return DQT_E_UNSUPPORTED;
    const uint64_t per = (uint64_t)k * (p - 1) * (p - 1);
    const uint64_t nq64 = per ? (((1ull << b) - 1) / per) : n;
    if (nq64 < 1) return DQT_E_UNSUPPORTED;   // not even one product fits a word
    const uint32_t nq = nq64 > n ? n : (uint32_t)nq64;
    if (b * (k - 1) + w > 32) return DQT_E_UNSUPPORTED;  // table indices gathered from 32-bit windows
    RedqArgs ra;
    DQT_TRY(make_redq_args(p, b, 2 * k - 1, (2 * k - 1) * b, &ra));
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, (uint64_t)n * k, (uint64_t)n * k}, {d_b, count, (uint64_t)n * k, (uint64_t)n * k}}));
    switch (k) {
        case 2: return launch_gf_dot<2>(d_a, d_b, d_out, count, n, nq, ra, ga, s);
        case 3: return launch_gf_dot<3>(d_a, d_b, d_out, count, n, nq, ra, ga, s);
        case 4: return launch_gf_dot<4>(d_a, d_b, d_out, count, n, nq, ra, ga, s);
        case 5: return launch_gf_dot<5>(d_a, d_b, d_out, count, n, nq, ra, ga, s);
        default: return launch_gf_dot<6>(d_a, d_b, d_out, count, n, nq, ra, ga, s);
    }
}

extern "C" dqt_status dqt_gf_matmul_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t m, uint64_t n, uint64_t kd,
                                       uint32_t k, uint32_t p, const uint8_t* modulus, uint8_t* d_out, void* stream) {
    if (m > 0x7FFFFFFFull || n > 0x7FFFFFFFull || kd > 0x7FFFFFFFull) return DQT_E_INVALID;
    GfArgs ga;
    RedqArgs ra;
    uint32_t nq = 0;
    DQT_TRY(fgdp_setup(k, p, modulus, kd, &ga, &ra, &nq));
    // the two tables and the tiles share 64 KiB of LDS
    if (2ull * (1ull << (k * ra.w)) * 8 + (size_t)kGmK * (kGmRows + kGmCols) * 4 > 65536) return DQT_E_UNSUPPORTED;
    if ((m + kGmRows - 1) / kGmRows > 65535) return DQT_E_UNSUPPORTED;   // row tiles on the grid's y axis
    if (m == 0 || n == 0) return DQT_OK;
    if ((kd && (!d_a || !d_b)) || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (kd) DQT_TRY(debug_gate(s, p, {{d_a, m, kd * k, kd * k}, {d_b, kd, n * k, n * k}}));
    switch (k) {
        case 2: return launch_gf_matmul<2>(d_a, d_b, d_out, (uint32_t)m, (uint32_t)n, (uint32_t)kd, nq, ra, ga, s);
        case 3: return launch_gf_matmul<3>(d_a, d_b, d_out, (uint32_t)m, (uint32_t)n, (uint32_t)kd, nq, ra, ga, s);
        case 4: return launch_gf_matmul<4>(d_a, d_b, d_out, (uint32_t)m, (uint32_t)n, (uint32_t)kd, nq, ra, ga, s);
        case 5: return launch_gf_matmul<5>(d_a, d_b, d_out, (uint32_t)m, (uint32_t)n, (uint32_t)kd, nq, ra, ga, s);
        default: return launch_gf_matmul<6>(d_a, d_b, d_out, (uint32_t)m, (uint32_t)n, (uint32_t)kd, nq, ra, ga, s);
    }
}
