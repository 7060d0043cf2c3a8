// Right, Left and Full compressed F_p matrix products on the FP64 matrix cores
// (section 7.4 "Right or Left Compressed Matrix Multiplication" and section
// 7.5 "Full Compression" of the paper).
//
// Right compression packs e consecutive columns of B into one word,
// CB[l][j'] = sum_t B[l][e j' + t] Q^t, and multiplies the uncompressed A by
// it: CC[i][j'] = sum_t (sum_l A[i][l] B[l][e j' + t]) Q^t, whose e digits are
// the dot products of e outputs; one REDQ_e per word recovers all of them
// (eq:LeftComp: A = Uncompress(CA); CC = A x CB; REDQ(CC)).  Left compression
// is the transpose: e consecutive rows of A per word, B uncompressed.  Full
// compression packs both: e_r rows of A in powers of Q and e_c columns of B in
// powers of Theta = Q^(e_r) (eq:qtheta with equality), so that a word of CC
// holds e_r e_c digits Q^(s + e_r t) (eq:dq).
//
// Exactness: every digit of CC is a dot product of length k bounded by
// k (p-1)^2 < Q (eq:lower), so no digit carries, and the words stay below
// Q^(e_r e_c) <= 2^52 (eq:upper with beta = 53 and one spare bit): every
// product and every partial sum is an integer below 2^52, exact in binary64
// in any order of summation, so the FP64 matrix cores compute CC exactly.
//
// On MI355X the FP64 matrix cores (v_mfma_f64_16x16x4_f64, 1024 multiply-adds
// per instruction) issue far fewer instructions per multiply-add than the
// vector units, and each multiply-add here carries e_r e_c F_p multiply-adds.
//
// Device layouts (workspace), Full:
//   Ad: [Mw_pad/16][K_pad/4][64] binary64, lane l of a 16x4 block holding
//       word row l%16 at k = l/16 (the matrix-core A operand layout);
//   Bd: [Nw_pad/16][K_pad/4][64] binary64, lane l holding k = l/16 of word
//       column l%16 (the B operand layout).
// Right (A uncompressed): A stays uint8, copied to [Mw_pad][K_pad] with zero
// padding (K_pad a multiple of 16), and converted to binary64 in registers;
// inside each group of 16 k the matrix-core steps take k = 4g + s (step s,
// lane group g = l/16), so that lane l reads the four A entries of its four
// steps as one dword.  Bd: [Nw_pad/16][K_pad/16][4][64] binary64, step s of
// group c, lane l holding k = 16c + 4(l/16) + s of word column l%16.
// Left runs the same kernel on the transpose, C^T = B^T A^T: B^T as the
// uint8 operand ([N_pad][K_pad], in the B half of the workspace) and the
// words of e rows of A in the step layout (in the A half).
// The accumulator of a 16x16 block holds, in lane l and element r, word row
// l/16 + 4r and word column l%16.

#include <string.h>

#include <hip/hip_ext.h>

#include "dqt_gemm_tile.h"
#include "dqt_internal.h"

namespace dqt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct F64Args {
    const double* Ad;
    const double* Bd;
    uint8_t* C;
    uint32_t m, n, ldc;
    uint32_t nks;          // k-steps of 4 (K_pad / 4)
    uint32_t ks_split;     // k-steps per wave
    uint32_t nrb;          // row blocks of the grid (Mw_pad / (16 TR))
    uint32_t er, ec;       // rows / columns per word
    uint32_t trans;        // Left through the uint8 kernel: X = B^T, words of e rows of A, C transposed
    RedqArgs ra;           // REDQ_(er ec) of a word of CC
};

struct F64PackArgs {
    const uint8_t* A;
    const uint8_t* B;
    double* Ad;
    double* Bd;
    uint32_t m, n, kdim, lda, ldb;
    uint32_t nks;
    uint64_t na;           // doubles of Ad
    uint64_t nb;           // doubles of Bd
    uint32_t er, ec, b;    // rows/columns per word, log2 Q
};

// Right: A copied as uint8 with zero padding (four bytes per thread), B
// packed e columns per binary64 word in the permuted-k step layout.
__global__ __launch_bounds__(256) void k_f64_pack_right(F64PackArgs a) {
    const uint32_t kp = a.nks * 4;           // K_pad (multiple of 16)
    const uint64_t nad = a.na / 4;           // dwords of the A copy
    const uint64_t total = nad + a.nb;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < total; t += (uint64_t)gridDim.x * 256) {
        if (t < nad) {
            const uint32_t row = (uint32_t)(t / (kp / 4)), k0 = (uint32_t)(t % (kp / 4)) * 4;
            uint32_t d = 0;
            if (row < a.m)
                for (uint32_t x = 0; x < 4; ++x)
                    if (k0 + x < a.kdim) d |= (uint32_t)a.A[(size_t)row * a.lda + k0 + x] << (8 * x);
            reinterpret_cast<uint32_t*>(a.Ad)[t] = d;
        } else {
            const uint64_t u = t - nad;
            const uint32_t l = (uint32_t)(u & 63), st = (uint32_t)((u >> 6) & 3);
            const uint64_t q = u >> 8;
            const uint32_t c = (uint32_t)(q % (kp / 16)), cb = (uint32_t)(q / (kp / 16));
            const uint32_t jw = cb * 16 + (l & 15), k = 16 * c + 4 * (l >> 4) + st;
            uint64_t w = 0;
            if (k < a.kdim)
                for (uint32_t x = 0; x < a.ec; ++x) {
                    const uint32_t col = jw * a.ec + x;
                    if (col < a.n) w |= (uint64_t)a.B[(size_t)k * a.ldb + col] << (a.b * x);
                }
            a.Bd[u] = (double)w;
        }
    }
}

// Left through the same kernel as Right, transposed (C^T = B^T A^T): B^T
// copied as uint8 [N_pad][K_pad] (column j of B becomes row j), and e rows of
// A packed per binary64 word in the step layout, word i' at k holding
// sum_t A[e i' + t][k] Q^t.
__global__ __launch_bounds__(256) void k_f64_pack_left(F64PackArgs a) {
    const uint32_t kp = a.nks * 4;
    const uint64_t nbd = a.nb / 4;           // dwords of the B^T copy
    const uint64_t total = a.na + nbd;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < total; t += (uint64_t)gridDim.x * 256) {
        if (t < a.na) {
            const uint32_t l = (uint32_t)(t & 63), st = (uint32_t)((t >> 6) & 3);
            const uint64_t q = t >> 8;
            const uint32_t c = (uint32_t)(q % (kp / 16)), rb = (uint32_t)(q / (kp / 16));
            const uint32_t iw = rb * 16 + (l & 15), k = 16 * c + 4 * (l >> 4) + st;
            uint64_t w = 0;
            if (k < a.kdim)
                for (uint32_t x = 0; x < a.er; ++x) {
                    const uint32_t row = iw * a.er + x;
                    if (row < a.m) w |= (uint64_t)a.A[(size_t)row * a.lda + k] << (a.b * x);
                }
            a.Ad[t] = (double)w;
        } else {
            const uint64_t u = t - a.na;
            const uint32_t col = (uint32_t)(u / (kp / 4)), k0 = (uint32_t)(u % (kp / 4)) * 4;
            uint32_t d = 0;
            if (col < a.n)
                for (uint32_t x = 0; x < 4; ++x)
                    if (k0 + x < a.kdim) d |= (uint32_t)a.B[(size_t)(k0 + x) * a.ldb + col] << (8 * x);
            reinterpret_cast<uint32_t*>(a.Bd)[u] = d;
        }
    }
}

// Uncompress/compress the operands into the matrix-core layouts (one double
// per thread, grid-stride).
__global__ __launch_bounds__(256) void k_f64_pack(F64PackArgs a) {
    const uint64_t total = a.na + a.nb;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < total; t += (uint64_t)gridDim.x * 256) {
        if (t < a.na) {
            const uint32_t l = (uint32_t)(t & 63), ks = (uint32_t)((t >> 6) % a.nks);
            const uint32_t rb = (uint32_t)((t >> 6) / a.nks);
            const uint32_t iw = rb * 16 + (l & 15), k = ks * 4 + (l >> 4);
            uint64_t w = 0;
            if (k < a.kdim)
                for (uint32_t s = 0; s < a.er; ++s) {
                    const uint32_t row = iw * a.er + s;
                    if (row < a.m) w |= (uint64_t)a.A[(size_t)row * a.lda + k] << (a.b * s);
                }
            a.Ad[t] = (double)w;
        } else {
            const uint64_t u = t - a.na;
            const uint32_t l = (uint32_t)(u & 63), ks = (uint32_t)((u >> 6) % a.nks);
            const uint32_t cb = (uint32_t)((u >> 6) / a.nks);
            const uint32_t jw = cb * 16 + (l & 15), k = ks * 4 + (l >> 4);
            uint64_t w = 0;
            if (k < a.kdim)
                for (uint32_t x = 0; x < a.ec; ++x) {
                    const uint32_t col = jw * a.ec + x;
                    if (col < a.n) w |= (uint64_t)a.B[(size_t)k * a.ldb + col] << (a.b * a.er * x);
                }
            a.Bd[u] = (double)w;
        }
    }
}

// One workgroup: KS waves on one block of 16 TR x 16 TC words, each wave a
// range of k-steps; partial sums (exact) added through LDS; then REDQ of
// every word and the bytes of its digits scattered to C.
template <int TR, int TC, int KS>
__global__ __launch_bounds__(64 * KS) void k_f64_mm(F64Args g) {
    __shared__ double red[KS > 1 ? KS * TR * TC * 4 * 64 : 1];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    uint32_t bid = blockIdx.x, nblk = gridDim.x, logical = bid;
    if ((nblk & 7u) == 0) logical = (bid & 7u) * (nblk >> 3) + (bid >> 3);
    const uint32_t rb = logical % g.nrb, cb = logical / g.nrb;
    const uint32_t ks0 = min(g.nks, wave * g.ks_split), ks1 = min(g.nks, ks0 + g.ks_split);

    const double* pa[TR];
    const double* pb[TC];
#pragma unroll
    for (int r = 0; r < TR; ++r) pa[r] = g.Ad + ((size_t)(rb * TR + r) * g.nks + ks0) * 64 + lane;
#pragma unroll
    for (int c = 0; c < TC; ++c) pb[c] = g.Bd + ((size_t)(cb * TC + c) * g.nks + ks0) * 64 + lane;
    f64x4 acc[TR][TC];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c) acc[r][c] = f64x4{0.0, 0.0, 0.0, 0.0};

    // operands of the next two k-steps are loaded while the current ones multiply
    constexpr int PF = 2;
    const uint32_t n = ks1 - ks0;
    double fa[PF][TR], fb[PF][TC];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
        for (int r = 0; r < TR; ++r) fa[u][r] = (u < (int)n) ? pa[r][u * 64] : 0.0;
#pragma unroll
        for (int c = 0; c < TC; ++c) fb[u][c] = (u < (int)n) ? pb[c][u * 64] : 0.0;
    }
    for (uint32_t s = 0; s < n; s += PF) {
        double ca[PF][TR], cbv[PF][TC];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int r = 0; r < TR; ++r) ca[u][r] = fa[u][r];
#pragma unroll
            for (int c = 0; c < TC; ++c) cbv[u][c] = fb[u][c];
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const uint32_t nx = s + PF + u;
            if (nx < n) {
#pragma unroll
                for (int r = 0; r < TR; ++r) fa[u][r] = pa[r][(size_t)nx * 64];
#pragma unroll
                for (int c = 0; c < TC; ++c) fb[u][c] = pb[c][(size_t)nx * 64];
            }
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            if (s + u < n) {
#pragma unroll
                for (int r = 0; r < TR; ++r)
#pragma unroll
                    for (int c = 0; c < TC; ++c)
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][r], cbv[u][c], acc[r][c], 0, 0, 0);
            }
        }
    }

    // split-k: wave w finishes the words q = w, w + KS, ... of its lane
    constexpr int NQ = TR * TC * 4;
    double v[NQ];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[(r * TC + c) * 4 + e] = acc[r][c][e];
    if (KS > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[(wave * NQ + q) * 64 + lane] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if ((uint32_t)q % KS != wave) continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < KS; ++w) sum += red[(w * NQ + q) * 64 + lane];
            v[q] = sum;
        }
    }
    const RedqArgs& ra = g.ra;
    const uint32_t nd = g.er * g.ec;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (KS > 1 && (uint32_t)q % KS != wave) continue;
        const int t = q / 4, e = q % 4;
        const uint32_t iw = (rb * TR + t / TC) * 16 + (lane >> 4) + 4 * e;
        const uint32_t jw = (cb * TC + t % TC) * 16 + (lane & 15u);
        const uint64_t word = (uint64_t)v[q];   // an integer below 2^52
        const uint64_t U = redq_compress(word, ra);
        // digit d = s + er x (row s of the word's rows, column x of its columns)
        uint32_t prev = field(U, 0, ra);
        for (uint32_t d = 0; d < nd; ++d) {
            const uint32_t next = d + 1 < nd ? field(U, d + 1, ra) : 0;
            const uint32_t mu = (ra.c && d + 1 < nd) ? correct_arith(prev, next, ra) : prev;
            prev = next;
            const uint32_t row = iw * g.er + d % g.er, col = jw * g.ec + d / g.er;
            if (row < g.m && col < g.n) g.C[(size_t)row * g.ldc + col] = (uint8_t)mu;
        }
    }
}

// Right compression: A as uint8 (four entries of a lane's four steps in one
// dword, converted to binary64 in registers), B words in the step layout; 2x2
// blocks of 16x16 words per wave, KS waves splitting the groups of 16 k.
template <int KS>
__global__ __launch_bounds__(64 * KS) void k_f64_right(F64Args g) {
    constexpr int TR = 2, TC = 2;
    __shared__ double red[KS > 1 ? KS * TR * TC * 4 * 64 : 1];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    uint32_t bid = blockIdx.x, nblk = gridDim.x, logical = bid;
    if ((nblk & 7u) == 0) logical = (bid & 7u) * (nblk >> 3) + (bid >> 3);
    const uint32_t rb = logical % g.nrb, cb = logical / g.nrb;
    const uint32_t ng = g.nks / 4;                       // groups of 16 k
    const uint32_t g0 = min(ng, wave * g.ks_split), g1 = min(ng, g0 + g.ks_split);
    const uint32_t kp = g.nks * 4;
    const uint8_t* A8 = reinterpret_cast<const uint8_t*>(g.Ad);
    const uint32_t* pa[TR];
#pragma unroll
    for (int r = 0; r < TR; ++r)
        pa[r] = reinterpret_cast<const uint32_t*>(A8 + (size_t)((rb * TR + r) * 16 + (lane & 15u)) * kp) + (lane >> 4);
    const double* pb[TC];
#pragma unroll
    for (int c = 0; c < TC; ++c) pb[c] = g.Bd + (size_t)(cb * TC + c) * ng * 256 + lane;
    f64x4 acc[TR][TC];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c) acc[r][c] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (uint32_t gi = g0; gi < g1; ++gi) {
        uint32_t ad[TR];
#pragma unroll
        for (int r = 0; r < TR; ++r) ad[r] = pa[r][(size_t)gi * 4];
        double bv[TC][4];
#pragma unroll
        for (int c = 0; c < TC; ++c)
#pragma unroll
            for (int st = 0; st < 4; ++st) bv[c][st] = pb[c][(size_t)gi * 256 + st * 64];
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                const double av = (double)((ad[r] >> (8 * st)) & 0xFFu);
#pragma unroll
                for (int c = 0; c < TC; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[c][st], acc[r][c], 0, 0, 0);
            }
    }
    constexpr int NQ = TR * TC * 4;
    double v[NQ];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[(r * TC + c) * 4 + e] = acc[r][c][e];
    if (KS > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[(wave * NQ + q) * 64 + lane] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if ((uint32_t)q % KS != wave) continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < KS; ++w) sum += red[(w * NQ + q) * 64 + lane];
            v[q] = sum;
        }
    }
    const RedqArgs& ra = g.ra;
    const uint32_t nd = g.er * g.ec;   // one of them is 1
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (KS > 1 && (uint32_t)q % KS != wave) continue;
        const int t = q / 4, e = q % 4;
        const uint32_t row = (rb * TR + t / TC) * 16 + (lane >> 4) + 4 * e;   // row of X
        const uint32_t jw = (cb * TC + t % TC) * 16 + (lane & 15u);           // word column
        if (row >= (g.trans ? g.n : g.m)) continue;
        const uint64_t U = redq_compress((uint64_t)v[q], ra);
        if (g.trans) {
            // digit d of word jw is the output at row e jw + d, column `row`
            uint32_t prev = field(U, 0, ra);
            for (uint32_t d = 0; d < nd; ++d) {
                const uint32_t next = d + 1 < nd ? field(U, d + 1, ra) : 0;
                const uint32_t mu = (ra.c && d + 1 < nd) ? correct_arith(prev, next, ra) : prev;
                prev = next;
                const uint32_t orow = jw * nd + d;
                if (orow < g.m) g.C[(size_t)orow * g.ldc + row] = (uint8_t)mu;
            }
            continue;
        }
        uint8_t* out = g.C + (size_t)row * g.ldc + jw * nd;
        uint32_t prev = field(U, 0, ra);
        if (nd == 4 && jw * 4 + 3 < g.n && ((uintptr_t)out & 3) == 0) {
            // the four digits are four adjacent outputs: one dword store
            uint32_t bytes = 0;
#pragma unroll
            for (uint32_t d = 0; d < 4; ++d) {
                const uint32_t next = d + 1 < 4 ? field(U, d + 1, ra) : 0;
                const uint32_t mu = (ra.c && d + 1 < 4) ? correct_arith(prev, next, ra) : prev;
                prev = next;
                bytes |= mu << (8 * d);
            }
            *reinterpret_cast<uint32_t*>(out) = bytes;
            continue;
        }
        for (uint32_t d = 0; d < nd; ++d) {
            const uint32_t next = d + 1 < nd ? field(U, d + 1, ra) : 0;
            const uint32_t mu = (ra.c && d + 1 < nd) ? correct_arith(prev, next, ra) : prev;
            prev = next;
            if (jw * nd + d < g.n) out[d] = (uint8_t)mu;
        }
    }
}

static uint64_t rup(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// Plan of a compressed product on the matrix cores.  algo: DQT_GEMM_RIGHT
// (er = 1), DQT_GEMM_LEFT (ec = 1), DQT_GEMM_FULL (both).  In the resolved
// plan, m_pad / n_pad are the padded word rows / columns, k_pad the padded
// inner dimension, tm / tn the 16x16 blocks per wave and s the k-split.
dqt_status f64_plan(uint32_t algo, uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint32_t want_b,
                    uint32_t want_ks, GemmPlanResolved* r) {
    // smallest Q with kdim (p-1)^2 < Q (eq:lower); digits per word within 52 bits
    const uint64_t bound = (kdim ? kdim : 1) * (uint64_t)(p - 1) * (p - 1);
    uint32_t b = 1;
    while (b < 52 && (1ull << b) <= bound) ++b;
    if (want_b) {
        if (want_b < b || want_b > 26) return DQT_E_BOUND;
        b = want_b;
    }
    const uint32_t D = 52 / b;
    if (D < 2) return DQT_E_UNSUPPORTED;   // not even two digits per word: no compression
    switch (algo) {
        case DQT_GEMM_RIGHT: r->er = 1; r->ec = D > 8 ? 8 : D; break;
        case DQT_GEMM_LEFT: r->er = D > 8 ? 8 : D; r->ec = 1; break;
        case DQT_GEMM_FULL:
            if (D < 4) return DQT_E_UNSUPPORTED;   // two rows and two columns per word at least
            r->er = 2;
            r->ec = D / 2 > 4 ? 4 : D / 2;
            break;
        default: return DQT_E_UNSUPPORTED;
    }
    r->algo = algo;
    r->b = b;
    r->tm = 2;
    r->tn = 2;
    const uint64_t Mw = (m + r->er - 1) / r->er, Nw = (n + r->ec - 1) / r->ec;
    r->m_pad = (uint32_t)rup(Mw ? Mw : 1, 16 * r->tm);
    r->n_pad = (uint32_t)rup(Nw ? Nw : 1, 16 * r->tn);
    const bool u8x = algo == DQT_GEMM_RIGHT || algo == DQT_GEMM_LEFT;   // one operand read as uint8
    const uint32_t kq = u8x ? 16 : 4;   // k padding (uint8 operand: groups of 16)
    const uint64_t kpad = (kdim + kq - 1) / kq * kq;
    r->k_pad = (uint32_t)(kpad ? kpad : kq);
    if (want_ks) {
        if (want_ks != 1 && want_ks != 2 && want_ks != 4 && want_ks != 8 && !(want_ks == 16 && u8x))
            return DQT_E_INVALID;
        r->s = want_ks;
    } else {
        // enough waves for the chip: k split across up to 8 waves of a workgroup
        const uint64_t blocks = (uint64_t)(r->m_pad / (16 * r->tm)) * (r->n_pad / (16 * r->tn));
        r->s = 1;
        if (u8x)
            while (r->s < 16 && blocks * r->s < 4096 && (r->k_pad / 16) / (r->s * 2) >= 2) r->s *= 2;
        else
            while (r->s < 8 && blocks * r->s < 2048 && (r->k_pad / 4) / (r->s * 2) >= 8) r->s *= 2;
    }
    r->ws_bytes = f64_side_bytes(*r, 0) + f64_side_bytes(*r, 1);
    return DQT_OK;
}

size_t f64_side_bytes(const GemmPlanResolved& r, int side) {
    if (side == 0 && r.algo == DQT_GEMM_RIGHT) return ((size_t)r.m_pad * r.k_pad + 15) / 16 * 16;  // uint8 copy of A
    if (side == 1 && r.algo == DQT_GEMM_LEFT) return ((size_t)r.n_pad * r.k_pad + 15) / 16 * 16;   // uint8 B^T
    return (size_t)(side == 0 ? r.m_pad : r.n_pad) * r.k_pad * sizeof(double);
}

template <int KS>
static void launch_f64_mm(const F64Args& g, unsigned grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(k_f64_mm<2, 2, KS>, dim3(grid), dim3(64 * KS), 0, s, e0, e1, 0, g);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_f64_mm<2, 2, KS>), dim3(grid), dim3(64 * KS), 0, s, g);
}

template <int KS>
static void launch_f64_right(const F64Args& g, unsigned grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(k_f64_right<KS>, dim3(grid), dim3(64 * KS), 0, s, e0, e1, 0, g);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_f64_right<KS>), dim3(grid), dim3(64 * KS), 0, s, g);
}

// Either operand may be NULL (its packed copy is kept).
dqt_status f64_pack_enqueue(const GemmPlanResolved& r, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A,
                            uint64_t lda, const uint8_t* B, uint64_t ldb, void* pA, void* pB, hipStream_t s) {
    F64PackArgs a;
    a.A = A;
    a.B = B;
    a.Ad = reinterpret_cast<double*>(pA);
    a.Bd = reinterpret_cast<double*>(pB);
    a.m = (uint32_t)m;
    a.n = (uint32_t)n;
    a.kdim = (uint32_t)kdim;
    a.lda = (uint32_t)lda;
    a.ldb = (uint32_t)ldb;
    a.nks = r.k_pad / 4;
    a.na = A ? (uint64_t)r.m_pad * r.k_pad : 0;   // Right: bytes of the uint8 copy; else doubles
    a.nb = B ? (uint64_t)r.n_pad * r.k_pad : 0;   // Left: bytes of the uint8 B^T; else doubles
    a.er = r.er;
    a.ec = r.ec;
    a.b = r.b;
    if (a.na + a.nb == 0) return DQT_OK;
    if (r.algo == DQT_GEMM_RIGHT) {
        hipLaunchKernelGGL(k_f64_pack_right, dim3(stream_grid(a.na / 4 + a.nb, 256, 8)), dim3(256), 0, s, a);
        DQT_LAUNCH_CHECK("fgemm(f64 pack)");
        return DQT_OK;
    }
    if (r.algo == DQT_GEMM_LEFT) {
        hipLaunchKernelGGL(k_f64_pack_left, dim3(stream_grid(a.na + a.nb / 4, 256, 8)), dim3(256), 0, s, a);
        DQT_LAUNCH_CHECK("fgemm(f64 pack)");
        return DQT_OK;
    }
    hipLaunchKernelGGL(k_f64_pack, dim3(stream_grid(a.na + a.nb, 256, 8)), dim3(256), 0, s, a);
    DQT_LAUNCH_CHECK("fgemm(f64 pack)");
    return DQT_OK;
}

dqt_status f64_compute_enqueue(const GemmPlanResolved& r, uint32_t p, uint64_t m, uint64_t n, uint8_t* C, uint64_t ldc,
                               const void* pA, const void* pB, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    F64Args g;
    memset(&g, 0, sizeof(g));
    g.Ad = reinterpret_cast<const double*>(pA);
    g.Bd = reinterpret_cast<const double*>(pB);
    g.C = C;
    g.m = (uint32_t)m;
    g.n = (uint32_t)n;
    g.ldc = (uint32_t)ldc;
    g.nks = r.k_pad / 4;
    const bool u8x = r.algo == DQT_GEMM_RIGHT || r.algo == DQT_GEMM_LEFT;
    g.ks_split = u8x ? (r.k_pad / 16 + r.s - 1) / r.s : (g.nks + r.s - 1) / r.s;
    g.nrb = r.m_pad / (16 * r.tm);
    g.er = r.er;
    g.ec = r.ec;
    const uint32_t nd = r.er * r.ec;
    DQT_TRY(make_redq_args(p, r.b, nd, nd * r.b, &g.ra));
    unsigned grid = g.nrb * (r.n_pad / (16 * r.tn));
    if (r.algo == DQT_GEMM_LEFT) {
        // the uint8 operand (rows of the kernel's X) is B^T; the words are the packed rows of A
        g.trans = 1;
        g.Ad = reinterpret_cast<const double*>(pB);
        g.Bd = reinterpret_cast<const double*>(pA);
        g.nrb = r.n_pad / (16 * r.tn);
        grid = g.nrb * (r.m_pad / (16 * r.tm));
    }
    if (u8x) {
        switch (r.s) {
            case 1: launch_f64_right<1>(g, grid, s, e0, e1); break;
            case 2: launch_f64_right<2>(g, grid, s, e0, e1); break;
            case 4: launch_f64_right<4>(g, grid, s, e0, e1); break;
            case 8: launch_f64_right<8>(g, grid, s, e0, e1); break;
            default: launch_f64_right<16>(g, grid, s, e0, e1); break;
        }
        DQT_LAUNCH_CHECK("fgemm(f64 right)");
        return DQT_OK;
    }
    switch (r.s) {
        case 1: launch_f64_mm<1>(g, grid, s, e0, e1); break;
        case 2: launch_f64_mm<2>(g, grid, s, e0, e1); break;
        case 4: launch_f64_mm<4>(g, grid, s, e0, e1); break;
        default: launch_f64_mm<8>(g, grid, s, e0, e1); break;
    }
    DQT_LAUNCH_CHECK("fgemm(f64)");
    return DQT_OK;
}

}  // namespace dqt
