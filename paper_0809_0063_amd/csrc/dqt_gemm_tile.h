// One output tile of an F_p matrix product on packed words (device code
// shared by the single-product and the batched kernels).
//
// Packed path (compressed matrix multiplication, section 7.1 of the paper):
// k is cut into groups of four; a group of a row of A becomes one 32-bit word
// of two 16-bit lanes, each lane the reversed Kronecker pair a_(2l) Q +
// a_(2l+1); the same group of a column of B becomes b_(2l) + b_(2l+1) Q.  One
// v_dot2_u32_u16 of the two words adds both lane products into a 32-bit
// accumulator whose digit of weight Q (the middle product) collects four
// multiply-adds of the dot product.  Digits never carry while the number of
// accumulated k (the delayed-reduction interval) times (p-1)^2 stays below Q
// (eq:lower); the accumulator wraps modulo 2^32 above digit 1, which leaves
// digits 0 and 1 exact.  After each interval the middle digit is extracted
// and added to a plain accumulator.  One reduction per output ends the
// product (REDC, section 7.2), or the dot products of several outputs are
// gathered into one word and reduced by one REDQ (section 3).
//
// Comparators in the same structure: one entry per word and one
// v_mad_u32_u24 per multiply-add (the paper's delayed baseline, section 5.1),
// or four u8 entries per word and v_dot4_u32_u8.
//
// A wave owns TM rows (uniform: their words are scalar loads, operands in
// SGPRs) and 64*TN columns (one per lane and per j, coalesced vector loads).
// S waves of a workgroup split k and add their partial sums through LDS.
#pragma once

#include "../../include/dqt.h"
#include "dqt_device.h"

namespace dqt {

enum GemmOp { OP_DOT2 = 0, OP_DOT4 = 1, OP_MAD = 2 };

struct GemmArgs {
    const uint32_t* CA;   // [KW][m_pad] packed words of A, k-major
    const uint32_t* CB;   // [KW][n_pad] packed words of B, k-major
    uint8_t* C;
    uint32_t m, n, ldc;
    uint32_t m_pad, n_pad;
    uint32_t KW;          // k-groups (words) along k
    uint32_t kw_split;    // k-groups per wave
    uint32_t lw;          // delayed-reduction interval in k-groups (0 = whole range)
    uint32_t nrb, ncb;    // row blocks, column blocks
    uint32_t b;           // log2 Q (packed path)
    uint32_t p, pmagic;
    uint32_t epi;         // 0 REDC, 1 REDQ
    uint32_t epi_e;       // outputs per REDQ word
    uint32_t op;          // GemmOp (batched kernel only)
    RedqArgs ra;          // REDQ_{epi_e} parameters of the epilogue
};

// x mod p for any 32-bit x: quotient from the rounded-up reciprocal, one fix.
__device__ __forceinline__ uint32_t mod_u32(uint32_t x, uint32_t p, uint32_t pmagic) {
    const uint32_t qt = __umulhi(x, pmagic);
    const int32_t r = (int32_t)(x - qt * p);
    return (uint32_t)(r < 0 ? r + (int32_t)p : r);
}

template <int OP>
__device__ __forceinline__ uint32_t mac(uint32_t a, uint32_t b, uint32_t acc) {
    if (OP == OP_DOT2) {
        typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b), acc, false);
    } else if (OP == OP_DOT4) {
        return __builtin_amdgcn_udot4(a, b, acc, false);
    } else {
        return __umul24(a, b) + acc;
    }
}

// LDS words a tile needs for its split-k reduction.
template <int TM, int TN, int S>
struct TileSmem {
    static constexpr int words = (S > 1) ? S * TM * TN * 64 : 1;
};

// FLUSH = false: the whole k range of a wave is one delayed-reduction
// interval (no intermediate extraction, no second accumulator).
// EPI: 0 = one REDC per output, 1 = REDQ over gathered dot products (a
// template parameter so that the REDC kernels keep no REDQ parameters in
// SGPRs, which hold the prefetched words of A during the k loop).
template <int OP, int TM, int TN, int S, bool FLUSH, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, uint32_t rb, uint32_t cb, uint32_t wave, uint32_t lane,
                                          uint32_t* red) {
    const uint32_t row0 = rb * TM;
    const uint32_t col0 = cb * 64u * TN;

    uint32_t acc[TM][TN];
    uint32_t wide[FLUSH ? TM : 1][FLUSH ? TN : 1];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = 0;
    if (FLUSH) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) wide[FLUSH ? i : 0][FLUSH ? j : 0] = 0;
    }

    const uint32_t kw0 = wave * g.kw_split;
    const uint32_t kw1 = min(g.KW, kw0 + g.kw_split);
    const uint32_t* __restrict__ pa = g.CA + row0;
    const uint32_t* __restrict__ pb = g.CB + col0 + lane;
    const uint32_t mask = (1u << g.b) - 1u;

    auto body = [&](uint32_t kw) {
        uint32_t av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = pa[(size_t)kw * g.m_pad + i];
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = pb[(size_t)kw * g.n_pad + 64 * j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = mac<OP>(av[i], bv[j], acc[i][j]);
    };

    if (!FLUSH) {
#pragma unroll 8
        for (uint32_t kw = kw0; kw < kw1; ++kw) body(kw);
    } else {
        // delayed-reduction interval in k-groups
        const uint32_t step = g.lw ? g.lw : (kw1 > kw0 ? kw1 - kw0 : 1u);
        for (uint32_t kc = kw0; kc < kw1; kc += step) {
            const uint32_t ke = min(kw1, kc + step);
#pragma unroll 4
            for (uint32_t kw = kc; kw < ke; ++kw) body(kw);
            // end of an interval: move the middle digit out
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    wide[FLUSH ? i : 0][FLUSH ? j : 0] += (acc[i][j] >> g.b) & mask;
                    acc[i][j] = 0;
                }
        }
    }
    const GemmArgs& ge = g;
    // value of each output over this wave's k range
    if (OP == OP_DOT2) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = FLUSH ? wide[FLUSH ? i : 0][FLUSH ? j : 0] : ((acc[i][j] >> ge.b) & mask);
    }

    // split-k: add the S partial sums through LDS; wave w finishes rows i = w, w+S, ...
    if (S > 1) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) red[((wave * TM + i) * TN + j) * 64 + lane] = acc[i][j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if ((uint32_t)i % S != wave) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                uint32_t s = 0;
#pragma unroll
                for (int w = 0; w < S; ++w) s += red[((w * TM + i) * TN + j) * 64 + lane];
                acc[i][j] = s;
            }
        }
    }

    // epilogue: reduce mod p and store bytes
    if (EPI == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (S > 1 && (uint32_t)i % S != wave) continue;
            const uint32_t row = row0 + i;
            if (row >= ge.m) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const uint32_t col = col0 + lane + 64 * j;
                if (col < ge.n) ge.C[(size_t)row * ge.ldc + col] = (uint8_t)mod_u32(acc[i][j], ge.p, ge.pmagic);
            }
        }
    } else {
        // REDQ_e: the dot products (each below the epilogue's q) of up to e
        // outputs of this lane packed into one word, one REDQ for all of them.
        const RedqArgs& ra = ge.ra;
        uint64_t word = 0;
        uint32_t nin = 0;
        uint32_t rows[8], cols[8];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (S > 1 && (uint32_t)i % S != wave) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                word |= (uint64_t)acc[i][j] << (ra.b * nin);
                rows[nin] = row0 + i;
                cols[nin] = col0 + lane + 64 * j;
                ++nin;
                const bool last = (i + S > TM - 1) && j == TN - 1;
                if (nin == ge.epi_e || last) {
                    const uint64_t U = redq_compress(word, ra);
                    for (uint32_t t = 0; t < nin; ++t) {
                        const uint32_t ut = field(U, t, ra);
                        uint32_t mu = ut;
                        if (ra.c && t + 1 < nin) mu = correct_arith(ut, field(U, t + 1, ra), ra);
                        if (rows[t] < ge.m && cols[t] < ge.n) ge.C[(size_t)rows[t] * ge.ldc + cols[t]] = (uint8_t)mu;
                    }
                    word = 0;
                    nin = 0;
                }
            }
        }
    }
}

// Pack one 256-word block of the operands of a product (A blocks first).
struct PackArgs {
    const uint8_t* A;
    const uint8_t* B;
    uint32_t* CA;
    uint32_t* CB;
    uint32_t m, n, kdim, lda, ldb;
    uint32_t m_pad, n_pad, KW;
    uint32_t b;       // log2 Q
    uint32_t op;      // GemmOp
    uint32_t nba;     // blocks for A
};

__device__ __forceinline__ void gemm_pack_block(const PackArgs& a, uint32_t blk, uint32_t tid) {
    const uint32_t epw = a.op == OP_MAD ? 1u : 4u;  // entries per word
    if (blk < a.nba) {
        // CA[kw][row]: word index = kw * m_pad + row (rows fastest: coalesced stores)
        const uint64_t t = (uint64_t)blk * 256 + tid;
        if (t >= (uint64_t)a.KW * a.m_pad) return;
        const uint32_t kw = (uint32_t)(t / a.m_pad), row = (uint32_t)(t % a.m_pad);
        uint32_t e[4] = {0, 0, 0, 0};
        if (row < a.m)
            for (uint32_t i = 0; i < epw; ++i) {
                const uint32_t k = kw * epw + i;
                if (k < a.kdim) e[i] = a.A[(size_t)row * a.lda + k];
            }
        uint32_t w;
        if (a.op == OP_DOT2)
            w = ((e[0] << a.b) | e[1]) | (((e[2] << a.b) | e[3]) << 16);
        else if (a.op == OP_DOT4)
            w = e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
        else
            w = e[0];
        a.CA[t] = w;
    } else {
        const uint64_t t = (uint64_t)(blk - a.nba) * 256 + tid;
        if (t >= (uint64_t)a.KW * a.n_pad) return;
        const uint32_t kw = (uint32_t)(t / a.n_pad), col = (uint32_t)(t % a.n_pad);
        uint32_t e[4] = {0, 0, 0, 0};
        if (col < a.n)
            for (uint32_t i = 0; i < epw; ++i) {
                const uint32_t k = kw * epw + i;
                if (k < a.kdim) e[i] = a.B[(size_t)k * a.ldb + col];
            }
        uint32_t w;
        if (a.op == OP_DOT2)
            w = (e[0] | (e[1] << a.b)) | ((e[2] | (e[3] << a.b)) << 16);
        else if (a.op == OP_DOT4)
            w = e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
        else
            w = e[0];
        a.CB[t] = w;
    }
}

// Resolved plan of one product (host side, dqt_gemm.hip).
struct GemmPlanResolved {
    uint32_t algo;
    uint32_t op;
    uint32_t b;         // log2 Q (packed)
    uint32_t lw;        // interval in k-groups (0 = none)
    uint32_t tm, tn, s;
    uint32_t epi;
    uint32_t KW, m_pad, n_pad, k_pad;
    size_t ws_bytes;
};
dqt_status fgemm_resolve(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan* plan,
                         GemmPlanResolved* r);
// Epilogue parameters (REDQ_e word layout) of a resolved plan.
dqt_status fgemm_epilogue_args(uint32_t p, uint64_t kdim, const GemmPlanResolved& r, GemmArgs* g);

}  // namespace dqt
