// Block-word helpers of the long products by the FQT (section 5.2 of the
// paper), shared by the kernels and by host-side checks of the same code.
#pragma once

#include "dqt_device.h"

namespace dqt {

// Reduces the block words W_0 .. W_{NW-1} of one product (Wof(w) gives W_w;
// one REDQ_{2d+1} each), adds the top d coefficients of every block to the
// next block's first d modulo p, and puts coefficient j of the product in
// byte j of the stream ob (NO dwords, zero on entry).  Coefficients at
// j >= nout = na + nb - 1 lie past the product's degree and come out 0.
// QB, QW, SMALL: compile-time q = 2^QB, residue width and word size (binary64
// floor without the AFDIV test), or 0 / false for the run-time values of ra.
template <int BS, int NW, int QB, int QW, bool SMALL, int NO, typename WordOf>
__host__ __device__ __forceinline__ void fqt_finish(WordOf Wof, uint32_t nout, const RedqArgs& ra, const uint16_t* tab,
                                           uint32_t (&ob)[NO]) {
    constexpr int NR = 2 * BS - 1;
    uint32_t carry[BS > 1 ? BS - 1 : 1];
#pragma unroll
    for (int s = 0; s < BS - 1; ++s) carry[s] = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t U = redq_compress_t<(QB ? NR : 0), QB, QW, SMALL>(Wof(w), ra);
        uint32_t mu[NR];
        redq_correct<NR, QB, QW>(U, ra, tab, [&](int s, uint32_t v) { mu[s] = v; });
#pragma unroll
        for (int s = 0; s < BS; ++s) {
            uint32_t v = mu[s] + (s < BS - 1 ? carry[s] : 0u);
            v = v >= ra.p ? v - ra.p : v;
            const int pos = BS * w + s;
            ob[pos >> 2] |= v << (8 * (pos & 3));
        }
#pragma unroll
        for (int s = 0; s < BS - 1; ++s) carry[s] = mu[BS + s];
    }
    // coefficients past the last block start: only the carry of the last block
    // (zero when the loop stopped early: those positions lie past the degree)
#pragma unroll
    for (int s = 0; s < BS - 1; ++s) {
        const int pos = BS * NW + s;
        ob[pos >> 2] |= carry[s] << (8 * (pos & 3));
    }
}

// Block words of one operand from its record (ND dwords, bytes past the
// record zero): block i holds coefficients i BS .. i BS + BS - 1 at q = 2^b.
template <int BS, int MAXB, typename Word, int ND>
__host__ __device__ __forceinline__ void fqt_words(const uint32_t (&d)[ND], uint32_t b, Word* w) {
    static_assert(4 * ND >= MAXB * BS, "record dwords");
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        Word v = 0;
#pragma unroll
        for (int s = 0; s < BS; ++s) {
            const int c = i * BS + s;
            v |= (Word)((d[c >> 2] >> (8 * (c & 3))) & 0xFFu) << (b * s);
        }
        w[i] = v;
    }
}

// Dwords of an operand record and of a result stream of the FQT kernels.
template <int BS, int MAXB>
struct FqtShape {
    static constexpr int ND = (MAXB * BS + 3) / 4;
    static constexpr int NO = (2 * MAXB * BS - 1 + 3) / 4;
    static constexpr int NW = 2 * MAXB - 1;
};

}  // namespace dqt
