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
// four u8 entries per word and v_dot4_u32_u8, or, for p <= 16, eight 4-bit
// entries per word and v_dot8_u32_u4 (eight multiply-adds per instruction).
//
// A wave owns TM rows (uniform: their words are scalar loads, operands in
// SGPRs) and 64*TN columns (TN adjacent columns per lane, one vector load per
// k-group).  S waves of a workgroup split k and add their partial sums
// through LDS.
#pragma once

#include "../../include/dqt.h"
#include "dqt_device.h"

namespace dqt {

enum GemmOp { OP_DOT2 = 0, OP_DOT4 = 1, OP_MAD = 2, OP_DOT8 = 3 };

// Entries of a matrix per packed word along k.
__host__ __device__ inline uint32_t entries_per_word(uint32_t op) {
    return op == OP_MAD ? 1u : (op == OP_DOT8 ? 8u : 4u);
}

struct GemmArgs {
    const uint32_t* CA;   // [m_pad/TM][KW][TM] packed words of A (tile-major, see gemm_tile)
    const uint32_t* CB;   // [n_pad/(64 TN)][KW][64 TN] packed words of B
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
    const uint32_t qt = mulhi_u32(x, pmagic);
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
    } else if (OP == OP_DOT8) {
        return __builtin_amdgcn_udot8(a, b, acc, false);
    } else {
        // one v_mad_u32_u24 per multiply-add, written out: from __umul24(a, b) + acc
        // the compiler reassociates a k-group's chain into separate products and
        // three-way adds, which takes more registers than the tile has (spills)
        // and 1.5 instructions per multiply-add.  a is an A word, wave-uniform,
        // held in an SGPR (scalar loads).
        uint32_t r;
        asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(acc));
        return r;
    }
}

// LDS words a tile needs for its split-k reduction.
template <int TM, int TN, int S>
struct TileSmem {
    static constexpr int words = (S > 1) ? S * TM * TN * 64 : 1;
};

// Words of TN consecutive columns held by one lane (one vector load; clang
// vector types, which load through any address space).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int TN>
struct LaneWords;
template <>
struct LaneWords<2> {
    typedef u32x2 T;
    static __device__ __forceinline__ void get(const u32x2& v, uint32_t (&o)[2]) {
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct LaneWords<4> {
    typedef u32x4 T;
    static __device__ __forceinline__ void get(const u32x4& v, uint32_t (&o)[4]) {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};

// Address-space views of read-only device memory: constant (scalar loads for
// wave-uniform addresses) and global.
typedef __attribute__((address_space(4))) uint32_t ConstU32;
template <class T>
using GlobalT = __attribute__((address_space(1))) T;

// k-groups per pipeline step: the A words of two steps (the one being
// multiplied and the one being loaded) stay within 64 SGPRs.
template <int TM>
struct PipeU {
    static constexpr int value = TM >= 32 ? 1 : 32 / TM;
};

// FLUSH = false: the whole k range of a wave is one delayed-reduction
// interval (no intermediate extraction, no second accumulator).
// EPI: 0 = one REDC per output, 1 = REDQ over gathered dot products (a
// template parameter so that the REDC kernels keep no REDQ parameters in
// SGPRs, which hold the prefetched words of A during the k loop).
//
// Packed layouts (tile-major, so that the operands of consecutive k-groups
// are consecutive in memory and the loads of a step share one base address
// with immediate offsets):
//   CA: [m_pad / TM][KW][TM]          row block, k-group, row in the block;
//   CB: [n_pad / (64 TN)][KW][64 TN]  column block, k-group, column in the
//                                     block (lane l owns columns l TN .. l TN + TN - 1).
//
// The k loop is software-pipelined in steps of U k-groups with two register
// buffers: the loads of step t+1 are issued right after the first k-group of
// step t has used step t's words, so they overlap the rest of step t.  (Scalar
// loads complete out of order, so a wave can only wait for all of its
// outstanding scalar loads at once; issuing the next step's A words after the
// current ones have been consumed keeps that wait from covering them.)
// Scheduling barriers keep the compiler from moving the loads across.
template <int OP, int TM, int TN, int S, bool FLUSH, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, uint32_t rb, uint32_t cb, uint32_t wave, uint32_t lane,
                                          uint32_t* red) {
    constexpr int U = PipeU<TM>::value;
    typedef typename LaneWords<TN>::T V;
    const uint32_t row0 = rb * TM;
    const uint32_t col0 = cb * 64u * TN + lane * TN;

    uint32_t acc[TM][TN];
    uint32_t wide[FLUSH ? TM : 1][FLUSH ? TN : 1];
    if (FLUSH) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) wide[FLUSH ? i : 0][FLUSH ? j : 0] = 0;
    }

    const uint32_t kw0 = min(g.KW, wave * g.kw_split);
    const uint32_t kw1 = min(g.KW, kw0 + g.kw_split);
    // The packed operands are read-only while this kernel runs (they are written by
    // the packing kernel before it): A through the constant address space, so
    // that its wave-uniform words come in by scalar loads, and B through the
    // global one, also when the pointers come from a descriptor in memory (the
    // batched kernel) rather than from the kernel arguments.
    const ConstU32* __restrict__ pa =
        reinterpret_cast<const ConstU32*>(reinterpret_cast<uintptr_t>(g.CA + ((size_t)rb * g.KW + kw0) * TM));
    const GlobalT<V>* __restrict__ pb = reinterpret_cast<const GlobalT<V>*>(
        reinterpret_cast<uintptr_t>(reinterpret_cast<const V*>(g.CB + ((size_t)cb * g.KW + kw0) * (64u * TN)) + lane));
    const uint32_t mask = (1u << g.b) - 1u;

    uint32_t a0[U][TM], a1[U][TM];
    V b0[U], b1[U];
    // the words of step t (U k-groups from pa, pb)
    auto load = [&](uint32_t (&a)[U][TM], V (&bv)[U], uint32_t t) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < TM; ++i) a[u][i] = pa[(t * U + u) * TM + i];
            bv[u] = pb[(t * U + u) * 64];
        }
    };
    // one k-group; zero = the accumulators start from 0 here
    auto kgroup = [&](const uint32_t (&a)[TM], const V& bvec, bool zero) {
        uint32_t bw[TN];
        LaneWords<TN>::get(bvec, bw);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = mac<OP>(a[i], bw[j], zero ? 0u : acc[i][j]);
    };
    // step t from (a, bv) while the words of step tn are loaded into (an, bn)
    auto step = [&](const uint32_t (&a)[U][TM], const V (&bv)[U], uint32_t (&an)[U][TM], V (&bn)[U], uint32_t tn,
                    bool zero) {
        kgroup(a[0], bv[0], zero);
        __builtin_amdgcn_sched_barrier(0);
        load(an, bn, tn);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 1; u < U; ++u) kgroup(a[u], bv[u], false);
    };
    // n consecutive k-groups from (pa, pb), advancing both; zero = the
    // accumulators start from 0 (folded into the first k-group)
    auto run = [&](uint32_t n, bool zero) {
        const uint32_t nsteps = n / U;
        if (nsteps) {
            // every load is unconditional: the last step reloads its own words
            const uint32_t last = nsteps - 1;
            load(a0, b0, 0);
            step(a0, b0, a1, b1, min(1u, last), zero);
            uint32_t t = 1;
            for (; t + 2 <= nsteps; t += 2) {
                step(a1, b1, a0, b0, t + 1, false);
                step(a0, b0, a1, b1, min(t + 2, last), false);
            }
            if (t < nsteps) step(a1, b1, a0, b0, t, false);
            pa += nsteps * U * TM;
            pb += nsteps * U * 64;
        } else if (zero) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = 0;
        }
        for (uint32_t c = nsteps * U; c < n; ++c) {
            uint32_t a[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = pa[i];
            const V bv = pb[0];
            kgroup(a, bv, false);
            pa += TM;
            pb += 64;
        }
    };

    const uint32_t nk = kw1 - kw0;
    if (!FLUSH) {
        run(nk, true);
    } else {
        // delayed-reduction interval in k-groups
        const uint32_t step_k = g.lw ? g.lw : (nk ? nk : 1u);
        for (uint32_t kc = 0; kc < nk; kc += step_k) {
            run(min(step_k, nk - kc), true);
            // end of an interval: move the middle digit out
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) wide[FLUSH ? i : 0][FLUSH ? j : 0] += (acc[i][j] >> g.b) & mask;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = wide[FLUSH ? i : 0][FLUSH ? j : 0];
    }
    const GemmArgs& ge = g;
    // Packed path without flush: acc holds the raw accumulators.  Their digits
    // 0 and 1 never carry over the whole k range (eq:lower for kdim), so the
    // raw words of the S waves are added as they are and the middle digit is
    // taken once, from the sum.
    constexpr bool RAW = (OP == OP_DOT2) && !FLUSH;

    // split-k: add the S partial sums through LDS; wave w finishes rows i = w, w+S, ...
    // Layout [wave][row][lane][TN]: each lane writes and reads its TN words as one vector.
    if (S > 1) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            uint32_t* dst = &red[((wave * TM + i) * 64 + lane) * TN];
            if (TN == 4) *reinterpret_cast<uint4*>(dst) = make_uint4(acc[i][0], acc[i][1], acc[i][TN - 2], acc[i][TN - 1]);
            else *reinterpret_cast<uint2*>(dst) = make_uint2(acc[i][0], acc[i][1]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if ((uint32_t)i % S != wave) continue;
            uint32_t sum[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) sum[j] = 0;
#pragma unroll
            for (int w = 0; w < S; ++w) {
                const uint32_t* src = &red[((w * TM + i) * 64 + lane) * TN];
                uint32_t v[TN];
                if (TN == 4) {
                    const uint4 x = *reinterpret_cast<const uint4*>(src);
                    v[0] = x.x;
                    v[1] = x.y;
                    v[TN - 2] = x.z;
                    v[TN - 1] = x.w;
                } else {
                    const uint2 x = *reinterpret_cast<const uint2*>(src);
                    v[0] = x.x;
                    v[TN - 1] = x.y;
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) sum[j] += v[j];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = sum[j];
        }
    }
    if (RAW) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (S > 1 && (uint32_t)i % S != wave) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = (acc[i][j] >> ge.b) & mask;
        }
    }

    // epilogue: reduce mod p and store bytes
    if (EPI == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (S > 1 && (uint32_t)i % S != wave) continue;
            const uint32_t row = row0 + i;
            if (row >= ge.m) continue;
            uint8_t* out = ge.C + (size_t)row * ge.ldc + col0;
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < TN; ++j) v |= mod_u32(acc[i][j], ge.p, ge.pmagic) << (8 * j);
            if (col0 + TN <= ge.n && ((uintptr_t)out & (TN - 1)) == 0) {
                if (TN == 4) *reinterpret_cast<uint32_t*>(out) = v;
                else *reinterpret_cast<uint16_t*>(out) = (uint16_t)v;
            } else {
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    if (col0 + j < ge.n) out[j] = (uint8_t)(v >> (8 * j));
            }
        }
    } else {
        // REDQ_e: the dot products (each below the epilogue's q) of up to e
        // consecutive outputs of one row of this lane packed into one word, one
        // REDQ for all of them; the row's TN residues are stored as one word, as
        // in the REDC path.  (Fields are taken by shifts, not from indexed arrays,
        // which would live in scratch memory.)
        const RedqArgs& ra = ge.ra;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (S > 1 && (uint32_t)i % S != wave) continue;
            const uint32_t row = row0 + i;
            uint32_t v = 0;
            uint64_t word = 0;
            uint32_t nin = 0;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                word |= (uint64_t)acc[i][j] << (ra.b * nin);
                ++nin;
                if (nin == ge.epi_e || j == TN - 1) {
                    const uint64_t U2 = redq_compress(word, ra);
                    const uint32_t first = (uint32_t)j + 1u - nin;
                    for (uint32_t t = 0; t < nin; ++t) {
                        const uint32_t ut = field(U2, t, ra);
                        uint32_t mu = ut;
                        if (ra.c && t + 1 < nin) mu = correct_arith(ut, field(U2, t + 1, ra), ra);
                        v |= mu << (8 * (first + t));
                    }
                    word = 0;
                    nin = 0;
                }
            }
            if (row >= ge.m) continue;
            uint8_t* out = ge.C + (size_t)row * ge.ldc + col0;
            if (col0 + TN <= ge.n && ((uintptr_t)out & (TN - 1)) == 0) {
                if (TN == 4) *reinterpret_cast<uint32_t*>(out) = v;
                else *reinterpret_cast<uint16_t*>(out) = (uint16_t)v;
            } else {
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    if (col0 + j < ge.n) out[j] = (uint8_t)(v >> (8 * j));
            }
        }
    }
}

// Pack one 256-word block of the operands of a product (A blocks first),
// into the tile-major layouts above.
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
    uint32_t tm;      // rows per row block of CA
    uint32_t cbw;     // columns per column block of CB (64 TN)
    uint32_t al;      // bit 0: A and lda 4-byte aligned; bit 1: B and ldb 4-byte aligned
};

// Words packed per thread: four (one 16-byte store) for the four- and
// eight-entry layouts, one for the one-entry layout.
__host__ __device__ inline uint32_t pack_words_per_thread(uint32_t op) { return op == OP_MAD ? 1u : 4u; }
__host__ __device__ inline uint32_t pack_blocks_for(uint64_t words, uint32_t op) {
    const uint64_t per_block = 256ull * pack_words_per_thread(op);
    return (uint32_t)((words + per_block - 1) / per_block);
}

__device__ __forceinline__ uint32_t pack_a_word(uint32_t op, uint32_t b, const uint32_t (&e)[4]) {
    if (op == OP_DOT2) return ((e[0] << b) | e[1]) | (((e[2] << b) | e[3]) << 16);
    if (op == OP_DOT4) return e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
    return e[0];
}

__device__ __forceinline__ uint32_t pack_b_word(uint32_t op, uint32_t b, const uint32_t (&e)[4]) {
    if (op == OP_DOT2) return (e[0] | (e[1] << b)) | ((e[2] | (e[3] << b)) << 16);
    if (op == OP_DOT4) return e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
    return e[0];
}

// Four entries (one k-group) of a row of A, or of four rows of B at one column
// group, as dwords: whole-dword loads when aligned and inside the matrix.
__device__ __forceinline__ uint32_t row_group(const uint8_t* p, uint32_t k0, uint32_t kdim, bool aligned) {
    if (aligned && k0 + 3 < kdim) return *reinterpret_cast<const uint32_t*>(p + k0);
    uint32_t d = 0;
    for (uint32_t x = 0; x < 4; ++x)
        if (k0 + x < kdim) d |= (uint32_t)p[k0 + x] << (8 * x);
    return d;
}

__device__ __forceinline__ void gemm_pack_block4(const PackArgs& a, uint32_t blk, uint32_t tid) {
    if (blk < a.nba) {
        // words w0 .. w0+3 of CA: rows i0 .. i0+3 of row block rb at k-group kw
        const uint64_t w0 = ((uint64_t)blk * 256 + tid) * 4;
        if (w0 >= (uint64_t)a.KW * a.m_pad) return;
        const uint32_t i0 = (uint32_t)(w0 % a.tm);
        const uint64_t q = w0 / a.tm;
        const uint32_t kw = (uint32_t)(q % a.KW), row0 = (uint32_t)(q / a.KW) * a.tm + i0;
        uint4 out;
        uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            const uint32_t row = row0 + x;
            const uint32_t d = row < a.m ? row_group(a.A + (size_t)row * a.lda, 4 * kw, a.kdim, a.al & 1u) : 0u;
            const uint32_t e[4] = {d & 0xFF, (d >> 8) & 0xFF, (d >> 16) & 0xFF, d >> 24};
            o[x] = pack_a_word(a.op, a.b, e);
        }
        *reinterpret_cast<uint4*>(a.CA + w0) = out;
    } else {
        // words w0 .. w0+3 of CB: columns c0 .. c0+3 of column block cb at k-group kw
        const uint64_t w0 = ((uint64_t)(blk - a.nba) * 256 + tid) * 4;
        if (w0 >= (uint64_t)a.KW * a.n_pad) return;
        const uint32_t c0 = (uint32_t)(w0 % a.cbw);
        const uint64_t q = w0 / a.cbw;
        const uint32_t kw = (uint32_t)(q % a.KW), col0 = (uint32_t)(q / a.KW) * a.cbw + c0;
        uint32_t d[4];
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            const uint32_t k = 4 * kw + x;
            d[x] = k < a.kdim ? row_group(a.B + (size_t)k * a.ldb, col0, a.n, a.al & 2u) : 0u;
        }
        uint4 out;
        uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t e[4] = {(d[0] >> (8 * j)) & 0xFF, (d[1] >> (8 * j)) & 0xFF, (d[2] >> (8 * j)) & 0xFF,
                                   (d[3] >> (8 * j)) & 0xFF};
            o[j] = pack_b_word(a.op, a.b, e);
        }
        *reinterpret_cast<uint4*>(a.CB + w0) = out;
    }
}

// Four bytes (each below 16) as four nibbles.
__device__ __forceinline__ uint32_t nibbles4(uint32_t d) {
    return (d & 0xFu) | ((d >> 4) & 0xF0u) | ((d >> 8) & 0xF00u) | ((d >> 12) & 0xF000u);
}

// Eight-entry layout (v_dot8_u32_u4, p <= 16): a word holds the entries of
// eight consecutive k as nibbles, entry 8 kw + x at bits 4x.  Four words per
// thread, as gemm_pack_block4.
__device__ __forceinline__ void gemm_pack_block8(const PackArgs& a, uint32_t blk, uint32_t tid) {
    if (blk < a.nba) {
        // words w0 .. w0+3 of CA: rows i0 .. i0+3 of row block rb at k-group kw
        const uint64_t w0 = ((uint64_t)blk * 256 + tid) * 4;
        if (w0 >= (uint64_t)a.KW * a.m_pad) return;
        const uint32_t i0 = (uint32_t)(w0 % a.tm);
        const uint64_t q = w0 / a.tm;
        const uint32_t kw = (uint32_t)(q % a.KW), row0 = (uint32_t)(q / a.KW) * a.tm + i0;
        uint4 out;
        uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            const uint32_t row = row0 + x;
            uint32_t lo = 0, hi = 0;
            if (row < a.m) {
                const uint8_t* r = a.A + (size_t)row * a.lda;
                lo = row_group(r, 8 * kw, a.kdim, a.al & 1u);
                hi = row_group(r, 8 * kw + 4, a.kdim, a.al & 1u);
            }
            o[x] = nibbles4(lo) | (nibbles4(hi) << 16);
        }
        *reinterpret_cast<uint4*>(a.CA + w0) = out;
    } else {
        // words w0 .. w0+3 of CB: columns c0 .. c0+3 of column block cb at k-group kw
        const uint64_t w0 = ((uint64_t)(blk - a.nba) * 256 + tid) * 4;
        if (w0 >= (uint64_t)a.KW * a.n_pad) return;
        const uint32_t c0 = (uint32_t)(w0 % a.cbw);
        const uint64_t q = w0 / a.cbw;
        const uint32_t kw = (uint32_t)(q % a.KW), col0 = (uint32_t)(q / a.KW) * a.cbw + c0;
        uint32_t d[8];
#pragma unroll
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t k = 8 * kw + x;
            d[x] = k < a.kdim ? row_group(a.B + (size_t)k * a.ldb, col0, a.n, a.al & 2u) : 0u;
        }
        uint4 out;
        uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            uint32_t w = 0;
#pragma unroll
            for (uint32_t x = 0; x < 8; ++x) w |= ((d[x] >> (8 * j)) & 0xFu) << (4 * x);
            o[j] = w;
        }
        *reinterpret_cast<uint4*>(a.CB + w0) = out;
    }
}

__device__ __forceinline__ void gemm_pack_block(const PackArgs& a, uint32_t blk, uint32_t tid) {
    const uint32_t epw = entries_per_word(a.op);
    if (epw == 8) {
        gemm_pack_block8(a, blk, tid);
        return;
    }
    if (epw == 4) {
        gemm_pack_block4(a, blk, tid);
        return;
    }
    if (blk < a.nba) {
        // word index t = (rb KW + kw) tm + i (stores coalesced)
        const uint64_t t = (uint64_t)blk * 256 + tid;
        if (t >= (uint64_t)a.KW * a.m_pad) return;
        const uint32_t i = (uint32_t)(t % a.tm);
        const uint64_t q = t / a.tm;
        const uint32_t kw = (uint32_t)(q % a.KW), row = (uint32_t)(q / a.KW) * a.tm + i;
        uint32_t e[4] = {0, 0, 0, 0};
        if (row < a.m)
            for (uint32_t x = 0; x < epw; ++x) {
                const uint32_t k = kw * epw + x;
                if (k < a.kdim) e[x] = a.A[(size_t)row * a.lda + k];
            }
        a.CA[t] = pack_a_word(a.op, a.b, e);
    } else {
        // word index t = (cb KW + kw) cbw + c
        const uint64_t t = (uint64_t)(blk - a.nba) * 256 + tid;
        if (t >= (uint64_t)a.KW * a.n_pad) return;
        const uint32_t c = (uint32_t)(t % a.cbw);
        const uint64_t q = t / a.cbw;
        const uint32_t kw = (uint32_t)(q % a.KW), col = (uint32_t)(q / a.KW) * a.cbw + c;
        uint32_t e[4] = {0, 0, 0, 0};
        if (col < a.n)
            for (uint32_t x = 0; x < epw; ++x) {
                const uint32_t k = kw * epw + x;
                if (k < a.kdim) e[x] = a.B[(size_t)k * a.ldb + col];
            }
        a.CB[t] = pack_b_word(a.op, a.b, e);
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
    uint32_t er, ec;    // rows / columns of the operands per word (matrix-core compressed products)
    size_t ws_bytes;
};
// Compressed products on the FP64 matrix cores (dqt_fgemm_f64.hip).
dqt_status f64_plan(uint32_t algo, uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint32_t want_b,
                    uint32_t want_ks, GemmPlanResolved* r);
size_t f64_side_bytes(const GemmPlanResolved& r, int side);
dqt_status f64_pack_enqueue(const GemmPlanResolved& r, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A,
                            uint64_t lda, const uint8_t* B, uint64_t ldb, void* pA, void* pB, hipStream_t s);
dqt_status f64_compute_enqueue(const GemmPlanResolved& r, uint32_t p, uint64_t m, uint64_t n, uint8_t* C, uint64_t ldc,
                               const void* pA, const void* pB, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Plain product on the INT8 matrix cores (dqt_gemm_mfma.hip).
dqt_status mfma_plan(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, GemmPlanResolved* r);
size_t mfma_side_bytes(const GemmPlanResolved& r, int side);
dqt_status mfma_pack_enqueue(const GemmPlanResolved& r, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A,
                             uint64_t lda, const uint8_t* B, uint64_t ldb, void* pA, void* pB, hipStream_t s);
dqt_status mfma_compute_enqueue(const GemmPlanResolved& r, uint32_t p, uint64_t m, uint64_t n, uint8_t* C,
                                uint64_t ldc, const void* pA, const void* pB, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1);
inline bool is_f64_algo(uint32_t algo) {
    return algo == DQT_GEMM_RIGHT || algo == DQT_GEMM_LEFT || algo == DQT_GEMM_FULL;
}
dqt_status fgemm_resolve(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan* plan,
                         GemmPlanResolved* r);
// Epilogue parameters (REDQ_e word layout) of a resolved plan.
dqt_status fgemm_epilogue_args(uint32_t p, uint64_t kdim, const GemmPlanResolved& r, GemmArgs* g);

}  // namespace dqt
