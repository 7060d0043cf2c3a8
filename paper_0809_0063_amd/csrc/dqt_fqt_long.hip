// Long polynomial products (more than 64 coefficients) by the FQT (section
// 5.2 of the paper), and their plain per-coefficient comparator.
//
// FQT: each operand is cut into blocks of BS = d+1 coefficients, block i
// holding coefficients i BS .. i BS + BS - 1 as the q-adic word
// sum_s a_{i BS + s} q^s with q = 2^b, kept as a binary64 in LDS.  Output
// block u, W_u = sum_i A_i B_{u-i}, is accumulated by binary64 FMAs (exact:
// every partial sum stays below 2^51), L block products at a time: with
// q > L BS (p-1)^2 no digit of the sum reaches q (eq:bounds), so one
// REDQ_{2BS-1} of the sum gives the 2BS-1 residues of its coefficients
// (section 5.3 counts these reductions).  The residues of the sums of one
// block are added mod p in byte lanes; the top BS-1 residues of block u fall on
// the first BS-1 coefficients of block u+1 and are added mod p when the
// coefficients are written.
//
// Work split (both kernels): a thread owns R consecutive outputs (output
// blocks for the FQT, coefficients for the plain one), a "chunk".  The number
// of terms of a chunk rises and falls along the product, so chunk c is paired
// with chunk C-1-c (or, within one wave, with chunk c + C/2) on the same
// thread: every thread then has about the same number of terms, and one pair
// per thread covers products of up to 4096 coefficients with at most 512
// threads.  Products of up to 32 chunk pairs share a wave, as many as have a
// lane for each of their pairs (64 / pairs of them), each with its own slot of
// LDS; a larger product has a wave (up to 64 pairs) or a workgroup to itself.
// The FQT kernel puts four waves of the first two kinds in a workgroup, which
// share one correction table.  The
// terms are taken G at a time: G values of a and the G+R-1 values of b that
// meet them are read from LDS once and used G R times.  The operands sit in LDS
// between zeros, so groups that overlap the ends of the operands need no test.
//
// The plain comparator keeps the coefficients as 32-bit values and does one
// v_mad_u32_u24 per coefficient product (the sums stay below
// 4096 (p-1)^2 < 2^32) and one reduction per output.

#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>

#include "dqt_internal.h"

namespace dqt {

namespace {

constexpr int kPlainR = 8;         // coefficients per plain chunk
constexpr int kPlainG = 8;         // terms per plain group
constexpr uint32_t kPad = 16;      // zeros in LDS before b (>= R + G - 2 for both kernels)

// LDS positions with one unused slot after every 2^S entries.  The lanes of a
// wave read b windows R entries apart (and the plain kernel's a values 8
// apart); without the gaps those strides put 4 lanes of every 16 on the same
// banks, with them the lanes of a 16-lane phase hit distinct banks.  Every
// window starts at an index = 1 mod 2^S (kPad - (G - 1) = 1 mod 4 for G = 4, 8;
// 16 - 7 = 1 mod 8 for the plain kernel), so the offset of its entry x from
// its start, x + ((1 + x) >> S), is a constant.
template <int S>
__host__ __device__ constexpr uint32_t gapped(uint32_t d) { return d + (d >> S); }
template <int S>
__device__ constexpr uint32_t gap_off(int x) { return (uint32_t)x + ((1u + (uint32_t)x) >> S); }
__host__ __device__ constexpr uint32_t gapped_n(int s, uint32_t d) { return d + (d >> s); }
// Gap spacing of the FQT's B rows for chunks of R blocks and term groups of G:
// windows start at kPad - (G - 1) + (multiple of R, G), 1 mod 8 only when G = 8.
__host__ __device__ constexpr int long_gap_shift(int r, int g) { return r == 8 && g == 8 ? 3 : 2; }

struct LongArgs {
    uint32_t na, nb, nout;
    uint32_t b;                     // log2 q
    uint32_t Na, Nb, NW;            // blocks of A, of B, output blocks
    uint32_t L;                     // block products per REDQ (a multiple of G)
    uint32_t C;                     // chunks of R output blocks (block NW, all zero, included)
    uint32_t na_pad, nb_tot;        // doubles of A (a multiple of G) and of B with its zeros
    uint32_t lds_a, lds_b, lds_bnd; // byte offsets in LDS: A words, B words, last residues of each chunk
    uint32_t tpp, ppw, pp_bytes;    // threads per product, products per wave (1 above 64 threads),
                                    // LDS bytes per product
    uint32_t ppg;                   // products per workgroup
    RedqArgs ra;
};

// coefficient-wise a + b mod p on byte lanes (each lane < p <= 127)
__device__ __forceinline__ uint64_t add_mod_lanes(uint64_t a, uint64_t b, uint32_t p) {
    const uint64_t ones = 0x0101010101010101ull;
    const uint64_t s = a + b;
    const uint64_t t = s + (uint64_t)(128 - p) * ones;
    return s - (uint64_t)p * ((t >> 7) & ones);
}

// the integer x < 2^52 held by a binary64
__device__ __forceinline__ uint64_t exact_u52(double x) {
    return __builtin_bit_cast(uint64_t, x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// Smallest / largest value over the 64 lanes of the wave (the same result in every lane).
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

// QB, QW: log2 q and the residue width as compile-time constants (0 = from the
// run-time arguments).
template <int BS, int G, int QB, int QW, int R, bool ONE>
__global__ __launch_bounds__(512) void k_polymul_fqt_long(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                          uint8_t* __restrict__ OUT, uint64_t count, LongArgs g) {
    constexpr int NR = 2 * BS - 1;
    static_assert(R + G - 2 <= (int)kPad, "the B windows stay inside the zeros around B");
    // B rows: a gap every 2^GS words, GS = log2 R for R = 4, and for R = 8 when G = 8 (the
    // windows then start at 1 mod 8); lanes read windows R words apart
    constexpr int GS = long_gap_shift(R, G);
    extern __shared__ __attribute__((aligned(16))) uint8_t lsm[];
    uint16_t* tab = reinterpret_cast<uint16_t*>(lsm);
    // Products of up to 64 chunk pairs share waves (tpp <= 64): each wave of the workgroup holds
    // ppw products of tpp lanes, the lanes past ppw tpp (when tpp does not divide 64) take none,
    // and the waves share the correction table.  A larger product (tpp = blockDim.x > 64) has
    // the workgroup to itself.  Each product has its own LDS slot.
    const bool shared = g.tpp <= 64;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t subw = shared ? lane / g.tpp : 0;
    const uint32_t pair = shared ? lane - subw * g.tpp : threadIdx.x;
    const bool has_slot = subw < g.ppw;
    const uint32_t sub = (shared ? (threadIdx.x >> 6) * g.ppw : 0) + (has_slot ? subw : 0);
    uint8_t* slot = lsm + g.lds_a + sub * g.pp_bytes;
    double* ad = reinterpret_cast<double*>(slot);
    double* bd = reinterpret_cast<double*>(slot + (g.lds_b - g.lds_a));   // bd[gapped<GS>(kPad + i)] = B_i
    uint64_t* bnd = reinterpret_cast<uint64_t*>(slot + (g.lds_bnd - g.lds_a));
    const RedqArgs& ra = g.ra;
    build_correction_table(tab, ra);
    // Two chunks per lane.  ONE: chunk c with chunk c + ceil(C/2) (the number of terms of a
    // chunk rises along the first half of the product and falls along the second, so the two
    // add up to about the same for every lane), walked as one sequence per lane, each sum
    // reduced once at the end (only when no sum needs an earlier reduction, L >= its terms).
    // Otherwise chunk c with chunk C-1-c, in two wave-wide phases (below).
    const uint32_t half = (g.C + 1) / 2;
    const uint32_t cs[2] = {pair, ONE ? pair + half : g.C - 1 - pair};
    const int nc_all = ONE ? (pair < half ? (cs[1] < g.C ? 2 : 1) : 0)
                           : (pair < (g.C + 1) / 2 ? (cs[1] > pair ? 2 : 1) : 0);
    // one REDQ_{2BS-1} of each of the R sums; their residues added to res
    auto reduce = [&](double (&W)[R], uint64_t (&res)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t U = redq_compress_t<NR, QB, QW, true>(exact_u52(W[r]), ra);
            uint64_t v = 0;
            redq_correct<NR, QB, QW>(U, ra, tab, [&](int s, uint32_t m) { v |= (uint64_t)m << (8 * s); });
            res[r] = add_mod_lanes(res[r], v, ra.p);
            W[r] = 0.0;
        }
    };
    for (uint64_t t0 = (uint64_t)blockIdx.x * g.ppg; t0 < count; t0 += (uint64_t)gridDim.x * g.ppg) {
        const uint64_t t = t0 + sub;
        const bool live = has_slot && t < count;
        const int nc = live ? nc_all : 0;
        __syncthreads();   // the table is built / the previous products have left LDS
        const uint8_t* a = A + (live ? t : 0) * g.na;
        const uint8_t* b = B + (live ? t : 0) * g.nb;
        for (uint32_t i = live ? pair : g.na_pad; i < g.na_pad; i += g.tpp) {
            uint64_t w = 0;
#pragma unroll
            for (int s = 0; s < BS; ++s) {
                const uint32_t c = i * BS + s;
                if (c < g.na) w |= (uint64_t)a[c] << (g.b * s);
            }
            ad[i] = (double)w;
        }
        for (uint32_t k = live ? pair : g.nb_tot; k < g.nb_tot; k += g.tpp) {
            uint64_t w = 0;
            const uint32_t i = k - kPad;
            if (k >= kPad && i < g.Nb) {
#pragma unroll
                for (int s = 0; s < BS; ++s) {
                    const uint32_t c = i * BS + s;
                    if (c < g.nb) w |= (uint64_t)b[c] << (g.b * s);
                }
            }
            bd[gapped<GS>(k)] = (double)w;
        }
        __syncthreads();
        if constexpr (ONE) {
            // term groups of chunk c: from ilo (rounded down to G) to ihi
            uint32_t lo[2] = {0, 0}, ng[2] = {0, 0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nc) continue;
                const uint32_t u0 = cs[h] * R;
                const uint32_t ilo = u0 + 1 > g.Nb ? u0 + 1 - g.Nb : 0;
                const uint32_t ihi = min(g.Na - 1, u0 + R - 1);
                lo[h] = ilo & ~(uint32_t)(G - 1);
                ng[h] = ihi >= lo[h] ? (ihi - lo[h]) / G + 1 : 0;
            }
            double W[R], WA[R];
#pragma unroll
            for (int r = 0; r < R; ++r) W[r] = WA[r] = 0.0;
            const uint32_t ntot = ng[0] + ng[1];
            for (uint32_t k = 0; k < ntot; ++k) {
                const bool inA = k < ng[0];
                if (k == ng[0]) {   // the first chunk is done: keep its sums, start the second
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        WA[r] = W[r];
                        W[r] = 0.0;
                    }
                }
                const uint32_t ig = inA ? lo[0] + k * G : lo[1] + (k - ng[0]) * G;
                const uint32_t u0 = (inA ? cs[0] : cs[1]) * R;
                double av[G], wv[G + R - 1];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2) av[s2] = ad[ig + s2];
                // wv[x] = B_{u0 - ig - (G-1) + x}
                const double* wb = bd + gapped<GS>(kPad + u0 - ig - (G - 1));
#pragma unroll
                for (int x = 0; x < G + R - 1; ++x) wv[x] = wb[gap_off<GS>(x)];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2)
#pragma unroll
                    for (int r = 0; r < R; ++r) W[r] = __builtin_fma(av[s2], wv[r - s2 + G - 1], W[r]);
            }
            if (ng[1] == 0) {   // one chunk only: its sums are still in W
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    WA[r] = W[r];
                    W[r] = 0.0;
                }
            }
            uint64_t res0[R], res1[R];
#pragma unroll
            for (int r = 0; r < R; ++r) res0[r] = res1[r] = 0;
            reduce(WA, res0);   // every lane, at the same point of the code
            reduce(W, res1);
            if (nc >= 1) bnd[cs[0]] = res0[R - 1];
            if (nc >= 2) bnd[cs[1]] = res1[R - 1];
            __syncthreads();
            uint8_t* o = OUT + t * g.nout;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nc) break;
                const uint32_t c = cs[h];
                uint64_t prev = c ? bnd[c - 1] : 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t u = c * R + r;
                    const uint64_t cur = h == 0 ? res0[r] : res1[r];
#pragma unroll
                    for (int s = 0; s < BS; ++s) {
                        const uint32_t j = u * BS + s;
                        uint32_t v = (uint32_t)(cur >> (8 * s)) & 0xFFu;
                        if (s + BS < NR) v += (uint32_t)(prev >> (8 * (s + BS))) & 0xFFu;
                        if (j < g.nout) o[j] = (uint8_t)(v >= ra.p ? v - ra.p : v);
                    }
                    prev = cur;
                }
            }
            continue;
        }
        // Each phase ends with its chunk written: the last block residues of every chunk
        // go to bnd first, and after a barrier each lane writes its chunk (chunk c - 1 of a
        // phase-1 chunk is a phase-1 chunk or the last phase-0 one, both in bnd by then).
        // So one phase's residues are held in registers at a time.
        uint8_t* o = OUT + t * g.nout;
        // (a loop, not unrolled: one copy of the phase keeps the register count down)
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const uint32_t ch = h == 0 ? cs[0] : cs[1];   // this phase's chunk (no indexed array)
            // The wave walks one common sequence of term groups (from the smallest first group
            // of its lanes to the largest last one); a lane multiplies only in its own groups.
            // The sums are reduced at multiples of L in the common sequence, so every lane of
            // the wave reduces at the same time and each sum holds at most L block products.
            const bool mine = h < nc;
            const uint32_t u0 = mine ? ch * R : 0;
            const uint32_t ilo = u0 + 1 > g.Nb ? u0 + 1 - g.Nb : 0;
            const uint32_t ihi = min(g.Na - 1, u0 + R - 1);
            const uint32_t lo = mine ? (ilo & ~(uint32_t)(G - 1)) : 0xFFFFFFFFu;
            const uint32_t hi = mine ? ihi : 0u;
            const uint32_t wlo = wave_min(lo), whi = wave_max(hi);
            double W[R];
            uint64_t res[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                W[r] = 0.0;
                res[r] = 0;
            }
            if (wlo <= whi) {
                uint32_t next_red = (wlo / g.L + 1) * g.L;
                for (uint32_t ig = wlo; ig <= whi; ig += G) {
                    if (ig >= lo && ig <= hi) {
                        double av[G], wv[G + R - 1];
#pragma unroll
                        for (int s = 0; s < G; ++s) av[s] = ad[ig + s];
                        // wv[x] = B_{u0 - ig - (G-1) + x}
                        const double* wb = bd + gapped<GS>(kPad + u0 - ig - (G - 1));
#pragma unroll
                        for (int x = 0; x < G + R - 1; ++x) wv[x] = wb[gap_off<GS>(x)];
#pragma unroll
                        for (int s = 0; s < G; ++s)
#pragma unroll
                            for (int r = 0; r < R; ++r) W[r] = __builtin_fma(av[s], wv[r - s + G - 1], W[r]);
                    }
                    if (ig + G == next_red) {
                        next_red += g.L;
                        reduce(W, res);
                    }
                }
                reduce(W, res);
            }
            if (mine) bnd[ch] = res[R - 1];
            __syncthreads();
            if (!mine) continue;
            // coefficient j = u BS + s: residue s of block u plus residue s + BS of block u - 1
            const uint32_t c = ch;
            uint64_t prev = c ? bnd[c - 1] : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t u = c * R + r;
                const uint64_t cur = res[r];
#pragma unroll
                for (int s = 0; s < BS; ++s) {
                    const uint32_t j = u * BS + s;
                    uint32_t v = (uint32_t)(cur >> (8 * s)) & 0xFFu;
                    if (s + BS < NR) v += (uint32_t)(prev >> (8 * (s + BS))) & 0xFFu;
                    if (j < g.nout) o[j] = (uint8_t)(v >= ra.p ? v - ra.p : v);
                }
                prev = cur;
            }
        }
    }
}

// Plain per-coefficient products c_j = sum_i a_i b_{j-i}; chunk c owns j = 8c .. 8c + 7.
template <bool ONE>
__global__ __launch_bounds__(512) void k_polymul_plain_long(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                            uint8_t* __restrict__ OUT, uint64_t count, uint32_t na,
                                                            uint32_t nb, uint32_t p, uint32_t pmagic, uint32_t na_pad,
                                                            uint32_t nb_tot, uint32_t tpp, uint32_t ppw,
                                                            uint32_t slot_words) {
    constexpr int R = kPlainR, G = kPlainG;
    extern __shared__ __attribute__((aligned(16))) uint8_t lsm[];
    // as in the FQT kernel: tpp threads and one LDS slot per product, ppw products per workgroup,
    // no product on the lanes past ppw tpp
    const uint32_t sub = threadIdx.x / tpp;
    const uint32_t pair = threadIdx.x - sub * tpp;
    const bool has_slot = sub < ppw;
    uint32_t* a32 = reinterpret_cast<uint32_t*>(lsm) + (has_slot ? sub : 0) * slot_words;   // a32[gapped<3>(i)] = a_i, zeros up to na_pad
    uint32_t* b32 = a32 + gapped<3>(na_pad);              // b32[gapped<3>(kPad + k)] = b_k, zeros around
    const uint32_t nout = na + nb - 1;
    const uint32_t C = (nout + R - 1) / R;
    // ONE: chunk c with chunk c + ceil(C/2), walked as one sequence per lane (as the FQT kernel's
    // single walk); else chunk c with chunk C - 1 - c, each walked by a loop of its own. Either
    // way the two chunks of a lane add up to about the same number of terms.
    const uint32_t half = (C + 1) / 2;
    const uint32_t cs[2] = {pair, ONE ? pair + half : C - 1 - pair};
    const int nc_all = ONE ? (pair < half ? (cs[1] < C ? 2 : 1) : 0) : (pair < half ? (cs[1] > pair ? 2 : 1) : 0);
    for (uint64_t t0 = (uint64_t)blockIdx.x * ppw; t0 < count; t0 += (uint64_t)gridDim.x * ppw) {
        const uint64_t t = t0 + sub;
        const bool live = has_slot && t < count;
        const int nc = live ? nc_all : 0;
        __syncthreads();
        const uint8_t* a = A + (live ? t : 0) * na;
        const uint8_t* b = B + (live ? t : 0) * nb;
        for (uint32_t i = live ? pair : na_pad; i < na_pad; i += tpp) a32[gapped<3>(i)] = i < na ? a[i] : 0u;
        for (uint32_t k = live ? pair : nb_tot; k < nb_tot; k += tpp)
            b32[gapped<3>(k)] = (k >= kPad && k - kPad < nb) ? b[k - kPad] : 0u;
        __syncthreads();
        uint8_t* o = OUT + t * nout;
        if (!ONE) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nc) break;
                const uint32_t j0 = cs[h] * R;
                // i with 0 <= j - i < nb for some j in [j0, j0 + R): j0 - nb < i <= j0 + R - 1
                const uint32_t ilo = j0 + 1 > nb ? j0 + 1 - nb : 0;
                const uint32_t ihi = min(na - 1, j0 + R - 1);
                uint32_t c[R];
#pragma unroll
                for (int r = 0; r < R; ++r) c[r] = 0;
                for (uint32_t ig = ilo & ~(uint32_t)(G - 1); ig <= ihi; ig += G) {
                    uint32_t av[G], wv[G + R - 1];
#pragma unroll
                    for (int s = 0; s < G; ++s) av[s] = a32[gapped<3>(ig) + s];   // ig = 0 mod 8
                    // wv[x] = b_{j0 - ig - (G-1) + x}
                    const uint32_t* wb = b32 + gapped<3>(kPad + j0 - ig - (G - 1));
#pragma unroll
                    for (int x = 0; x < G + R - 1; ++x) wv[x] = wb[gap_off<3>(x)];
#pragma unroll
                    for (int s = 0; s < G; ++s)
#pragma unroll
                        for (int r = 0; r < R; ++r) c[r] = __umul24(av[s], wv[r - s + G - 1]) + c[r];
                }
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (j0 + r < nout) o[j0 + r] = (uint8_t)mod_small(c[r] > 0xFFFFFFu ? c[r] % p : c[r], p, pmagic);
            }
            continue;
        }
        // the same ranges of i, for both chunks, then one loop over both
        uint32_t lo[2] = {0, 0}, ng[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nc) continue;
            const uint32_t j0 = cs[h] * R;
            const uint32_t ilo = j0 + 1 > nb ? j0 + 1 - nb : 0;
            const uint32_t ihi = min(na - 1, j0 + R - 1);
            lo[h] = ilo & ~(uint32_t)(G - 1);
            ng[h] = ihi >= lo[h] ? (ihi - lo[h]) / G + 1 : 0;
        }
        uint32_t c[R], cA[R];
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = cA[r] = 0;
        const uint32_t ntot = ng[0] + ng[1];
        for (uint32_t k = 0; k < ntot; ++k) {
            const bool inA = k < ng[0];
            if (k == ng[0]) {   // the first chunk is done: keep its sums, start the second
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cA[r] = c[r];
                    c[r] = 0;
                }
            }
            const uint32_t ig = inA ? lo[0] + k * G : lo[1] + (k - ng[0]) * G;
            const uint32_t j0 = (inA ? cs[0] : cs[1]) * R;
            uint32_t av[G], wv[G + R - 1];
#pragma unroll
            for (int s = 0; s < G; ++s) av[s] = a32[gapped<3>(ig) + s];   // ig = 0 mod 8
            // wv[x] = b_{j0 - ig - (G-1) + x}
            const uint32_t* wb = b32 + gapped<3>(kPad + j0 - ig - (G - 1));
#pragma unroll
            for (int x = 0; x < G + R - 1; ++x) wv[x] = wb[gap_off<3>(x)];
#pragma unroll
            for (int s = 0; s < G; ++s)
#pragma unroll
                for (int r = 0; r < R; ++r) c[r] = __umul24(av[s], wv[r - s + G - 1]) + c[r];
        }
        if (ng[1] == 0) {   // one chunk only: its sums are still in c
#pragma unroll
            for (int r = 0; r < R; ++r) cA[r] = c[r];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nc) break;
            const uint32_t j0 = cs[h] * R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t v = h == 0 ? cA[r] : c[r];
                if (j0 + r < nout) o[j0 + r] = (uint8_t)mod_small(v > 0xFFFFFFu ? v % p : v, p, pmagic);
            }
        }
    }
}

}  // namespace

static constexpr uint32_t kLongMaxCoeffs = 4096;

// LDS bytes of the correction table at the start of a workgroup's LDS: its entries as 16-bit
// words (64 for F_3 with windows of three residues, up to 4096; none where the correction is
// computed), rounded to 16 bytes.
static uint32_t long_table_bytes(const RedqArgs& ra) { return (ra.tab_entries * 2u + 15u) & ~15u; }

// LDS layout and launch shape of a long product for one block size, group width G and chunk size R.
struct LongShape {
    uint32_t Na, Nb, NW, C, pairs;
    uint32_t na_pad, nb_tot, lds_b, lds_bnd, pp_bytes;
    uint32_t tpp, ppw, ppg, threads;
    size_t smem;
};

static LongShape long_shape(uint32_t na, uint32_t nb, uint32_t bs, uint32_t G, uint32_t R, uint32_t lds_a) {
    LongShape h;
    h.Na = (na + bs - 1) / bs;
    h.Nb = (nb + bs - 1) / bs;
    h.NW = h.Na + h.Nb - 1;
    // chunks of R output blocks (blocks 0 .. NW; block NW only carries the top residues of NW-1)
    h.C = (h.NW + 1 + R - 1) / R;
    h.pairs = (h.C + 1) / 2;   // one chunk pair per thread
    h.na_pad = (h.Na + G - 1) / G * G;
    h.nb_tot = kPad + h.Nb + kPad;
    h.lds_b = lds_a + h.na_pad * 8;
    h.lds_bnd = h.lds_b + ((gapped_n(long_gap_shift(R, G), h.nb_tot) * 8 + 15) & ~15u);
    h.pp_bytes = (uint32_t)((h.lds_bnd - lds_a + (size_t)h.C * 8 + 15) & ~(size_t)15);
    if (h.pairs <= 64) {
        // Shared waves: 64 / pairs products per wave (a thread for each chunk pair; each product
        // given 64 / ppw threads, the spare ones only stage) and four waves per workgroup sharing
        // one correction table (two or one where their slots would pass 64 KiB of LDS).  With a
        // table per wave, LDS held the kernel to a few waves per CU at these sizes.
        uint32_t wpg = 4;
        h.ppw = h.pairs <= 32 ? 64 / h.pairs : 1;
        while (h.ppw > 1 && lds_a + (size_t)h.ppw * h.pp_bytes > 65536) --h.ppw;
        while (wpg > 1 && lds_a + (size_t)wpg * h.ppw * h.pp_bytes > 65536) wpg /= 2;
        h.tpp = 64 / h.ppw;
        h.ppg = wpg * h.ppw;
        h.threads = 64 * wpg;
    } else {
        h.threads = (h.pairs + 63) / 64 * 64;
        h.tpp = h.threads;
        h.ppw = 1;
        h.ppg = 1;
    }
    h.smem = lds_a + (size_t)h.ppg * h.pp_bytes;
    return h;
}

// F_3 (residues of 2 bits) in blocks of three at q = 2^10 or of two at q = 2^17 (the block
// sizes the cost picks over F_3) have instances with a compile-time q and residue width.
static bool long_f3(uint32_t p, uint32_t bs, uint32_t b, uint32_t G) {
    return p == 3 && G == 8 && ((bs == 3 && b == 10) || (bs == 2 && b == 17));
}

// Vector registers per lane of each instance (its kernel attribute, read once; 128 where it
// cannot be read), for the occupancy term of the cost estimate.
static int long_regs(uint32_t bs, uint32_t G, uint32_t R, bool one, bool f3) {
    static const std::array<int, 64> regs = [] {
        std::array<int, 64> r;
        r.fill(128);
        auto put = [&](int idx, const void* fn) {
            hipFuncAttributes at;
            if (hipFuncGetAttributes(&at, fn) == hipSuccess && at.numRegs > 0) r[idx] = at.numRegs;
            else (void)hipGetLastError();
        };
#define DQT_REGS(BSV, GV, QBV, QWV, RV, ONEV, F3V)                                                             \
    put((((BSV - 2) * 2 + (GV == 8)) * 2 + (RV == 8)) * 4 + (ONEV ? 2 : 0) + (F3V ? 1 : 0),                   \
        reinterpret_cast<const void*>(&k_polymul_fqt_long<BSV, GV, QBV, QWV, RV, ONEV>))
#define DQT_REGS4(BSV, GV, QBV, QWV, F3V)                                                                      \
    DQT_REGS(BSV, GV, QBV, QWV, 4, false, F3V); DQT_REGS(BSV, GV, QBV, QWV, 4, true, F3V);                     \
    DQT_REGS(BSV, GV, QBV, QWV, 8, false, F3V); DQT_REGS(BSV, GV, QBV, QWV, 8, true, F3V)
        DQT_REGS4(2, 8, 17, 2, true);
        DQT_REGS4(3, 8, 10, 2, true);
        DQT_REGS4(2, 4, 0, 0, false);
        DQT_REGS4(2, 8, 0, 0, false);
        DQT_REGS4(3, 4, 0, 0, false);
        DQT_REGS4(3, 8, 0, 0, false);
        DQT_REGS4(4, 4, 0, 0, false);
        DQT_REGS4(4, 8, 0, 0, false);
#undef DQT_REGS4
#undef DQT_REGS
        return r;
    }();
    return regs[(((bs - 2) * 2 + (G == 8)) * 2 + (R == 8)) * 4 + (one ? 2 : 0) + (f3 ? 1 : 0)];
}

// Vector registers per lane of the plain kernel's two instances (as long_regs).
static int plain_long_regs(bool one) {
    static const std::array<int, 2> regs = [] {
        std::array<int, 2> r{128, 128};
        auto put = [&](int idx, const void* fn) {
            hipFuncAttributes at;
            if (hipFuncGetAttributes(&at, fn) == hipSuccess && at.numRegs > 0) r[idx] = at.numRegs;
            else (void)hipGetLastError();
        };
        put(0, reinterpret_cast<const void*>(&k_polymul_plain_long<false>));
        put(1, reinterpret_cast<const void*>(&k_polymul_plain_long<true>));
        return r;
    }();
    return regs[one ? 1 : 0];
}

// Block size, q, L, the group width G and the chunk size R of a long product:
// the smallest estimated cost over block sizes 2..4 (the 2 BS - 1 residues of a
// block stay within the eight byte lanes of one word) and chunks of R = 4 or 8
// output blocks, with q = 2^b, (2 BS - 1) b <= 51 and at least four block
// products per reduction.  p <= 127 (two residues add within a byte lane).  The
// estimate counts what section 5.3's model counts, block products and
// reductions, the way the kernel runs them, in units of one lane's binary64 FMA:
// per wave (or per share of a wave, for products of up to 32 chunk pairs), about
// Na / G term groups per phase of G R FMAs and G + R - 1 B words read from LDS
// (about 2 FMAs' worth each), and a REDQ_{2BS-1} of each of the R sums at every
// L-th term and at the end (about 12 (2 BS - 1) each); that divided by the
// waves per SIMD that registers and LDS let the launch keep resident (counted
// up to four: the kernel waits on LDS and memory, and fewer waves hide less of
// it); plus the product's own loads and stores (19 per 64 bytes) and 8 for its
// set-up.  The weights are a least-squares fit of measured times over F_3
// (21 lengths from 65 to 4096, both chunk sizes, both walks, every block size);
// the choice they give was within 10% of the measured fastest at every one (2%
// on average).
dqt_status fqt_long_plan(uint32_t p, uint32_t na, uint32_t nb, uint32_t block, uint32_t* bs_out, uint32_t* b_out,
                         uint32_t* L_out, uint32_t* G_out, uint32_t* R_out, bool* one_out) {
    if (p > 127) return DQT_E_UNSUPPORTED;
    const uint64_t e2 = (uint64_t)(p - 1) * (p - 1);
    double best = 1e300;
    uint32_t best_bs = 0;
    for (uint32_t bs = 2; bs <= 4; ++bs) {
        if (block && bs != block) continue;
        const uint32_t b = 51 / (2 * bs - 1);
        const uint64_t nq = ((1ull << b) - 1) / ((uint64_t)bs * e2);
        if (nq < 4) continue;
        const uint32_t G = nq >= 8 ? 8 : 4;
        const uint32_t L = (uint32_t)(nq / G) * G;
        RedqArgs ra;
        if (make_redq_args(p, b, 2 * bs - 1, (2 * bs - 1) * b, &ra) != DQT_OK) continue;
        for (uint32_t R = 4; R <= 8; R += 4) {
            const LongShape h = long_shape(na, nb, bs, G, R, long_table_bytes(ra));
            if (h.pairs > 512 || h.threads > 512 || h.smem > 65536) continue;
            // waves per product (a share of one below 65 chunk pairs)
            const double waves = h.pairs <= 64 ? 1.0 / h.ppw : h.threads / 64.0;
            const double span = (double)(h.Na < h.Nb ? h.Na : h.Nb);
            const double groups = 2.0 * std::ceil(span / G);
            const double reductions = 2.0 * (std::floor((span - 1) / L) + 1.0) * R;
            const double io = (na + nb + 2.0 * (na + nb - 1)) / 64.0;
            const uint32_t wpg = h.threads / 64;
            for (int one = 0; one <= 1; ++one) {
                // one sequence per lane over balanced chunks: about (span + R) / G groups per
                // lane instead of two wave-wide walks of span / G, but A words read per lane
                // (not broadcast); only where one reduction per sum suffices (L >= span)
                // (and only within one wave: above 64 pairs the later waves of the wave-wide walk
                // have nearly equal ranges, and measured faster)
                if (one && (L < span || h.pairs > 64)) continue;
                const int regs = long_regs(bs, G, R, one != 0, long_f3(p, bs, b, G));
                const uint32_t by_regs = 512u / (uint32_t)((regs + 7) / 8 * 8);   // waves per SIMD
                const uint32_t groups_cu = std::min<uint32_t>((uint32_t)((160u * 1024u) / h.smem), 4u * by_regs / wpg);
                const double resident = std::max(0.25, std::min(4.0, groups_cu * wpg / 4.0));
                const double gr = one ? std::ceil((span + R) / G) + 2.0 : groups;
                const double reds = one ? 2.0 * R : reductions;
                const double cost = waves * 4.0 / resident *
                                        (gr * R * G + 2.06 * gr * (G + R - 1 + (one ? G : 0)) +
                                         12.35 * reds * (2 * bs - 1)) +
                                    18.7 * io + 8.5;
                if (cost < best) {
                    best = cost;
                    best_bs = bs;
                    *b_out = b;
                    *L_out = L;
                    *G_out = G;
                    *R_out = R;
                    *one_out = one != 0;
                }
            }
        }
    }
    if (!best_bs) return block ? DQT_E_BOUND : DQT_E_UNSUPPORTED;
    *bs_out = best_bs;
    return DQT_OK;
}

// Workgroups per CU that the LDS (160 KiB) and the wave slots allow.
// Workgroups per CU that the LDS (160 KiB), the wave slots and the registers
// (512 per lane of a SIMD, allocated in granules of 8) allow.
static unsigned groups_per_cu(size_t smem, unsigned threads, int regs) {
    const unsigned waves = (threads + 63) / 64;
    const unsigned by_lds = (unsigned)((160u * 1024u) / (smem ? smem : 1));
    const unsigned by_waves = 32u / waves;
    const unsigned by_regs = 4u * std::min(8u, 512u / (unsigned)((regs + 7) / 8 * 8)) / waves;
    const unsigned n = std::min(by_lds, std::min(by_waves, by_regs));
    return n ? n : 1;
}

// A grid of workgroups that loop over `units` (groups of products): no more than
// fit the device at once, and as many units for each of them (without it, e.g.
// 2,048 units on 1,280 workgroups of which 1,024 fit would leave a tail).
static unsigned balanced_grid(uint64_t units, unsigned per_cu) {
    const uint64_t cap = stream_grid(units, 1, per_cu);
    const uint64_t rounds = (units + cap - 1) / cap;
    return (unsigned)((units + rounds - 1) / rounds);
}

dqt_status fqt_long_enqueue(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint64_t count, uint32_t p,
                            uint32_t block, uint8_t* out, hipStream_t s, bool check_only) {
    if (na > kLongMaxCoeffs || nb > kLongMaxCoeffs) return DQT_E_UNSUPPORTED;
    uint32_t bs = 0, b = 0, L = 0, G = 0, R = 0;
    bool one = false;
    DQT_TRY(fqt_long_plan(p, na, nb, block, &bs, &b, &L, &G, &R, &one));
    LongArgs g;
    memset(&g, 0, sizeof(g));
    DQT_TRY(make_redq_args(p, b, 2 * bs - 1, (2 * bs - 1) * b, &g.ra));
    if (check_only) return DQT_OK;
    g.na = na;
    g.nb = nb;
    g.nout = na + nb - 1;
    g.b = b;
    g.L = L;
    const uint32_t lds_a = long_table_bytes(g.ra);
    const LongShape h = long_shape(na, nb, bs, G, R, lds_a);
    g.Na = h.Na;
    g.Nb = h.Nb;
    g.NW = h.NW;
    g.C = h.C;
    g.na_pad = h.na_pad;
    g.nb_tot = h.nb_tot;
    g.lds_a = lds_a;
    g.lds_b = h.lds_b;
    g.lds_bnd = h.lds_bnd;
    g.pp_bytes = h.pp_bytes;
    g.tpp = h.tpp;
    g.ppw = h.ppw;
    g.ppg = h.ppg;
    const unsigned threads = h.threads;
    const size_t smem = h.smem;
    if (threads > 512 || smem > 65536) return DQT_E_UNSUPPORTED;
    const int regs = long_regs(bs, G, R, one, long_f3(p, bs, b, G));
    const unsigned grid = balanced_grid((count + g.ppg - 1) / g.ppg, groups_per_cu(smem, threads, regs));
    // the F_3 instances with a compile-time q and residue width, else the run-time form
    if (long_f3(p, bs, b, G)) {
#define DQT_LONG_F3(BSV, QBV, RV, ONEV)                                                                    \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_long<BSV, 8, QBV, 2, RV, ONEV>), dim3(grid), dim3(threads), \
                       smem, s, A, B, out, count, g)
        const unsigned k3 = (bs == 3 ? 4u : 0u) + (R == 8 ? 2u : 0u) + (one ? 1u : 0u);
        switch (k3) {
            case 0: DQT_LONG_F3(2, 17, 4, false); break;
            case 1: DQT_LONG_F3(2, 17, 4, true); break;
            case 2: DQT_LONG_F3(2, 17, 8, false); break;
            case 3: DQT_LONG_F3(2, 17, 8, true); break;
            case 4: DQT_LONG_F3(3, 10, 4, false); break;
            case 5: DQT_LONG_F3(3, 10, 4, true); break;
            case 6: DQT_LONG_F3(3, 10, 8, false); break;
            default: DQT_LONG_F3(3, 10, 8, true); break;
        }
#undef DQT_LONG_F3
        DQT_LAUNCH_CHECK("dqt_polymul_fqt_u8 (long)");
        return DQT_OK;
    }
    const unsigned key = bs * 1024 + G * 64 + R * 2 + (one ? 1u : 0u);
    switch (key) {
#define DQT_LONG_CASE(BSV, GV, RV, ONEV)                                                                          \
    case BSV * 1024 + GV * 64 + RV * 2 + (ONEV ? 1 : 0):                                                          \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_long<BSV, GV, 0, 0, RV, ONEV>), dim3(grid), dim3(threads), \
                           smem, s, A, B, out, count, g);                                                         \
        break;
#define DQT_LONG_CASES(BSV, GV) \
    DQT_LONG_CASE(BSV, GV, 4, false) DQT_LONG_CASE(BSV, GV, 4, true) DQT_LONG_CASE(BSV, GV, 8, false) DQT_LONG_CASE(BSV, GV, 8, true)
        DQT_LONG_CASES(2, 4)
        DQT_LONG_CASES(2, 8)
        DQT_LONG_CASES(3, 4)
        DQT_LONG_CASES(3, 8)
        DQT_LONG_CASES(4, 4)
        DQT_LONG_CASES(4, 8)
#undef DQT_LONG_CASES
#undef DQT_LONG_CASE
        default: return DQT_E_UNSUPPORTED;
    }
    DQT_LAUNCH_CHECK("dqt_polymul_fqt_u8 (long)");
    return DQT_OK;
}

dqt_status plain_long_enqueue(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint64_t count, uint32_t p,
                              uint8_t* out, hipStream_t s) {
    if (na > kLongMaxCoeffs || nb > kLongMaxCoeffs) return DQT_E_UNSUPPORTED;
    const uint32_t pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    const uint32_t na_pad = (na + kPlainG - 1) / kPlainG * kPlainG;
    const uint32_t nb_tot = kPad + nb + kPad;
    const uint32_t slot_words = (gapped<3>(na_pad) + gapped<3>(nb_tot) + 3) & ~3u;
    const uint32_t C = (na + nb - 1 + kPlainR - 1) / kPlainR;
    const uint32_t pairs = (C + 1) / 2;
    unsigned threads;
    uint32_t tpp, ppw;
    if (pairs <= 32) {
        ppw = 64 / pairs;
        while (ppw > 1 && (size_t)ppw * slot_words * 4 > 65536) --ppw;
        tpp = 64 / ppw;
        threads = 64;
    } else {
        threads = (pairs + 63) / 64 * 64;
        tpp = threads;
        ppw = 1;
    }
    const size_t smem = (size_t)ppw * slot_words * 4;
    if (threads > 512 || smem > 65536) return DQT_E_UNSUPPORTED;
    const unsigned grid = balanced_grid((count + ppw - 1) / ppw, groups_per_cu(smem, threads, plain_long_regs(pairs <= 64)));
    // the single walk pays off while the chunk pairs fit one wave (measured from 65 to 4096
    // coefficients, as for the FQT kernel); with more, the two loops per lane are faster
    if (pairs <= 64)
        hipLaunchKernelGGL(k_polymul_plain_long<true>, dim3(grid), dim3(threads), smem, s, A, B, out, count, na, nb, p,
                           pmagic, na_pad, nb_tot, tpp, ppw, slot_words);
    else
        hipLaunchKernelGGL(k_polymul_plain_long<false>, dim3(grid), dim3(threads), smem, s, A, B, out, count, na, nb, p,
                           pmagic, na_pad, nb_tot, tpp, ppw, slot_words);
    DQT_LAUNCH_CHECK("dqt_polymul_plain_u8 (long)");
    return DQT_OK;
}

}  // namespace dqt
