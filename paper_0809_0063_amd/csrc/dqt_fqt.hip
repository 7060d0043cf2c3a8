// Long polynomial products by the FQT (section 5.2 of the paper), with the
// block products either schoolbook or by Karatsuba's recursion on the packed
// block words (the subquadratic variant of figure fig:pmkara).
//
// A polynomial of degree < na is cut into blocks of BS = d+1 coefficients,
// P = sum_i P_i Y^i with Y = X^BS, and each block is packed in one word at
// q = 2^b.  The product is sum_t W_t Y^t with W_t = sum_i P_i Q_{t-i}: every
// block product is one machine multiply (a 32x32 -> 64-bit multiply-add), and
// the block products of one W_t are summed in packed form (delayed
// reduction): q > n (d+1) (p-1)^2 with n the number of summed products keeps
// every digit below q (eq:bounds) and (2d+1) b <= 53 keeps W_t exact in
// binary64 for REDQ_{2d+1}.  Output block t covers coefficients
// BS*t .. BS*t + 2d; its top d coefficients overlap the next block and are
// added modulo p after both are reduced.

#include <string.h>

#include "dqt_fqt.h"
#include "dqt_internal.h"

namespace dqt {

// Tiles of 256 products through LDS (record_tiles); each product: block
// words, their packed products summed per output block (delayed reduction),
// one REDQ_{2d+1} per block word.  QB, QW, SMALL as in fqt_finish; the
// compile-time instances ask for three waves per SIMD (168 VGPRs, a few
// spilled).
template <int BS, int MAXB, int QB = 0, int QW = 0, bool SMALL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QB ? 3 : 1))) void k_polymul_fqt(
    const uint8_t* __restrict__ A, uint32_t na, const uint8_t* __restrict__ B, uint32_t nb,
    uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra) {
    using F = FqtShape<BS, MAXB>;
    extern __shared__ uint32_t fqt_smem[];
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    const uint32_t nout = na + nb - 1;
    record_tiles<F::ND, F::ND, F::NO>(fqt_smem, A, na, B, nb, OUT, count,
                                      [&](const uint32_t (&xa)[F::ND], const uint32_t (&xb)[F::ND],
                                          uint32_t (&ob)[F::NO]) {
        uint32_t aw[MAXB], bw[MAXB];
        fqt_words<BS, MAXB>(xa, QB ? QB : ra.b, aw);
        fqt_words<BS, MAXB>(xb, QB ? QB : ra.b, bw);
        if constexpr (QB != 0) {
            // All block words first, then the reductions.  (The compile-time
            // instance of the on-demand form below gave wrong bytes in the first
            // two coefficients of some blocks on the device, with no fault found
            // in the source; it is not built.)
            uint64_t W[F::NW];
#pragma unroll
            for (int w = 0; w < F::NW; ++w) {
                uint64_t Wt = 0;
#pragma unroll
                for (int i = 0; i < MAXB; ++i) {
                    const int j = w - i;
                    if (j >= 0 && j < MAXB) Wt += (uint64_t)aw[i] * (uint64_t)bw[j];
                }
                W[w] = Wt;
            }
            fqt_finish<BS, F::NW, QB, QW, SMALL>([&](int w) { return W[w]; }, nout, ra, tab, ob);
        } else {
            auto Wof = [&](int w) {
                uint64_t Wt = 0;
#pragma unroll
                for (int i = 0; i < MAXB; ++i) {
                    const int j = w - i;
                    if (j >= 0 && j < MAXB) Wt += (uint64_t)aw[i] * (uint64_t)bw[j];
                }
                return Wt;
            };
            fqt_finish<BS, F::NW, 0, 0, false>(Wof, nout, ra, tab, ob);
        }
    });
}

// Karatsuba on polynomials (in Y = X^BS) whose coefficients are packed block
// words.  The evaluation at q is a ring morphism, so the recursion can run on
// the words as integers modulo 2^64: the middle term (a0 + a1)(b0 + b1) - a0 b0
// - a1 b1 is, as an integer, exactly the packed word of a0 b1 + a1 b0, even
// where the intermediate words wrap, and every final W_t equals the
// schoolbook's sum of block products, below 2^53 with every digit below q.
// LEV levels of recursion, schoolbook below.
template <int N, int LEV>
struct Kara {
    static __device__ __forceinline__ void mul(const uint64_t* a, const uint64_t* b, uint64_t* r) {
        if constexpr (LEV == 0 || N < 4) {
#pragma unroll
            for (int t = 0; t < 2 * N - 1; ++t) r[t] = 0;
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = 0; j < N; ++j) r[i + j] += a[i] * b[j];
        } else {
            constexpr int H = N / 2;       // low half; the high half has N - H >= H words
            constexpr int G = N - H;
            uint64_t r0[2 * H - 1], r2[2 * G - 1], m[2 * G - 1], sa[G], sb[G];
            Kara<H, LEV - 1>::mul(a, b, r0);
            Kara<G, LEV - 1>::mul(a + H, b + H, r2);
#pragma unroll
            for (int i = 0; i < G; ++i) {
                sa[i] = a[H + i] + (i < H ? a[i] : 0ull);
                sb[i] = b[H + i] + (i < H ? b[i] : 0ull);
            }
            Kara<G, LEV - 1>::mul(sa, sb, m);
#pragma unroll
            for (int t = 0; t < 2 * G - 1; ++t) m[t] -= r2[t] + (t < 2 * H - 1 ? r0[t] : 0ull);
#pragma unroll
            for (int t = 0; t < 2 * N - 1; ++t) r[t] = 0;
#pragma unroll
            for (int t = 0; t < 2 * H - 1; ++t) r[t] += r0[t];
#pragma unroll
            for (int t = 0; t < 2 * G - 1; ++t) r[H + t] += m[t];
#pragma unroll
            for (int t = 0; t < 2 * G - 1; ++t) r[2 * H + t] += r2[t];
        }
    }
};

template <int BS, int MAXB, int LEV, int QB = 0, int QW = 0, bool SMALL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QB ? 3 : 1))) void k_polymul_fqt_kara(
    const uint8_t* __restrict__ A, uint32_t na, const uint8_t* __restrict__ B, uint32_t nb,
    uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra) {
    using F = FqtShape<BS, MAXB>;
    extern __shared__ uint32_t fqt_smem[];
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    const uint32_t nout = na + nb - 1;
    record_tiles<F::ND, F::ND, F::NO>(fqt_smem, A, na, B, nb, OUT, count,
                                      [&](const uint32_t (&xa)[F::ND], const uint32_t (&xb)[F::ND],
                                          uint32_t (&ob)[F::NO]) {
        uint64_t aw[MAXB], bw[MAXB], W[F::NW];
        fqt_words<BS, MAXB>(xa, QB ? QB : ra.b, aw);
        fqt_words<BS, MAXB>(xb, QB ? QB : ra.b, bw);
        Kara<MAXB, LEV>::mul(aw, bw, W);
        fqt_finish<BS, F::NW, QB, QW, SMALL>([&](int w) { return W[w]; }, nout, ra, tab, ob);
    });
}

// Cost of one product with block size bs (block multiplies + REDQ words),
// the time-memory trade-off model of table tab:mulpol with a REDQ priced at
// about 40 machine operations.
static double fqt_cost(uint32_t na, uint32_t nb, uint32_t bs) {
    const uint32_t Na = (na + bs - 1) / bs, Nb = (nb + bs - 1) / bs;
    return 1.5 * Na * Nb + 40.0 * (Na + Nb - 1) + 2.0 * (na + nb);
}

// Smallest b for block size bs with n summed products: q > n bs (p-1)^2,
// (2bs-1) b <= 53, bs b <= 32, and the residue field fits the digit.
static bool fqt_q(uint32_t p, uint32_t bs, uint32_t n, uint32_t* b_out) {
    const uint64_t need = (uint64_t)n * bs * (uint64_t)(p - 1) * (p - 1);
    const uint32_t w = residue_bits(p);
    for (uint32_t b = (w > 1 ? w : 1); b <= 32; ++b) {
        if ((2 * bs - 1) * b > 53 || bs * b > 32) return false;
        if ((1ull << b) > need) {
            *b_out = b;
            return true;
        }
    }
    return false;
}

// Compile-time q and residue width for blocks of three coefficients over F_3
// and 11 to 16 blocks per operand (q = 2^8, w = 2: 31 to 48 coefficients), else
// the run-time values.
static bool fqt_f3_blocks(uint32_t bs, const RedqArgs& ra) { return bs == 3 && ra.b == 8 && ra.w == 2 && ra.small; }

template <int BS, int MAXB>
static void launch_fqt(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint8_t* out, uint64_t count,
                       const RedqArgs& ra, hipStream_t s) {
    const dim3 grid(stream_grid(count, 256)), blk(256);
    const size_t sm = record_tiles_smem(na, nb);
    if constexpr (BS == 3 && MAXB == 16) {
        if (fqt_f3_blocks(BS, ra)) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt<BS, MAXB, 8, 2, true>), grid, blk, sm, s, A, na, B, nb, out,
                               count, ra);
            return;
        }
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt<BS, MAXB>), grid, blk, sm, s, A, na, B, nb, out, count, ra);
}

template <int BS>
static void launch_fqt_b(uint32_t maxb, const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint8_t* out,
                         uint64_t count, const RedqArgs& ra, hipStream_t s) {
    if (maxb <= 2) launch_fqt<BS, 2>(A, na, B, nb, out, count, ra, s);
    else if (maxb <= 4) launch_fqt<BS, 4>(A, na, B, nb, out, count, ra, s);
    else if (maxb <= 8) launch_fqt<BS, 8>(A, na, B, nb, out, count, ra, s);
    else launch_fqt<BS, 16>(A, na, B, nb, out, count, ra, s);
}

template <int BS, int LEV>
static void launch_kara_b(uint32_t maxb, const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint8_t* out,
                          uint64_t count, const RedqArgs& ra, hipStream_t s) {
    const dim3 grid(stream_grid(count, 256)), blk(256);
    const size_t sm = record_tiles_smem(na, nb);
    if (maxb <= 4) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_kara<BS, 4, LEV>), grid, blk, sm, s, A, na, B, nb, out, count, ra);
    else if (maxb <= 8) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_kara<BS, 8, LEV>), grid, blk, sm, s, A, na, B, nb, out, count, ra);
    else {
        if constexpr (BS == 3) {
            if (fqt_f3_blocks(BS, ra)) {
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_kara<BS, 16, LEV, 8, 2, true>), grid, blk, sm, s, A, na,
                                   B, nb, out, count, ra);
                return;
            }
        }
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt_kara<BS, 16, LEV>), grid, blk, sm, s, A, na, B, nb, out, count,
                           ra);
    }
}

template <int BS>
static void launch_kara(uint32_t levels, uint32_t maxb, const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb,
                        uint8_t* out, uint64_t count, const RedqArgs& ra, hipStream_t s) {
    if (levels == 1) launch_kara_b<BS, 1>(maxb, A, na, B, nb, out, count, ra, s);
    else launch_kara_b<BS, 2>(maxb, A, na, B, nb, out, count, ra, s);
}

// Block size and q of a product (shared by both entry points).
static dqt_status fqt_choose(uint32_t p, uint32_t na, uint32_t nb, uint32_t block, uint32_t* bs_out, uint32_t* b_out) {
    uint32_t best_bs = 0, best_b = 0;
    double best = 1e300;
    for (uint32_t bs = 2; bs <= 6; ++bs) {
        if (block && bs != block) continue;
        const uint32_t Na = (na + bs - 1) / bs, Nb = (nb + bs - 1) / bs;
        if (Na > 16 || Nb > 16) continue;
        uint32_t b = 0;
        if (!fqt_q(p, bs, Na < Nb ? Na : Nb, &b)) continue;
        const double c = fqt_cost(na, nb, bs);
        if (c < best) {
            best = c;
            best_bs = bs;
            best_b = b;
        }
    }
    if (!best_bs) return block ? DQT_E_BOUND : DQT_E_UNSUPPORTED;
    *bs_out = best_bs;
    *b_out = best_b;
    return DQT_OK;
}

}  // namespace dqt

using namespace dqt;

extern "C" dqt_status dqt_polymul_fqt_kara_u8(const uint8_t* d_a, uint32_t na, const uint8_t* d_b, uint32_t nb,
                                              uint64_t count, uint32_t p, uint32_t block, uint32_t levels,
                                              uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || na < 1 || nb < 1 || na > 64 || nb > 64) return DQT_E_INVALID;
    if (levels < 1 || levels > 2) return DQT_E_INVALID;
    uint32_t bs = 0, b = 0;
    DQT_TRY(fqt_choose(p, na, nb, block, &bs, &b));
    RedqArgs ra;
    DQT_TRY(make_redq_args(p, b, 2 * bs - 1, (2 * bs - 1) * b, &ra));
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, na, na}, {d_b, count, nb, nb}}));
    const uint32_t Na = (na + bs - 1) / bs, Nb = (nb + bs - 1) / bs;
    const uint32_t maxb = Na > Nb ? Na : Nb;
    switch (bs) {
        case 2: launch_kara<2>(levels, maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 3: launch_kara<3>(levels, maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 4: launch_kara<4>(levels, maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 5: launch_kara<5>(levels, maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        default: launch_kara<6>(levels, maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
    }
    DQT_LAUNCH_CHECK("dqt_polymul_fqt_kara_u8");
    return DQT_OK;
}

namespace dqt {
dqt_status fqt_long_enqueue(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint64_t count, uint32_t p,
                            uint32_t block, uint8_t* out, hipStream_t s, bool check_only);
}

extern "C" dqt_status dqt_polymul_fqt_u8(const uint8_t* d_a, uint32_t na, const uint8_t* d_b, uint32_t nb,
                                         uint64_t count, uint32_t p, uint32_t block, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || na < 1 || nb < 1 || na > 4096 || nb > 4096) return DQT_E_INVALID;
    // long products: one workgroup per product, chunked packed sums (dqt_fqt_long.hip)
    auto chunked = [&]() -> dqt_status {
        DQT_TRY(fqt_long_enqueue(d_a, na, d_b, nb, count, p, block, d_out, nullptr, true));
        if (count == 0) return DQT_OK;
        if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
        DQT_TRY(ensure_device_ready());
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        DQT_TRY(debug_gate(s, p, {{d_a, count, na, na}, {d_b, count, nb, nb}}));
        return fqt_long_enqueue(d_a, na, d_b, nb, count, p, block, d_out, s, false);
    };
    if (na > 64 || nb > 64) return chunked();
    uint32_t best_bs = 0, best_b = 0;
    RedqArgs ra;
    dqt_status st = fqt_choose(p, na, nb, block, &best_bs, &best_b);
    if (st == DQT_OK) st = make_redq_args(p, best_b, 2 * best_bs - 1, (2 * best_bs - 1) * best_b, &ra);
    if (st != DQT_OK) {
        // no block size keeps a whole output block's sum in one word (larger p, longer
        // operands): with the size left to the library, the chunked sums take it (p <= 127)
        if (block == 0 && p <= 127) return chunked();
        return st;
    }
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, na, na}, {d_b, count, nb, nb}}));
    const uint32_t Na = (na + best_bs - 1) / best_bs, Nb = (nb + best_bs - 1) / best_bs;
    const uint32_t maxb = Na > Nb ? Na : Nb;
    switch (best_bs) {
        case 2: launch_fqt_b<2>(maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 3: launch_fqt_b<3>(maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 4: launch_fqt_b<4>(maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        case 5: launch_fqt_b<5>(maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
        default: launch_fqt_b<6>(maxb, d_a, na, d_b, nb, d_out, count, ra, s); break;
    }
    DQT_LAUNCH_CHECK("dqt_polymul_fqt_u8");
    return DQT_OK;
}
