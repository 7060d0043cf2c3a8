// Long polynomial products by the FQT (section 5.2 of the paper).
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

#include "dqt_internal.h"

namespace dqt {

template <int BS, int MAXB>
__global__ __launch_bounds__(256) void k_polymul_fqt(const uint8_t* __restrict__ A, uint32_t na,
                                                     const uint8_t* __restrict__ B, uint32_t nb,
                                                     uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra) {
    constexpr int NR = 2 * BS - 1;
    constexpr int NW = 2 * MAXB - 1;
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    __syncthreads();
    const uint32_t nout = na + nb - 1;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        const uint8_t* x = A + t * na;
        const uint8_t* y = B + t * nb;
        uint32_t aw[MAXB], bw[MAXB];
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            uint32_t va = 0, vb = 0;
#pragma unroll
            for (int s = 0; s < BS; ++s) {
                const uint32_t c = i * BS + s;
                if (c < na) va |= (uint32_t)x[c] << (ra.b * s);
                if (c < nb) vb |= (uint32_t)y[c] << (ra.b * s);
            }
            aw[i] = va;
            bw[i] = vb;
        }
        // For each output block t: packed sum of its block products (delayed
        // reduction), one REDQ_{2d+1}, then the coefficients that no later
        // block touches are final and stored; the top d are carried.
        uint8_t* z = OUT + t * nout;
        uint32_t carry[BS > 1 ? BS - 1 : 1];
#pragma unroll
        for (int s = 0; s < BS - 1; ++s) carry[s] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if ((uint32_t)(BS * w) >= nout) break;
            uint64_t Wt = 0;
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                const int j = w - i;
                if (j >= 0 && j < MAXB) Wt += (uint64_t)aw[i] * (uint64_t)bw[j];
            }
            const uint64_t U = redq_compress(Wt, ra);
            uint32_t mu[NR];
            redq_correct<NR>(U, ra, tab, [&](int s, uint32_t v) { mu[s] = v; });
#pragma unroll
            for (int s = 0; s < BS; ++s) {
                uint32_t v = mu[s] + (s < BS - 1 ? carry[s] : 0u);
                v = v >= ra.p ? v - ra.p : v;
                const uint32_t pos = BS * w + s;
                if (pos < nout) z[pos] = (uint8_t)v;
            }
#pragma unroll
            for (int s = 0; s < BS - 1; ++s) carry[s] = mu[BS + s];
        }
        // coefficients past the last block start: only the carry of the last block
#pragma unroll
        for (int s = 0; s < BS - 1; ++s) {
            const uint32_t pos = BS * NW + s;
            if (pos < nout) z[pos] = (uint8_t)carry[s];
        }
    }
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

template <int BS, int MAXB>
static void launch_fqt(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint8_t* out, uint64_t count,
                       const RedqArgs& ra, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fqt<BS, MAXB>), dim3(stream_grid(count, 256)), dim3(256), 0, s, A, na,
                       B, nb, out, count, ra);
}

template <int BS>
static void launch_fqt_b(uint32_t maxb, const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint8_t* out,
                         uint64_t count, const RedqArgs& ra, hipStream_t s) {
    if (maxb <= 2) launch_fqt<BS, 2>(A, na, B, nb, out, count, ra, s);
    else if (maxb <= 4) launch_fqt<BS, 4>(A, na, B, nb, out, count, ra, s);
    else if (maxb <= 8) launch_fqt<BS, 8>(A, na, B, nb, out, count, ra, s);
    else launch_fqt<BS, 16>(A, na, B, nb, out, count, ra, s);
}

}  // namespace dqt

using namespace dqt;

extern "C" dqt_status dqt_polymul_fqt_u8(const uint8_t* d_a, uint32_t na, const uint8_t* d_b, uint32_t nb,
                                         uint64_t count, uint32_t p, uint32_t block, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || na < 1 || nb < 1 || na > 64 || nb > 64) return DQT_E_INVALID;
    // choose the block size (2..6) and q
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
    RedqArgs ra;
    DQT_TRY(make_redq_args(p, best_b, 2 * best_bs - 1, (2 * best_bs - 1) * best_b, &ra));
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
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
