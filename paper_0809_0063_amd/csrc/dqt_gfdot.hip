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

// G lanes share one dot product: lane g of a group takes the pairs l = g,
// g + G, g + 2G, ..., so the G lanes of a group read G consecutive records of
// k bytes (whole runs of the operands, G k bytes per step), each lane keeps
// its own packed sums of n_q products and its own field result, and the G
// results are added in the field across the group by shuffles.  G = 1 is one
// thread per dot product (short dot products).
template <int K, int G>
__global__ __launch_bounds__(256) void k_gf_dot(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                uint8_t* __restrict__ OUT, uint64_t count, uint32_t n, uint32_t nq,
                                                RedqArgs ra, GfArgs ga) {
    extern __shared__ uint64_t gfd_smem[];
    const uint32_t tn = 1u << (K * ra.w);
    uint64_t* tl = gfd_smem;
    uint64_t* th = gfd_smem + tn;
    build_gf_tables_dot<K>(tl, th, ra, ga);
    __syncthreads();
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    const uint32_t wm = (1u << ra.w) - 1u;
    const uint32_t g = threadIdx.x % G;
    const uint64_t groups = (uint64_t)gridDim.x * (256 / G);
    // every lane of a group runs the same number of outer iterations (the
    // shuffles below need the whole wave), so the loop runs to the padded count
    const uint64_t padded = (count + groups - 1) / groups * groups;
    for (uint64_t t = (uint64_t)blockIdx.x * (256 / G) + threadIdx.x / G; t < padded; t += groups) {
        const bool live = t < count;
        const uint8_t* x = A + (live ? t : 0) * (uint64_t)n * K;
        const uint8_t* y = B + (live ? t : 0) * (uint64_t)n * K;
        uint64_t R = 0;
        // this lane's pairs: l = g + G j; n_q of them per packed word
        const uint32_t mine = live && g < n ? (n - g + G - 1) / G : 0;
        for (uint32_t j0 = 0; j0 < mine; j0 += nq) {
            const uint32_t j1 = min(mine, j0 + nq);
            uint64_t acc = 0;
            for (uint32_t j = j0; j < j1; ++j) {
                const uint64_t l = (uint64_t)g + (uint64_t)G * j;
                uint64_t xa = 0, yb = 0;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    xa |= (uint64_t)x[l * K + i] << (ra.b * i);
                    yb |= (uint64_t)y[l * K + i] << (ra.b * i);
                }
                acc += xa * yb;
            }
            const uint64_t U = redq_compress(acc, ra);
            const uint32_t xl = (uint32_t)U;
            const uint64_t xh64 = U >> (ra.b * (K - 1));
            uint32_t il = 0, ih = 0;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                il |= ((xl >> (ra.b * jj)) & wm) << (ra.w * jj);
                ih |= ((uint32_t)(xh64 >> (ra.b * jj)) & wm) << (ra.w * jj);
            }
            R = add_mod_bytes(R, add_mod_bytes(th[ih], tl[il], ra.p, ones), ra.p, ones);
        }
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
    const uint64_t threads = count * G;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_dot<K, G>), dim3(stream_grid(threads, 256, 4)), dim3(256), smem, s, A, B,
                       out, count, n, nq, ra, ga);
}

// Lanes per dot product: one wave for long ones, fewer for short ones.
template <int K>
static dqt_status launch_gf_dot(const uint8_t* A, const uint8_t* B, uint8_t* out, uint64_t count, uint32_t n,
                                uint32_t nq, const RedqArgs& ra, const GfArgs& ga, hipStream_t s) {
    if (n >= 256) launch_gf_dot_g<K, 64>(A, B, out, count, n, nq, ra, ga, s);
    else if (n >= 32) launch_gf_dot_g<K, 16>(A, B, out, count, n, nq, ra, ga, s);
    else if (n >= 8) launch_gf_dot_g<K, 4>(A, B, out, count, n, nq, ra, ga, s);
    else launch_gf_dot_g<K, 1>(A, B, out, count, n, nq, ra, ga, s);
    DQT_LAUNCH_CHECK("dqt_gf_dot_u8");
    return DQT_OK;
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
    uint32_t b = 53 / (2 * k - 1);
    if (b > 32) b = 32;
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
