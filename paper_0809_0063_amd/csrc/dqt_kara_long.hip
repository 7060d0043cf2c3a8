// Karatsuba's recursion over F_p on top of the FQT (section 5.3, figure
// fig:pmkara: the subquadratic product with the packed product at its base).
//
// One level turns each product a.b of two n-coefficient polynomials into three
// products of h = ceil(n/2) coefficients: a = a0 + x^h a1, b = b0 + x^h b1,
//   P0 = a0 b0,  P2 = a1 b1,  P1 = (a0 + a1)(b0 + b1),
//   a b = P0 + x^h (P1 - P0 - P2) + x^2h P2,
// every coefficient taken mod p (the identity holds in F_p[x], so the sums
// a0 + a1 are reduced to [0, p) and the inputs of the next level are again
// residues).  L levels give 3^L products of h_L coefficients, computed by the
// packed FQT (dqt_polymul_fqt_u8) in one call; the combinations run level by
// level back up.  Each split (both operands) and each combination is one
// launch over the whole batch, a wave per product row, four bytes per lane.
//
// Workspace: for each level l = 1..L, the 3^l operand pairs of h_l
// coefficients (a then b) and the 3^l products of 2 h_l - 1 coefficients.

#include <string.h>

#include "dqt_internal.h"

namespace dqt {

namespace {

constexpr unsigned kWaves = 4;   // waves per workgroup; each wave takes one product at a time

// Four bytes at any address (the rows are not word aligned; global memory takes
// unaligned dword accesses).
__device__ __forceinline__ uint32_t ld4(const uint8_t* x) {
    uint32_t v;
    __builtin_memcpy(&v, x, 4);
    return v;
}
__device__ __forceinline__ void st4(uint8_t* x, uint32_t v) { __builtin_memcpy(x, &v, 4); }

constexpr uint32_t kEven = 0x00FF00FFu;   // bytes 0 and 2 of a word as two 16-bit lanes
__device__ __forceinline__ uint32_t even16(uint32_t x) { return x & kEven; }
__device__ __forceinline__ uint32_t odd16(uint32_t x) { return (x >> 8) & kEven; }

// v - m in each 16-bit lane where the lane is >= m (lanes below 2^15, m <= 2^15)
__device__ __forceinline__ uint32_t sub_if_ge16(uint32_t v, uint32_t m) {
    const uint32_t ge = ((v | 0x80008000u) - m * 0x00010001u) & 0x80008000u;
    return v - (ge >> 15) * m;
}

// Operands [count][n] (blockIdx.y: 0 = a, 1 = b) -> parts [count][3][h]: a0, a1, a0 + a1 (mod p).
// A lane takes four consecutive coefficients; words that reach past a half fall back to bytes.
__global__ __launch_bounds__(256) void k_kara_split(const uint8_t* __restrict__ sa, const uint8_t* __restrict__ sb,
                                                    uint64_t count, uint32_t n, uint32_t h, uint32_t p,
                                                    uint8_t* __restrict__ da, uint8_t* __restrict__ db) {
    const uint8_t* src = blockIdx.y ? sb : sa;
    uint8_t* dst = blockIdx.y ? db : da;
    const uint32_t lane = threadIdx.x & 63;
    for (uint64_t t = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); t < count; t += (uint64_t)gridDim.x * kWaves) {
        const uint8_t* s = src + t * n;
        uint8_t* d = dst + t * 3ull * h;
        for (uint32_t i = 4 * lane; i < h; i += 256) {   // i < h <= n
            if (i + 3 < h && h + i + 3 < n) {
                const uint32_t lo = ld4(s + i), hi = ld4(s + h + i);
                const uint32_t me = sub_if_ge16(even16(lo) + even16(hi), p);
                const uint32_t mo = sub_if_ge16(odd16(lo) + odd16(hi), p);
                st4(d + i, lo);
                st4(d + h + i, hi);
                st4(d + 2 * h + i, me | (mo << 8));
                continue;
            }
            for (uint32_t x = i; x < i + 4 && x < h; ++x) {
                const uint32_t lo = s[x];
                const uint32_t hi = h + x < n ? s[h + x] : 0u;
                const uint32_t m = lo + hi;
                d[x] = (uint8_t)lo;
                d[h + x] = (uint8_t)hi;
                d[2 * h + x] = (uint8_t)(m >= p ? m - p : m);
            }
        }
    }
}

// Products [count][3][2h-1] of the parts above (P0 = a0 b0, P2 = a1 b1, P1 = (a0+a1)(b0+b1),
// in that order) -> [count][2n-1]:  out_j = P0_j + P2_{j-2h} + (P1 - P0 - P2)_{j-h} mod p, each
// term present where its index falls inside its product.  A lane takes four consecutive outputs;
// words where a term starts or ends, or that reach past the row, fall back to bytes.
__global__ __launch_bounds__(256) void k_kara_combine(const uint8_t* __restrict__ prod, uint64_t count, uint32_t n,
                                                      uint32_t h, uint32_t p, uint8_t* __restrict__ out) {
    const uint32_t no = 2 * n - 1, np = 2 * h - 1;
    const uint32_t lane = threadIdx.x & 63;
    for (uint64_t t = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); t < count; t += (uint64_t)gridDim.x * kWaves) {
        const uint8_t* P0 = prod + t * 3ull * np;
        const uint8_t* P2 = P0 + np;
        const uint8_t* P1 = P2 + np;
        uint8_t* o = out + t * no;
        for (uint32_t j = 4 * lane; j < no; j += 256) {
            // a term boundary T inside (j, j + 3] splits the word
            auto splits = [&](uint32_t T) { return j < T && T <= j + 3; };
            if (j + 3 < no && !splits(np) && !splits(2 * h) && !splits(h) && !splits(h + np)) {
                const bool c0 = j < np, c2 = j >= 2 * h, c1 = j >= h && j - h < np;
                uint32_t ve = 0, vo = 0;
                if (c0) {
                    const uint32_t x = ld4(P0 + j);
                    ve += even16(x);
                    vo += odd16(x);
                }
                if (c2) {   // j - 2h + 3 <= 2n - 2 - 2h < np
                    const uint32_t x = ld4(P2 + j - 2 * h);
                    ve += even16(x);
                    vo += odd16(x);
                }
                if (c1) {   // (P1 - P0 - P2) kept non-negative by 2p per lane
                    const uint32_t m = j - h;
                    const uint32_t x1 = ld4(P1 + m), x0 = ld4(P0 + m), x2 = ld4(P2 + m);
                    ve += even16(x1) + 2 * p * 0x00010001u - even16(x0) - even16(x2);
                    vo += odd16(x1) + 2 * p * 0x00010001u - odd16(x0) - odd16(x2);
                }
                // lanes < 5p
                ve = sub_if_ge16(sub_if_ge16(sub_if_ge16(ve, 4 * p), 2 * p), p);
                vo = sub_if_ge16(sub_if_ge16(sub_if_ge16(vo, 4 * p), 2 * p), p);
                st4(o + j, ve | (vo << 8));
                continue;
            }
            for (uint32_t x = j; x < j + 4 && x < no; ++x) {
                uint32_t v = x < np ? P0[x] : 0u;
                if (x >= 2 * h) v += P2[x - 2 * h];
                if (x >= h && x - h < np) {
                    const uint32_t m = x - h;
                    v += P1[m] + 2 * p - P0[m] - P2[m];
                }
                if (v >= 4 * p) v -= 4 * p;
                if (v >= 2 * p) v -= 2 * p;
                if (v >= p) v -= p;
                o[x] = (uint8_t)v;
            }
        }
    }
}

struct KaraLevels {
    uint32_t L;
    uint32_t h[4];          // h[0] = n, h[l] = ceil(h[l-1] / 2)
    uint64_t cnt[4];        // count * 3^l
    size_t opnd[4], prod[4];  // workspace offsets of level l's operands (a then b) and products
    size_t total;
};

dqt_status kara_levels(uint64_t count, uint32_t n, uint32_t levels, KaraLevels* K) {
    if (levels < 1 || levels > 3 || n < 2 || n > 4096) return DQT_E_INVALID;
    memset(K, 0, sizeof(*K));
    K->L = levels;
    K->h[0] = n;
    K->cnt[0] = count;
    size_t off = 0;
    for (uint32_t l = 1; l <= levels; ++l) {
        K->h[l] = (K->h[l - 1] + 1) / 2;
        if (K->h[l] < 2) return DQT_E_INVALID;
        K->cnt[l] = K->cnt[l - 1] * 3;
        K->opnd[l] = off;
        off += (2 * K->cnt[l] * K->h[l] + 255) & ~(size_t)255;
        K->prod[l] = off;
        off += (K->cnt[l] * (2 * K->h[l] - 1) + 255) & ~(size_t)255;
    }
    K->total = off;
    return DQT_OK;
}

}  // namespace

}  // namespace dqt

using namespace dqt;

extern "C" size_t dqt_polymul_kara_long_workspace(uint64_t count, uint32_t n, uint32_t levels) {
    KaraLevels K;
    if (kara_levels(count, n, levels, &K) != DQT_OK) return 0;
    return K.total;
}

extern "C" dqt_status dqt_polymul_kara_long_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t n,
                                               uint32_t p, uint32_t levels, uint8_t* d_out, void* d_work,
                                               size_t work_bytes, void* stream) {
    if (p < 2 || p > 255) return DQT_E_INVALID;
    KaraLevels K;
    DQT_TRY(kara_levels(count, n, levels, &K));
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    if (!d_work || work_bytes < K.total) return DQT_E_WORKSPACE;
    // the base products (3^L count of them, h_L coefficients) must be ones the FQT takes
    DQT_TRY(dqt_polymul_fqt_u8(nullptr, K.h[K.L], nullptr, K.h[K.L], 0, p, 0, nullptr, nullptr));
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, n, n}, {d_b, count, n, n}}));
    uint8_t* w = reinterpret_cast<uint8_t*>(d_work);
    // splits, level by level
    for (uint32_t l = 1; l <= K.L; ++l) {
        const uint8_t* sa = l == 1 ? d_a : w + K.opnd[l - 1];
        const uint8_t* sb = l == 1 ? d_b : w + K.opnd[l - 1] + K.cnt[l - 1] * K.h[l - 1];
        uint8_t* da = w + K.opnd[l];
        uint8_t* db = da + K.cnt[l] * K.h[l];
        hipLaunchKernelGGL(k_kara_split, dim3(stream_grid(K.cnt[l - 1], kWaves), 2), dim3(64 * kWaves), 0, s, sa, sb,
                           K.cnt[l - 1], K.h[l - 1], K.h[l], p, da, db);
        DQT_LAUNCH_CHECK("dqt_polymul_kara_long_u8 (split)");
    }
    // the base products by the packed FQT
    {
        const uint8_t* ba = w + K.opnd[K.L];
        const uint8_t* bb = ba + K.cnt[K.L] * K.h[K.L];
        DQT_TRY(dqt_polymul_fqt_u8(ba, K.h[K.L], bb, K.h[K.L], K.cnt[K.L], p, 0, w + K.prod[K.L], stream));
    }
    // combinations, level by level back up; level 1's result is the output
    for (uint32_t l = K.L; l >= 1; --l) {
        uint8_t* dst = l == 1 ? d_out : w + K.prod[l - 1];
        hipLaunchKernelGGL(k_kara_combine, dim3(stream_grid(K.cnt[l - 1], kWaves)), dim3(64 * kWaves), 0, s,
                           w + K.prod[l], K.cnt[l - 1], K.h[l - 1], K.h[l], p, dst);
        DQT_LAUNCH_CHECK("dqt_polymul_kara_long_u8 (combine)");
    }
    return DQT_OK;
}
