// Plain F_p matrix product on the INT8 matrix cores (comparator).
//
// C = A.B mod p with exact int32 accumulation: entries are residues below
// p <= 128, so they are valid int8 values, and every dot product is at most
// kdim (p-1)^2 < 2^31 (checked when the plan is resolved).  One reduction per
// output.
//
// Layouts (workspace, written by the packing launch):
//   A8:  [m_pad][k_pad] int8, the rows of A zero-padded to k_pad (a multiple of 64);
//   BT8: [n_pad][k_pad] int8, B transposed (column j of B as row j), zero-padded.
// m_pad and n_pad are multiples of 64.  B is transposed through LDS in tiles
// of 64 k x 64 columns, so both the reads of B and the writes of BT8 are
// whole 16-byte runs.
//
// Multiply: a workgroup of 4 waves owns a 64 x 64 square of C; the waves split
// k into S contiguous ranges (S = 4, 2 or 1 by the depth of k).  Each wave
// computes the whole square over its range as 4 x 4 tiles of
// v_mfma_i32_16x16x64_i8 (each loaded fragment feeds four matrix
// instructions): lane l supplies row (or column) l % 16 and the 16
// consecutive k of slot l / 16, for both operands, and receives rows
// 4 (l / 16) .. + 3 of column l % 16.  The loads of four k-steps (32 vector
// loads) are issued before their 64 matrix instructions.  The S partial
// squares are added through LDS.

#include <string.h>

#include <hip/hip_ext.h>

#include "dqt_gemm_tile.h"
#include "dqt_internal.h"

namespace dqt {

namespace {

struct MfmaPackArgs {
    const uint8_t* A;
    const uint8_t* B;
    uint8_t* A8;
    uint8_t* BT8;
    uint32_t m, n, kdim, lda, ldb, k_pad, m_pad, n_pad;
    uint32_t nba;          // workgroups copying A (16 bytes per thread)
    uint32_t tiles_n;      // 64-column tiles of B
    uint32_t al;           // bit 0: A and lda 16-byte aligned; bit 1: B and ldb 16-byte aligned
};

// 16 bytes of a row from x[0 .. len) (zero beyond len), as one vector load
// when aligned and whole.
__device__ __forceinline__ uint4 load16(const uint8_t* x, uint32_t len, bool aligned) {
    if (aligned && len >= 16) return *reinterpret_cast<const uint4*>(x);
    uint32_t w[4] = {0, 0, 0, 0};
    for (uint32_t i = 0; i < 16 && i < len; ++i) w[i >> 2] |= (uint32_t)x[i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ __launch_bounds__(256) void k_mfma_pack(MfmaPackArgs a) {
    if (blockIdx.x < a.nba) {
        // A8[row][16 c .. 16 c + 15]
        const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
        const uint32_t cpr = a.k_pad / 16;
        if (t >= (uint64_t)a.m_pad * cpr) return;
        const uint32_t row = (uint32_t)(t / cpr), c = (uint32_t)(t % cpr);
        const uint32_t k0 = 16 * c;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row < a.m && k0 < a.kdim) v = load16(a.A + (size_t)row * a.lda + k0, a.kdim - k0, a.al & 1u);
        *reinterpret_cast<uint4*>(a.A8 + (size_t)row * a.k_pad + k0) = v;
        return;
    }
    // BT8 tile: k0 .. k0+63 x columns n0 .. n0+63
    __shared__ uint8_t tile[64][64 + 4];
    const uint32_t b = blockIdx.x - a.nba;
    const uint32_t n0 = (b % a.tiles_n) * 64, k0 = (b / a.tiles_n) * 64;
    {
        const uint32_t kk = threadIdx.x >> 2, cc = (threadIdx.x & 3) * 16;
        const uint32_t k = k0 + kk, col = n0 + cc;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (k < a.kdim && col < a.n) v = load16(a.B + (size_t)k * a.ldb + col, a.n - col, a.al & 2u);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&tile[kk][cc]);
        dst[0] = v.x;
        dst[1] = v.y;
        dst[2] = v.z;
        dst[3] = v.w;
    }
    __syncthreads();
    const uint32_t nn = threadIdx.x >> 2, kc = (threadIdx.x & 3) * 16;
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i) w[i >> 2] |= (uint32_t)tile[kc + i][nn] << (8 * (i & 3));
    *reinterpret_cast<uint4*>(a.BT8 + (size_t)(n0 + nn) * a.k_pad + k0 + kc) = make_uint4(w[0], w[1], w[2], w[3]);
}

struct MfmaArgs {
    const uint8_t* A8;
    const uint8_t* BT8;
    uint8_t* C;
    uint32_t m, n, ldc, k_pad;
    uint32_t nrb;          // 64-row blocks
    uint32_t ks;           // 64-k steps per wave
    uint32_t p, pmagic;
};

typedef int v4i __attribute__((ext_vector_type(4)));

// Square of C of workgroup `bid`: consecutive workgroups go to the eight XCDs in
// turn, so each XCD first gets a contiguous range of the order below; in that
// order the squares come in groups of 8 row blocks, column by column, so that
// the workgroups running together on an XCD share 8 row blocks of A and 8
// column blocks of B (within its L2) rather than all of A.
__device__ __forceinline__ void mfma_tile_of(uint32_t bid, uint32_t nblk, uint32_t nrb, uint32_t* rb, uint32_t* cb) {
    uint32_t logical = bid;
    if ((nblk & 7u) == 0) logical = (bid & 7u) * (nblk >> 3) + (bid >> 3);
    constexpr uint32_t GR = 8;
    const uint32_t ncb = nblk / nrb;
    const uint32_t group = logical / (GR * ncb), first = group * GR;
    const uint32_t rows = min(GR, nrb - first);
    const uint32_t in = logical - group * GR * ncb;
    *rb = first + in % rows;
    *cb = in / rows;
}

// T x T tiles of 16 x 16 per wave (a 16 T square of C); the S waves of a
// workgroup take contiguous k ranges of the same square and meet in LDS.
template <int S, int T>
__global__ __launch_bounds__(256) void k_gemm_mfma(MfmaArgs g) {
    constexpr int CH = 4;                        // k-steps whose loads are issued together
    __shared__ v4i red[S > 1 ? S * T * T * 64 : 1];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    uint32_t rb, cb;
    mfma_tile_of(blockIdx.x, gridDim.x, g.nrb, &rb, &cb);
    const uint32_t row0 = rb * 16 * T, col0 = cb * 16 * T;
    const uint32_t r = lane & 15u, slot = lane >> 4;
    v4i acc[T][T];
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) acc[i][j] = (v4i){0, 0, 0, 0};
    const uint32_t nsteps = g.k_pad / 64;
    const uint32_t s0 = min(nsteps, (wave % S) * g.ks), s1 = min(nsteps, s0 + g.ks);
    if (wave < (uint32_t)S) {
        const uint8_t* pa = g.A8 + (size_t)(row0 + r) * g.k_pad + slot * 16;
        const uint8_t* pb = g.BT8 + (size_t)(col0 + r) * g.k_pad + slot * 16;
        const size_t rs = (size_t)16 * g.k_pad;      // 16 rows (or columns) further
        uint32_t st = s0;
        for (; st + CH <= s1; st += CH) {
            v4i fa[CH][T], fb[CH][T];
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const size_t o = (size_t)(st + u) * 64 + i * rs;
                    fa[u][i] = *reinterpret_cast<const v4i*>(pa + o);
                    fb[u][i] = *reinterpret_cast<const v4i*>(pb + o);
                }
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int i = 0; i < T; ++i)
#pragma unroll
                    for (int j = 0; j < T; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[u][i], fb[u][j], acc[i][j], 0, 0, 0);
        }
        for (; st < s1; ++st) {
            v4i fa[T], fb[T];
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const size_t o = (size_t)st * 64 + i * rs;
                fa[i] = *reinterpret_cast<const v4i*>(pa + o);
                fb[i] = *reinterpret_cast<const v4i*>(pb + o);
            }
#pragma unroll
            for (int i = 0; i < T; ++i)
#pragma unroll
                for (int j = 0; j < T; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
    }
    // with one wave on the k range, that wave holds the whole square and writes it alone
    if (S == 1 && wave != 0) return;
    // the S partial squares meet in LDS; wave w finishes the 16 x 16 tiles t = w, w + 4, ...
    if (S > 1) {
        if (wave < (uint32_t)S) {
#pragma unroll
            for (int i = 0; i < T; ++i)
#pragma unroll
                for (int j = 0; j < T; ++j) red[((wave * T + i) * T + j) * 64 + lane] = acc[i][j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < T * T; ++t) {
        if (S > 1 && (uint32_t)t % 4 != wave) continue;
        const int ti = t / T, tj = t % T;
        v4i sum = acc[ti][tj];
        if (S > 1) {
            sum = (v4i){0, 0, 0, 0};
#pragma unroll
            for (int w = 0; w < S; ++w) sum += red[((w * T + ti) * T + tj) * 64 + lane];
        }
        const uint32_t col = col0 + 16 * tj + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t row = row0 + 16 * ti + 4 * slot + e;
            if (row < g.m && col < g.n)
                g.C[(size_t)row * g.ldc + col] = (uint8_t)mod_u32((uint32_t)sum[e], g.p, g.pmagic);
        }
    }
}

}  // namespace

static uint64_t ru(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

dqt_status mfma_plan(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, GemmPlanResolved* r) {
    if (p > 128) return DQT_E_UNSUPPORTED;   // entries must be valid int8
    if (kdim * (uint64_t)(p - 1) * (p - 1) >= (1ull << 31)) return DQT_E_UNSUPPORTED;
    r->k_pad = (uint32_t)ru(kdim ? kdim : 64, 64);
    r->m_pad = (uint32_t)ru(m ? m : 64, 64);
    r->n_pad = (uint32_t)ru(n ? n : 64, 64);   // whole 64-column transpose tiles
    const uint32_t steps = r->k_pad / 64;
    r->s = steps >= 4 ? 4 : (steps >= 2 ? 2 : 1);
    r->ws_bytes = (size_t)r->k_pad * (r->m_pad + r->n_pad);
    return DQT_OK;
}

size_t mfma_side_bytes(const GemmPlanResolved& r, int side) { return (size_t)r.k_pad * (side == 0 ? r.m_pad : r.n_pad); }

dqt_status mfma_pack_enqueue(const GemmPlanResolved& r, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A,
                             uint64_t lda, const uint8_t* B, uint64_t ldb, void* pA, void* pB, hipStream_t s) {
    if ((A && ((uintptr_t)pA & 15)) || (B && ((uintptr_t)pB & 15))) {
        set_error("fgemm(mfma): packed operands must be 16-byte aligned");
        return DQT_E_INVALID;
    }
    MfmaPackArgs a;
    a.A = A;
    a.B = B;
    a.A8 = reinterpret_cast<uint8_t*>(pA);
    a.BT8 = reinterpret_cast<uint8_t*>(pB);
    a.m = (uint32_t)m;
    a.n = (uint32_t)n;
    a.kdim = (uint32_t)kdim;
    a.lda = (uint32_t)lda;
    a.ldb = (uint32_t)ldb;
    a.k_pad = r.k_pad;
    a.m_pad = r.m_pad;
    a.n_pad = r.n_pad;
    a.al = ((A && ((uintptr_t)A & 15) == 0 && (lda & 15) == 0) ? 1u : 0u) |
           ((B && ((uintptr_t)B & 15) == 0 && (ldb & 15) == 0) ? 2u : 0u);
    a.nba = A ? (uint32_t)(((uint64_t)r.m_pad * (r.k_pad / 16) + 255) / 256) : 0;
    a.tiles_n = r.n_pad / 64;
    const uint64_t nbb = B ? (uint64_t)a.tiles_n * (r.k_pad / 64) : 0;
    if (a.nba + nbb == 0) return DQT_OK;
    hipLaunchKernelGGL(k_mfma_pack, dim3((uint32_t)(a.nba + nbb)), dim3(256), 0, s, a);
    DQT_LAUNCH_CHECK("fgemm(mfma pack)");
    return DQT_OK;
}

dqt_status mfma_compute_enqueue(const GemmPlanResolved& r, uint32_t p, uint64_t m, uint64_t n, uint8_t* C,
                                uint64_t ldc, const void* pA, const void* pB, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
    MfmaArgs g;
    g.A8 = reinterpret_cast<const uint8_t*>(pA);
    g.BT8 = reinterpret_cast<const uint8_t*>(pB);
    g.C = C;
    g.m = (uint32_t)m;
    g.n = (uint32_t)n;
    g.ldc = (uint32_t)ldc;
    g.k_pad = r.k_pad;
    g.nrb = r.m_pad / 64;
    const uint32_t steps = r.k_pad / 64;
    g.ks = (steps + r.s - 1) / r.s;
    g.p = p;
    g.pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    const unsigned grid = (r.m_pad / 64) * (r.n_pad / 64);
    auto go = [&](auto kern) {
        if (e0 || e1) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, e0, e1, 0, g);
        else hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, g);
    };
    if (r.s == 4) go(k_gemm_mfma<4, 4>);
    else if (r.s == 2) go(k_gemm_mfma<2, 4>);
    else go(k_gemm_mfma<1, 4>);
    DQT_LAUNCH_CHECK("fgemm(mfma)");
    return DQT_OK;
}

}  // namespace dqt
