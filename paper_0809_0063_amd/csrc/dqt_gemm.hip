// F_p matrix products C = A.B mod p (section 7 of the paper).
//
// Packed path (compressed matrix multiplication, section 7.1, "CMM"): k is cut
// into groups of four; a group of a row of A becomes one 32-bit word of two
// 16-bit lanes, each lane the reversed Kronecker pair a_(2l) Q + a_(2l+1); the
// same group of a column of B becomes b_(2l) + b_(2l+1) Q.  One
// v_dot2_u32_u16 of the two words adds the two lane products into a 32-bit
// accumulator whose digit of weight Q (the middle product) collects four
// multiply-adds of the dot product.  Digits never carry while the number of
// accumulated k (the delayed-reduction interval) times (p-1)^2 stays below Q
// (eq:lower); the accumulator wraps modulo 2^32 above digit 1, which leaves
// digits 0 and 1 exact.  After the interval the middle digit is extracted and
// added to a plain accumulator.  One reduction per output ends the product
// (REDC, section 7.2), or the middle digits of several outputs are gathered
// into one word and reduced by one REDQ (section 3).
//
// Comparators in the same kernel structure: one entry per word and one
// v_mad_u32_u24 per multiply-add ("plain", the paper's delayed baseline),
// four u8 entries per word with v_dot4_u32_u8, and eight 4-bit entries per
// word with v_dot8_u32_u4 (p <= 16).  The INT8 matrix-core comparator is in
// dqt_gemm_mfma.hip.
//
// Layout on the device (workspace, written by the pack kernel each call):
//   CA: [m_pad/TM][KW][TM] uint32: the words of the TM rows of a row block at
//       consecutive k-groups are consecutive, so one unrolled step of the k
//       loop reads them with scalar loads from one base address;
//   CB: [n_pad/(64 TN)][KW][64 TN] uint32: the words of a column block at one
//       k-group are consecutive, lane l of a wave holding columns
//       l TN .. l TN + TN - 1 (one vector load per lane and k-group).
// Each wave owns TM rows (uniform, held in SGPRs) and 64*TN columns; S waves
// of a workgroup split k and add their partial sums through LDS before the
// epilogue.  On this chip every instruction of the k loop other than the
// dot product costs an issue slot of the SIMD, so the layouts exist to keep
// the loop down to the dot products, one scalar and one vector load per
// k-group and a pointer increment per unrolled step.

#include <string.h>

#include <hip/hip_ext.h>

#include "dqt_gemm_tile.h"
#include "dqt_internal.h"

namespace dqt {

// Logical tile of a workgroup: on a launch whose size is a multiple of 8,
// workgroup i runs on XCD i mod 8; consecutive logical tiles on one XCD share
// a column block so that the XCD's L2 keeps one slice of CB.
__device__ __forceinline__ void tile_of(uint32_t bid, uint32_t nblk, uint32_t nrb, uint32_t* rb, uint32_t* cb) {
    uint32_t logical = bid;
    if ((nblk & 7u) == 0) logical = (bid & 7u) * (nblk >> 3) + (bid >> 3);
    *rb = logical % nrb;
    *cb = logical / nrb;
}

template <int OP, int TM, int TN, int S, bool FLUSH, int EPI>
__global__ __launch_bounds__(64 * S) void k_gemm_words(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint32_t red[TileSmem<TM, TN, S>::words];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t rb, cb;
    tile_of(blockIdx.x, gridDim.x, g.nrb, &rb, &cb);
    gemm_tile<OP, TM, TN, S, FLUSH, EPI>(g, rb, cb, wave, lane, red);
}

// Pack A (rows, reversed pairs) and B (columns) into the word layouts.
// Grid: blocks [0, nba) pack A, blocks [nba, ...) pack B; 256 threads, one word each.
__global__ __launch_bounds__(256) void k_gemm_pack(PackArgs a) { gemm_pack_block(a, blockIdx.x, threadIdx.x); }

// Coalesced packing of the four-entry layouts when rows start on 4-byte
// boundaries.  A: a workgroup packs a 64-row x 16-word tile of A (one dword
// of a row per word) through LDS and writes it as the 64/TM row blocks of the
// tile-major layout.  B: a thread takes four consecutive columns of one
// k-group (one dword from each of four rows) and writes their four words.
// Blocks [0, nta) pack A tiles, the rest pack B.
struct Pack4Args {
    PackArgs a;
    uint32_t nta;           // A tiles
    uint32_t tiles_m;       // A tiles along rows
};

__global__ __launch_bounds__(256) void k_gemm_pack4(Pack4Args pa) {
    const PackArgs& a = pa.a;
    if (blockIdx.x < pa.nta) {
        __shared__ uint32_t tile[16][65];
        const uint32_t tr = blockIdx.x % pa.tiles_m, tw = blockIdx.x / pa.tiles_m;
        const uint32_t r0 = tr * 64, w0 = tw * 16;
        const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t rr = wave * 16 + it * 4 + (lane >> 4);
            const uint32_t ww = lane & 15u;
            const uint32_t row = r0 + rr, kw = w0 + ww;
            uint32_t w = 0;
            if (row < a.m && kw < a.KW) {
                uint32_t e[4] = {0, 0, 0, 0};
                if (4 * kw + 3 < a.kdim) {
                    const uint32_t d = *reinterpret_cast<const uint32_t*>(a.A + (size_t)row * a.lda + 4 * kw);
                    e[0] = d & 0xFF;
                    e[1] = (d >> 8) & 0xFF;
                    e[2] = (d >> 16) & 0xFF;
                    e[3] = d >> 24;
                } else {
                    for (uint32_t i = 0; i < 4; ++i)
                        if (4 * kw + i < a.kdim) e[i] = a.A[(size_t)row * a.lda + 4 * kw + i];
                }
                w = pack_a_word(a.op, a.b, e);
            }
            tile[ww][rr] = w;
        }
        __syncthreads();
        // out: row block s of the tile, k-group ww, row i: consecutive threads
        // write consecutive words of one row block
        const uint32_t rb0 = r0 / a.tm;
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t t = it * 256 + threadIdx.x;
            const uint32_t i = t % a.tm, ww = (t / a.tm) % 16, sb = t / (16 * a.tm);
            const uint32_t row = r0 + sb * a.tm + i, kw = w0 + ww;
            if (kw < a.KW && row < a.m_pad)
                a.CA[((size_t)(rb0 + sb) * a.KW + kw) * a.tm + i] = tile[ww][sb * a.tm + i];
        }
    } else {
        const uint64_t t = (uint64_t)(blockIdx.x - pa.nta) * 256 + threadIdx.x;
        const uint32_t q4 = a.n_pad / 4;
        if (t >= (uint64_t)a.KW * q4) return;
        const uint32_t kw = (uint32_t)(t / q4), c4 = (uint32_t)(t % q4) * 4;
        uint32_t d[4] = {0, 0, 0, 0};
        for (uint32_t i = 0; i < 4; ++i) {
            const uint32_t k = 4 * kw + i;
            if (k >= a.kdim) continue;
            if (c4 + 3 < a.n) {
                d[i] = *reinterpret_cast<const uint32_t*>(a.B + (size_t)k * a.ldb + c4);
            } else {
                for (uint32_t j = 0; j < 4; ++j)
                    if (c4 + j < a.n) d[i] |= (uint32_t)a.B[(size_t)k * a.ldb + c4 + j] << (8 * j);
            }
        }
        uint4 out;
        uint32_t* o = reinterpret_cast<uint32_t*>(&out);
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t e[4] = {(d[0] >> (8 * j)) & 0xFF, (d[1] >> (8 * j)) & 0xFF, (d[2] >> (8 * j)) & 0xFF,
                                   (d[3] >> (8 * j)) & 0xFF};
            o[j] = pack_b_word(a.op, a.b, e);
        }
        const uint32_t cb = c4 / a.cbw, c = c4 % a.cbw;
        *reinterpret_cast<uint4*>(a.CB + ((size_t)cb * a.KW + kw) * a.cbw + c) = out;
    }
}

// ---------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------


static uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// Largest interval (in k) and its Q for the packed path: L (p-1)^2 < Q and
// (p-1)(Q+1) < 2^16 so that a Kronecker pair fits one 16-bit lane, 2 log2 Q <= 32.
// Returns false when not even four multiply-adds fit.
bool cmm_params(uint32_t p, uint64_t kdim, uint32_t want_interval, uint32_t want_b, uint32_t* b_out,
                uint32_t* interval_out) {
    const uint64_t e2 = (uint64_t)(p - 1) * (p - 1);
    uint32_t bmax = 0;
    for (uint32_t b = 1; b <= 16; ++b)
        if ((uint64_t)(p - 1) * ((1ull << b) + 1) < 65536ull) bmax = b;
    if (want_b) {
        if (want_b > bmax) return false;
        bmax = want_b;
    }
    if (e2 == 0) {  // p = 2 with (p-1)^2 = 1 handled by the general formula below
    }
    // interval L (multiple of 4) with L * (p-1)^2 < 2^bmax
    uint64_t lmax = e2 ? ((1ull << bmax) - 1) / e2 : kdim;
    lmax = lmax / 4 * 4;
    if (lmax < 4) return false;
    uint64_t L = kdim <= lmax ? round_up(kdim ? kdim : 4, 4) : lmax;
    if (want_interval) {
        if (want_interval % 4 || want_interval > lmax) return false;
        L = want_interval < round_up(kdim, 4) ? want_interval : round_up(kdim, 4);
    }
    // smallest Q for that interval: L (p-1)^2 < Q (strict, eq:lower)
    uint32_t b = 1;
    while (b < bmax && !((1ull << b) > L * e2)) ++b;
    if (!((1ull << b) > L * e2)) return false;
    if (want_b) b = want_b;
    *b_out = b;
    *interval_out = (uint32_t)L;
    return true;
}

static dqt_status resolve_plan(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan* plan,
                               GemmPlanResolved* r) {
    memset(r, 0, sizeof(*r));
    dqt_gemm_plan pl;
    memset(&pl, 0, sizeof(pl));
    if (plan) pl = *plan;
    if (p < 2 || p > 255) return DQT_E_INVALID;
    if (m > 0x7FFFFFFFull || n > 0x7FFFFFFFull || kdim > 0x7FFFFFFFull) return DQT_E_INVALID;
    uint32_t algo = pl.algo;
    if (algo == DQT_GEMM_BY_SHAPE) {
        // section 7.6.2: the middle product when the common dimension is the
        // largest, Right compression when n is, Left compression when m is
        // (each when its words hold at least two digits)
        uint32_t pick = DQT_GEMM_AUTO;
        if (kdim < m || kdim < n) pick = n >= m ? DQT_GEMM_RIGHT : DQT_GEMM_LEFT;
        if (pick != DQT_GEMM_AUTO && f64_plan(pick, p, m, n, kdim, pl.log2Q, pl.ksplit, r) == DQT_OK) return DQT_OK;
        memset(r, 0, sizeof(*r));
        algo = DQT_GEMM_AUTO;
        pl.log2Q = 0;
    }
    if (is_f64_algo(algo)) return f64_plan(algo, p, m, n, kdim, pl.log2Q, pl.ksplit, r);
    uint32_t b = 0, interval = 0;
    // Every kernel of this file adds whole dot products (each at most
    // kdim (p-1)^2) in uint32: the middle digits of all intervals and k-splits
    // of the packed path as well as the plain sums.  Above 2^32 they would wrap.
    const bool sums_fit = kdim * (uint64_t)(p - 1) * (p - 1) < (1ull << 32);
    const bool cmm_ok = cmm_params(p, kdim, pl.interval, pl.log2Q, &b, &interval);
    if (algo == DQT_GEMM_AUTO) algo = cmm_ok ? DQT_GEMM_CMM : DQT_GEMM_PLAIN;
    r->algo = algo;
    r->epi = pl.epilogue;
    if (r->epi > 1) return DQT_E_INVALID;
    switch (algo) {
        case DQT_GEMM_CMM:
            if (!sums_fit) return DQT_E_UNSUPPORTED;
            if (!cmm_ok) return (pl.interval || pl.log2Q) ? DQT_E_BOUND : DQT_E_UNSUPPORTED;
            r->op = OP_DOT2;
            r->b = b;
            r->lw = interval >= round_up(kdim, 4) ? 0 : interval / 4;
            break;
        case DQT_GEMM_PLAIN:
            r->op = OP_MAD;
            if (!sums_fit) return DQT_E_UNSUPPORTED;
            if (r->epi) return DQT_E_UNSUPPORTED;
            break;
        case DQT_GEMM_DOT4:
            r->op = OP_DOT4;
            if (!sums_fit) return DQT_E_UNSUPPORTED;
            if (r->epi) return DQT_E_UNSUPPORTED;
            break;
        case DQT_GEMM_DOT8:
            r->op = OP_DOT8;
            if (p > 16) return DQT_E_UNSUPPORTED;   // entries must fit four bits
            if (!sums_fit) return DQT_E_UNSUPPORTED;
            if (r->epi) return DQT_E_UNSUPPORTED;
            break;
        case DQT_GEMM_MFMA:
            if (r->epi) return DQT_E_UNSUPPORTED;
            return mfma_plan(p, m, n, kdim, r);
        default:
            return DQT_E_UNSUPPORTED;
    }
    // Tile shape: fixed defaults (not derived from m or n), so that the packed
    // layout of one operand never depends on the other operand's size.
    r->tm = pl.tile_rows ? pl.tile_rows : 8;
    r->tn = pl.tile_cols ? pl.tile_cols : 4;
    if (r->tm != 8 && r->tm != 16 && r->tm != 32) return DQT_E_INVALID;
    if (r->tn != 2 && r->tn != 4) return DQT_E_INVALID;
    if (r->tm == 32 && r->tn == 4) return DQT_E_INVALID;
    const uint32_t epw = entries_per_word(r->op);
    r->KW = (uint32_t)((kdim + epw - 1) / epw);
    if (pl.ksplit) {
        r->s = pl.ksplit;
    } else {
        // enough waves to fill the chip: aim at >= 8 waves per CU
        const uint64_t tiles = ((m + r->tm - 1) / r->tm) * ((n + 64 * r->tn - 1) / (64 * r->tn));
        r->s = 1;
        while (r->s < 8 && tiles * r->s < 4096 && (uint64_t)r->KW / (r->s * 2) >= 16) r->s *= 2;
    }
    if (r->s != 1 && r->s != 2 && r->s != 4 && r->s != 8) return DQT_E_INVALID;
    // the split-k reduction buffer (s tm tn 64 words) stays within 64 KB of LDS
    if (pl.ksplit && (uint64_t)r->s * r->tm * r->tn * 256 > 65536) return DQT_E_INVALID;
    while ((uint64_t)r->s * r->tm * r->tn * 256 > 65536) r->s /= 2;
    // split-k boundaries must fall on interval boundaries of the packed path
    r->m_pad = (uint32_t)round_up(m ? m : 1, r->tm);
    r->n_pad = (uint32_t)round_up(n ? n : 1, 64 * r->tn);
    r->ws_bytes = (size_t)r->KW * (r->m_pad + r->n_pad) * sizeof(uint32_t);
    if (r->epi == 1 && r->op != OP_DOT2) return DQT_E_UNSUPPORTED;
    return DQT_OK;
}

// Events that the next multiply-kernel launch of this thread records at its
// own start and end (dqt_fgemm_compute_timed); null for ordinary launches.
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

template <int OP, int TM, int TN, int S, bool FLUSH, int EPI>
static void launch_words_k(const GemmArgs& g, unsigned grid, hipStream_t s) {
    if (g_ev_start || g_ev_stop)
        hipExtLaunchKernelGGL(k_gemm_words<OP, TM, TN, S, FLUSH, EPI>, dim3(grid), dim3(64 * S), 0, s, g_ev_start,
                              g_ev_stop, 0, g);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_words<OP, TM, TN, S, FLUSH, EPI>), dim3(grid), dim3(64 * S), 0, s,
                           g);
}

template <int OP, int TM, int TN, int S>
static void launch_words(const GemmArgs& g, unsigned grid, hipStream_t s) {
    if (OP == OP_DOT2) {
        if (g.lw) {
            if (g.epi) launch_words_k<OP, TM, TN, S, true, 1>(g, grid, s);
            else launch_words_k<OP, TM, TN, S, true, 0>(g, grid, s);
        } else {
            if (g.epi) launch_words_k<OP, TM, TN, S, false, 1>(g, grid, s);
            else launch_words_k<OP, TM, TN, S, false, 0>(g, grid, s);
        }
    } else {
        launch_words_k<OP, TM, TN, S, false, 0>(g, grid, s);
    }
}

template <int OP, int TM, int TN>
static void launch_words_s(const GemmArgs& g, unsigned grid, uint32_t S_, hipStream_t s) {
    switch (S_) {
        case 1: launch_words<OP, TM, TN, 1>(g, grid, s); break;
        case 2: launch_words<OP, TM, TN, 2>(g, grid, s); break;
        case 4: launch_words<OP, TM, TN, 4>(g, grid, s); break;
        default:
            // plans whose reduction buffer exceeds 64 KB are refused by resolve_plan
            if constexpr (8 * TM * TN * 256 <= 65536) launch_words<OP, TM, TN, 8>(g, grid, s);
            break;
    }
}

// (TM, TN) in {(8,2), (8,4), (16,2), (16,4), (32,2)} (checked by resolve_plan)
template <int OP>
static void launch_words_tm(const GemmArgs& g, unsigned grid, uint32_t tm, uint32_t tn, uint32_t S_, hipStream_t s) {
    if (tn == 4) {
        if (tm == 8) launch_words_s<OP, 8, 4>(g, grid, S_, s);
        else launch_words_s<OP, 16, 4>(g, grid, S_, s);
    } else {
        switch (tm) {
            case 8: launch_words_s<OP, 8, 2>(g, grid, S_, s); break;
            case 16: launch_words_s<OP, 16, 2>(g, grid, S_, s); break;
            default: launch_words_s<OP, 32, 2>(g, grid, S_, s); break;
        }
    }
}

// C = 0 for an empty inner dimension (every dot product is the empty sum).
__global__ __launch_bounds__(256) void k_zero_c(uint8_t* C, uint64_t m, uint64_t n, uint64_t ldc) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < m * n; t += (uint64_t)gridDim.x * 256)
        C[(t / n) * ldc + t % n] = 0;
}

static dqt_status zero_c(uint8_t* C, uint64_t m, uint64_t n, uint64_t ldc, hipStream_t s) {
    DQT_TRY(ensure_device_ready());
    hipLaunchKernelGGL(k_zero_c, dim3(stream_grid(m * n, 256, 4)), dim3(256), 0, s, C, m, n, ldc);
    DQT_LAUNCH_CHECK("fgemm(k = 0)");
    return DQT_OK;
}

dqt_status fgemm_epilogue_args(uint32_t p, uint64_t kdim, const GemmPlanResolved& r, GemmArgs* g) {
    g->epi = r.epi;
    if (r.epi == 1) {
        // The gathered values are whole dot products (all intervals and all
        // k-splits added), at most kdim (p-1)^2: they are the digits of the
        // REDQ word, so its q is the smallest power of two above that bound,
        // and e = floor(53 / log2 q) of them share one word (section 7.6.1).
        const uint64_t maxdot = (uint64_t)kdim * (p - 1) * (p - 1);
        uint32_t be = residue_bits(p);
        while (be < 32 && (1ull << be) <= maxdot) ++be;
        uint32_t e = 53 / be;
        if (e > 8) e = 8;
        if (e < 1) return DQT_E_UNSUPPORTED;
        g->epi_e = e;
        DQT_TRY(make_redq_args(p, be, e, e * be, &g->ra));
    }
    return DQT_OK;
}

// Bytes of the packed copy of one side (0 = A, 1 = B).
static size_t side_bytes(const GemmPlanResolved& r, int side) {
    if (is_f64_algo(r.algo)) return f64_side_bytes(r, side);
    if (r.algo == DQT_GEMM_MFMA) return mfma_side_bytes(r, side);
    return (size_t)r.KW * (side == 0 ? r.m_pad : r.n_pad) * sizeof(uint32_t);
}

// Packing step: operands to the word layout of the plan's kernel, A's packed
// copy to pA and B's to pB (either operand may be skipped by passing NULL,
// to reuse a packed one; its target is then not touched).
static dqt_status fgemm_pack_sides(uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A, uint64_t lda,
                                   const uint8_t* B, uint64_t ldb, const GemmPlanResolved& r, void* pA, void* pB,
                                   hipStream_t s) {
    if (is_f64_algo(r.algo)) return f64_pack_enqueue(r, m, n, kdim, A, lda, B, ldb, pA, pB, s);
    if (r.algo == DQT_GEMM_MFMA) return mfma_pack_enqueue(r, m, n, kdim, A, lda, B, ldb, pA, pB, s);
    uint32_t* CA = reinterpret_cast<uint32_t*>(pA);
    uint32_t* CB = reinterpret_cast<uint32_t*>(pB);
    PackArgs pa;
    pa.A = A;
    pa.B = B;
    pa.CA = CA;
    pa.CB = CB;
    pa.m = (uint32_t)m;
    pa.n = (uint32_t)n;
    pa.kdim = (uint32_t)kdim;
    pa.lda = (uint32_t)lda;
    pa.ldb = (uint32_t)ldb;
    pa.m_pad = r.m_pad;
    pa.n_pad = r.n_pad;
    pa.KW = r.KW;
    pa.b = r.b;
    pa.op = r.op;
    pa.tm = r.tm;
    pa.cbw = 64 * r.tn;
    const bool a_al = !A || (((uintptr_t)A & 3) == 0 && (lda & 3) == 0);
    const bool b_al = !B || (((uintptr_t)B & 3) == 0 && (ldb & 3) == 0);
    const bool out_al = (!A || ((uintptr_t)pA & 15) == 0) && (!B || ((uintptr_t)pB & 15) == 0);
    if ((r.op == OP_DOT2 || r.op == OP_DOT4) && a_al && b_al && (r.n_pad & 3) == 0 && out_al) {
        Pack4Args p4;
        p4.a = pa;
        p4.tiles_m = (r.m_pad + 63) / 64;
        p4.nta = A ? p4.tiles_m * ((r.KW + 15) / 16) : 0;
        const uint32_t nbb = B ? (uint32_t)(((uint64_t)r.KW * (r.n_pad / 4) + 255) / 256) : 0;
        if (p4.nta + nbb == 0) return DQT_OK;
        hipLaunchKernelGGL(k_gemm_pack4, dim3(p4.nta + nbb), dim3(256), 0, s, p4);
        DQT_LAUNCH_CHECK("fgemm(pack4)");
        return DQT_OK;
    }
    const uint32_t nba = A ? pack_blocks_for((uint64_t)r.KW * r.m_pad, r.op) : 0;
    const uint32_t nbb = B ? pack_blocks_for((uint64_t)r.KW * r.n_pad, r.op) : 0;
    pa.nba = nba;
    pa.al = (a_al ? 1u : 0u) | (b_al ? 2u : 0u);
    if (r.op != OP_MAD && !out_al) return DQT_E_INVALID;   // 16-byte stores
    if (nba + nbb == 0) return DQT_OK;
    hipLaunchKernelGGL(k_gemm_pack, dim3(nba + nbb), dim3(256), 0, s, pa);
    DQT_LAUNCH_CHECK("fgemm(pack)");
    return DQT_OK;
}

// Packing step into a workspace: A's packed copy at its start, B's after it.
dqt_status fgemm_pack_enqueue(uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A, uint64_t lda, const uint8_t* B,
                              uint64_t ldb, const GemmPlanResolved& r, void* work, hipStream_t s) {
    uint8_t* w = reinterpret_cast<uint8_t*>(work);
    return fgemm_pack_sides(m, n, kdim, A, lda, B, ldb, r, w, w + side_bytes(r, 0), s);
}

// Multiplication and extraction on packed operands.
dqt_status fgemm_compute_enqueue2(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t* C, uint64_t ldc,
                                  const GemmPlanResolved& r, const void* pA, const void* pB, hipStream_t s) {
    const uint32_t pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    if (is_f64_algo(r.algo)) {
        if (((uintptr_t)pA & 15) || ((uintptr_t)pB & 15)) {
            set_error("fgemm: packed operands (workspace) must be 16-byte aligned");
            return DQT_E_INVALID;
        }
        return f64_compute_enqueue(r, p, m, n, C, ldc, pA, pB, s, g_ev_start, g_ev_stop);
    }
    if (r.algo == DQT_GEMM_MFMA) return mfma_compute_enqueue(r, p, m, n, C, ldc, pA, pB, s, g_ev_start, g_ev_stop);
    // the k loop reads B with 8- or 16-byte vector loads
    if (((uintptr_t)pA & 15) || ((uintptr_t)pB & 15)) {
        set_error("fgemm: packed operands (workspace) must be 16-byte aligned");
        return DQT_E_INVALID;
    }
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.CA = reinterpret_cast<const uint32_t*>(pA);
    g.CB = reinterpret_cast<const uint32_t*>(pB);
    g.C = C;
    g.m = (uint32_t)m;
    g.n = (uint32_t)n;
    g.ldc = (uint32_t)ldc;
    g.m_pad = r.m_pad;
    g.n_pad = r.n_pad;
    g.KW = r.KW;
    // split-k boundaries on interval boundaries (packed path)
    uint32_t ks = (r.KW + r.s - 1) / r.s;
    if (r.lw) ks = (uint32_t)round_up(ks, r.lw);
    g.kw_split = ks;
    g.lw = r.lw;
    g.nrb = r.m_pad / r.tm;
    g.ncb = r.n_pad / (64 * r.tn);
    g.b = r.b ? r.b : 1;
    g.p = p;
    g.pmagic = pmagic;
    g.op = r.op;
    DQT_TRY(fgemm_epilogue_args(p, kdim, r, &g));
    const unsigned grid = g.nrb * g.ncb;
    switch (r.op) {
        case OP_DOT2: launch_words_tm<OP_DOT2>(g, grid, r.tm, r.tn, r.s, s); break;
        case OP_DOT4: launch_words_tm<OP_DOT4>(g, grid, r.tm, r.tn, r.s, s); break;
        case OP_DOT8: launch_words_tm<OP_DOT8>(g, grid, r.tm, r.tn, r.s, s); break;
        default: launch_words_tm<OP_MAD>(g, grid, r.tm, r.tn, r.s, s); break;
    }
    DQT_LAUNCH_CHECK("fgemm");
    return DQT_OK;
}

dqt_status fgemm_compute_enqueue(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t* C, uint64_t ldc,
                                 const GemmPlanResolved& r, const void* work, hipStream_t s) {
    const uint8_t* w = reinterpret_cast<const uint8_t*>(work);
    const size_t a_bytes = is_f64_algo(r.algo)        ? f64_side_bytes(r, 0)
                           : r.algo == DQT_GEMM_MFMA ? mfma_side_bytes(r, 0)
                                                     : (size_t)r.KW * r.m_pad * 4;
    return fgemm_compute_enqueue2(p, m, n, kdim, C, ldc, r, w, w + a_bytes, s);
}

dqt_status fgemm_enqueue(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A, uint64_t lda,
                         const uint8_t* B, uint64_t ldb, uint8_t* C, uint64_t ldc, const GemmPlanResolved& r,
                         void* work, hipStream_t s) {
    DQT_TRY(fgemm_pack_enqueue(m, n, kdim, A, lda, B, ldb, r, work, s));
    return fgemm_compute_enqueue(p, m, n, kdim, C, ldc, r, work, s);
}

dqt_status fgemm_resolve(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan* plan,
                         GemmPlanResolved* r) {
    return resolve_plan(p, m, n, kdim, plan, r);
}

}  // namespace dqt

using namespace dqt;

extern "C" size_t dqt_fgemm_workspace_size(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim,
                                           const dqt_gemm_plan* plan) {
    GemmPlanResolved r;
    if (resolve_plan(p, m, n, kdim, plan, &r) != DQT_OK) return 0;
    return r.ws_bytes;
}

static dqt_status fgemm_common_checks(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const dqt_gemm_plan* plan,
                                      size_t work_bytes, const void* d_work, GemmPlanResolved* r) {
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, r));
    if (r->ws_bytes && (!d_work || work_bytes < r->ws_bytes)) return DQT_E_WORKSPACE;
    if (r->ws_bytes && ((uintptr_t)d_work & 15)) return DQT_E_INVALID;
    return DQT_OK;
}

extern "C" dqt_status dqt_fgemm_pack(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* d_A,
                                     uint64_t lda, const uint8_t* d_B, uint64_t ldb, const dqt_gemm_plan* plan,
                                     void* d_work, size_t work_bytes, void* stream) {
    GemmPlanResolved r;
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, &r));
    if (m == 0 || n == 0 || kdim == 0) return DQT_OK;
    if (!d_A && !d_B) return DQT_E_INVALID;
    if ((d_A && lda < kdim) || (d_B && ldb < n) || lda > 0xFFFFFFFFull || ldb > 0xFFFFFFFFull) return DQT_E_INVALID;
    DQT_TRY(fgemm_common_checks(p, m, n, kdim, plan, work_bytes, d_work, &r));
    DQT_TRY(ensure_device_ready());
    DQT_TRY(debug_gate(reinterpret_cast<hipStream_t>(stream), p, {{d_A, m, kdim, lda}, {d_B, kdim, n, ldb}}));
    return fgemm_pack_enqueue(m, n, kdim, d_A, lda, d_B, ldb, r, d_work, reinterpret_cast<hipStream_t>(stream));
}

extern "C" dqt_status dqt_fgemm_compute(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t* d_C, uint64_t ldc,
                                        const dqt_gemm_plan* plan, const void* d_work, size_t work_bytes,
                                        void* stream) {
    GemmPlanResolved r;
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, &r));
    if (m == 0 || n == 0) return DQT_OK;
    if (!d_C || ldc < n || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
    if (kdim == 0) return zero_c(d_C, m, n, ldc, reinterpret_cast<hipStream_t>(stream));
    DQT_TRY(fgemm_common_checks(p, m, n, kdim, plan, work_bytes, d_work, &r));
    DQT_TRY(ensure_device_ready());
    return fgemm_compute_enqueue(p, m, n, kdim, d_C, ldc, r, d_work, reinterpret_cast<hipStream_t>(stream));
}

extern "C" dqt_status dqt_fgemm_compute_timed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, uint8_t* d_C,
                                              uint64_t ldc, const dqt_gemm_plan* plan, const void* d_work,
                                              size_t work_bytes, void* start_event, void* stop_event,
                                              void* stream) {
    GemmPlanResolved r;
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, &r));
    g_ev_start = reinterpret_cast<hipEvent_t>(start_event);
    g_ev_stop = reinterpret_cast<hipEvent_t>(stop_event);
    const dqt_status st = dqt_fgemm_compute(p, m, n, kdim, d_C, ldc, plan, d_work, work_bytes, stream);
    g_ev_start = g_ev_stop = nullptr;
    return st;
}

extern "C" dqt_status dqt_fgemm_timed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* d_A,
                                      uint64_t lda, const uint8_t* d_B, uint64_t ldb, uint8_t* d_C, uint64_t ldc,
                                      const dqt_gemm_plan* plan, void* d_work, size_t work_bytes, void* start_event,
                                      void* stop_event, void* stream) {
    g_ev_start = reinterpret_cast<hipEvent_t>(start_event);
    g_ev_stop = reinterpret_cast<hipEvent_t>(stop_event);
    const dqt_status st = dqt_fgemm(p, m, n, kdim, d_A, lda, d_B, ldb, d_C, ldc, plan, d_work, work_bytes, stream);
    g_ev_start = g_ev_stop = nullptr;
    return st;
}

// Packed operands in caller-chosen buffers (one side at a time), so that a
// packed B can stay resident and be multiplied by many row blocks of A.
static dqt_status side_plan(uint32_t p, uint64_t rows_or_cols, uint64_t kdim, int side, const dqt_gemm_plan* plan,
                            GemmPlanResolved* r) {
    if (side != 0 && side != 1) return DQT_E_INVALID;
    // The layout of a packed side must follow from (p, kdim, plan) alone; the
    // shape rule picks its algorithm from all three dimensions, so a side
    // packed on its own could disagree with the product that reads it.
    if (plan && plan->algo == DQT_GEMM_BY_SHAPE) return DQT_E_INVALID;
    // the packed layout of one side does not depend on the other dimension
    return resolve_plan(p, side == 0 ? rows_or_cols : 1, side == 1 ? rows_or_cols : 1, kdim, plan, r);
}

extern "C" size_t dqt_fgemm_packed_bytes(uint32_t p, uint64_t rows_or_cols, uint64_t kdim, int side,
                                         const dqt_gemm_plan* plan) {
    GemmPlanResolved r;
    if (side_plan(p, rows_or_cols, kdim, side, plan, &r) != DQT_OK) return 0;
    return side_bytes(r, side);
}

extern "C" dqt_status dqt_fgemm_pack_side(uint32_t p, uint64_t rows_or_cols, uint64_t kdim, const uint8_t* d_X,
                                          uint64_t ldx, int side, const dqt_gemm_plan* plan, void* d_packed,
                                          void* stream) {
    GemmPlanResolved r;
    DQT_TRY(side_plan(p, rows_or_cols, kdim, side, plan, &r));
    if (rows_or_cols == 0 || kdim == 0) return DQT_OK;
    if (!d_X || !d_packed || ((uintptr_t)d_packed & 15)) return DQT_E_INVALID;
    if ((side == 0 && ldx < kdim) || (side == 1 && ldx < rows_or_cols) || ldx > 0xFFFFFFFFull) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (side == 0) DQT_TRY(debug_gate(s, p, {{d_X, rows_or_cols, kdim, ldx}}));
    else DQT_TRY(debug_gate(s, p, {{d_X, kdim, rows_or_cols, ldx}}));
    if (side == 0)
        return fgemm_pack_sides(rows_or_cols, 1, kdim, d_X, ldx, nullptr, 1, r, d_packed, nullptr, s);
    return fgemm_pack_sides(1, rows_or_cols, kdim, nullptr, 1, d_X, ldx, r, nullptr, d_packed, s);
}

extern "C" dqt_status dqt_fgemm_packed(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const void* d_CA,
                                       const void* d_CB, uint8_t* d_C, uint64_t ldc, const dqt_gemm_plan* plan,
                                       void* stream) {
    GemmPlanResolved r;
    if (plan && plan->algo == DQT_GEMM_BY_SHAPE) return DQT_E_INVALID;   // as dqt_fgemm_pack_side
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, &r));
    if (m == 0 || n == 0) return DQT_OK;
    if (kdim == 0) {
        if (!d_C || ldc < n || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
        return zero_c(d_C, m, n, ldc, reinterpret_cast<hipStream_t>(stream));
    }
    if (!d_CA || !d_CB || !d_C || ldc < n || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
    if (((uintptr_t)d_CA & 15) || ((uintptr_t)d_CB & 15)) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    return fgemm_compute_enqueue2(p, m, n, kdim, d_C, ldc, r, d_CA, d_CB, reinterpret_cast<hipStream_t>(stream));
}

extern "C" dqt_status dqt_fgemm(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* d_A, uint64_t lda,
                                const uint8_t* d_B, uint64_t ldb, uint8_t* d_C, uint64_t ldc,
                                const dqt_gemm_plan* plan, void* d_work, size_t work_bytes, void* stream) {
    GemmPlanResolved r;
    DQT_TRY(resolve_plan(p, m, n, kdim, plan, &r));
    if (m == 0 || n == 0) return DQT_OK;
    if (kdim == 0) {
        if (!d_C || ldc < n || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
        return zero_c(d_C, m, n, ldc, reinterpret_cast<hipStream_t>(stream));
    }
    if (!d_A || !d_B || !d_C) return DQT_E_INVALID;
    if (lda < kdim || ldb < n || ldc < n) return DQT_E_INVALID;
    if (lda > 0xFFFFFFFFull || ldb > 0xFFFFFFFFull || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
    if (r.ws_bytes && (!d_work || work_bytes < r.ws_bytes)) return DQT_E_WORKSPACE;
    if (r.ws_bytes && ((uintptr_t)d_work & 15)) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    DQT_TRY(debug_gate(reinterpret_cast<hipStream_t>(stream), p, {{d_A, m, kdim, lda}, {d_B, kdim, n, ldb}}));
    return fgemm_enqueue(p, m, n, kdim, d_A, lda, d_B, ldb, d_C, ldc, r, d_work, reinterpret_cast<hipStream_t>(stream));
}
