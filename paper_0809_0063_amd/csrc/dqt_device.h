// Device-side building blocks of the packed-DQT / REDQ path (gfx950).
//
// Notation follows the paper: p the prime, q = 2^b the evaluation point,
// w = ceil(log2 p) the bit width of a residue, nres the number of q-adic
// digits of a packed word (REDQ_nres), c = q mod p the correction constant.
//
// The helpers take B and W as template parameters: a positive value fixes
// b or w at compile time (shifts, masks and index gathers become constants);
// 0 reads them from RedqArgs at run time.  Both give the same results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqt {

// Parameters of one REDQ_nres (section 3), precomputed on the host.
struct RedqArgs {
    double invp;       // smallest binary64 >= 1/p (AFDIV: o1 = up, o2 = nearest)
    double invp52;     // 2^52 * invp (exact)
    uint64_t M;        // w-bit field masks at bit b*i, i < nres
    uint64_t G;        // guard 2^(2w) at bit b*i (field-parallel compression)
    uint32_t p, b, w, nres;
    uint32_t c;        // q mod p; 0 means p | q and no correction
    uint32_t fix;      // words may reach B = 2^53/(3+2^-52): one-sided AFDIV test
    uint32_t swar;     // b >= 2w+1: all u_i from one masked multiply-subtract
    uint32_t tabj;     // correction table window: 3 (2 outputs), 2 (1 output), 0 = arithmetic
    uint32_t pmagic;   // ceil(2^32 / p): x mod p = x - p*mulhi(x, pmagic) for x < 2^24
    uint32_t tab_entries;  // 2^(tabj*w), or 0
    uint32_t small;    // words < 2^52 (fast binary64 floor, no AFDIV test)
    uint32_t pad;
};

// High 32 bits of a 32 x 32-bit product (v_mul_hi_u32 on the device).
__host__ __device__ __forceinline__ uint32_t mulhi_u32(uint32_t x, uint32_t y) {
    return (uint32_t)(((uint64_t)x * y) >> 32);
}

// x mod p for x < 2^24 and p < 2^8, by the precomputed reciprocal (a REDC).
__host__ __device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t p, uint32_t pmagic) {
    uint32_t qt = mulhi_u32(x, pmagic);
    uint32_t r = x - qt * p;
    return r >= p ? r - p : r;
}

// floor(r / p) for r < 2^53 by one binary64 multiply (algorithm FDIV, case 2
// of table tab:fdiv: invp rounded up on the host, the product rounded to
// nearest, the default mode of the device).  floor(x) is k or k+1; it can only
// be k+1 when r >= 2^53/(3+2^-52), where the single test of AFDIV corrects it.
//
// For r < 2^52 the conversions are bit operations: the binary64 whose bit
// pattern is 2^52's exponent with r in the mantissa is 2^52 + r, so
// fma(2^52 + r, invp, -2^52 invp) is r * invp rounded once (the same x), and
// floor(x) + 2^52 carries floor(x) in its mantissa bits.
template <bool SMALL>
__host__ __device__ __forceinline__ uint64_t fdiv_floor(uint64_t r, const struct RedqArgs& a) {
#pragma clang fp contract(off)
    if (SMALL) {
        const double z = __builtin_bit_cast(double, r | 0x4330000000000000ull);
        const double x = __builtin_fma(z, a.invp, -a.invp52);
        const double t = __builtin_floor(x) + 4503599627370496.0;
        return __builtin_bit_cast(uint64_t, t) & 0x000FFFFFFFFFFFFFull;
    }
    const double hi = (double)(uint32_t)(r >> 32);
    const double lo = (double)(uint32_t)r;
    const double rd = hi * 4294967296.0 + lo;  // exact: r < 2^53
    const double x = rd * a.invp;
    const double y = __builtin_floor(x);
    uint64_t s = (uint64_t)y;
    if (a.fix) {
        if (s * (uint64_t)a.p > r) s -= 1;
    }
    return s;
}

// Compile-time masks of the field-parallel compression.
template <int NR, int B, int W>
struct SwarMasks {
    static constexpr uint64_t mask() {
        uint64_t m = 0;
        for (int i = 0; i < NR; ++i) m |= (uint64_t)((1u << W) - 1u) << (B * i);
        return m;
    }
    static constexpr uint64_t guard() {
        uint64_t g = 0;
        for (int i = 0; i < NR; ++i) g |= (uint64_t)1 << (B * i + 2 * W);
        return g;
    }
};

// REDQ compression (algorithm REDQ, first part, binary case of section 3.3):
// returns U with u_i = floor(r/q^i) - p*floor(s/q^i) in the w low bits of the
// field at bit b*i, zeros elsewhere.  Since u_i < p <= 2^w, only the w low bits
// of floor(r/q^i) and floor(s/q^i) matter; with 2w+1 bits per field all fields
// are computed by one masked multiply-subtract (each field value stays in
// [1, 2^(2w+1)), so no borrow or carry crosses a field).
template <int NR, int B, int W, bool SMALL>
__host__ __device__ __forceinline__ uint64_t redq_compress_t(uint64_t r, const RedqArgs& a) {
    const uint64_t s = fdiv_floor<SMALL>(r, a);
    if (B && W && B >= 2 * W + 1 && NR > 0) {
        constexpr uint64_t M = SwarMasks<(NR > 0 ? NR : 1), (B ? B : 1), (W ? W : 1)>::mask();
        constexpr uint64_t G = SwarMasks<(NR > 0 ? NR : 1), (B ? B : 1), (W ? W : 1)>::guard();
        const uint64_t z = ((r & M) | G) - (uint64_t)a.p * (s & M);
        return z & M;
    }
    if (a.swar) {
        const uint64_t z = ((r & a.M) | a.G) - (uint64_t)a.p * (s & a.M);
        return z & a.M;
    }
    uint64_t U = 0;
    const uint32_t b = B ? B : a.b, w = W ? W : a.w;
    const uint32_t wm = (1u << w) - 1u;
    for (uint32_t i = 0; i < a.nres; ++i) {
        const uint32_t sh = b * i;
        const uint32_t ui = ((uint32_t)(r >> sh) - a.p * (uint32_t)(s >> sh)) & wm;
        U |= (uint64_t)ui << sh;
    }
    return U;
}

// Run-time form (words up to 2^53).
__host__ __device__ __forceinline__ uint64_t redq_compress(uint64_t r, const RedqArgs& a) {
    return redq_compress_t<0, 0, 0, false>(r, a);
}

// Residue i of U (w bits at b*i).
template <int B = 0, int W = 0>
__host__ __device__ __forceinline__ uint32_t field(uint64_t U, uint32_t i, const RedqArgs& a) {
    const uint32_t b = B ? B : a.b, w = W ? W : a.w;
    return (uint32_t)(U >> (b * i)) & ((1u << w) - 1u);
}

// Correction of one residue without a table: (u_i - c*u_{i+1}) mod p.
__host__ __device__ __forceinline__ uint32_t correct_arith(uint32_t ui, uint32_t ui1, const RedqArgs& a) {
    return mod_small(ui + a.p * a.p - a.c * ui1, a.p, a.pmagic);
}

// Build the correction table in LDS: for window j = tabj, entry
// idx = u_0 | u_1 << w | ... | u_{j-1} << (j-1)w holds the j-1 corrected
// residues mu_t = (u_t - c*u_{t+1}) mod p as bytes (section 3.5: the first
// j-1 rows of Q_{j-1} times a window of j residues, binary indexing).
__host__ __device__ __forceinline__ uint16_t correction_entry(uint32_t idx, const RedqArgs& a) {
    const uint32_t wm = (1u << a.w) - 1u;
    const uint32_t u0 = idx & wm, u1 = (idx >> a.w) & wm;
    uint32_t e = mod_small(u0 + a.p * a.p - a.c * u1, a.p, a.pmagic);
    if (a.tabj == 3) {
        const uint32_t u2 = (idx >> (2 * a.w)) & wm;
        e |= mod_small(u1 + a.p * a.p - a.c * u2, a.p, a.pmagic) << 8;
    }
    return (uint16_t)e;
}

__device__ __forceinline__ void build_correction_table(uint16_t* tab, const RedqArgs& a) {
    if (a.tabj == 0) return;
    for (uint32_t idx = threadIdx.x; idx < a.tab_entries; idx += blockDim.x) tab[idx] = correction_entry(idx, a);
}

// Gathering three w-bit fields spaced b apart into one 3w-bit index with one
// multiply: the nine partial products land on distinct, non-overlapping bit
// ranges of a 32-bit word exactly when this holds.
template <int B, int W>
__host__ __device__ constexpr bool gather3_by_multiply() {
    if (B <= W || 2 * B + W > 32) return false;
    int pos[9] = {};
    int n = 0;
    for (int t = 0; t < 3; ++t)
        for (int u = 0; u < 3; ++u) pos[n++] = B * t + (B - W) * (2 - u);
    for (int x = 0; x < 9; ++x) {
        if (pos[x] + W > 32) return false;
        for (int y = x + 1; y < 9; ++y) {
            const int d = pos[x] > pos[y] ? pos[x] - pos[y] : pos[y] - pos[x];
            if (d < W) return false;
        }
    }
    return true;
}

// Table index of the window of `j` residues starting at residue s.
template <int B = 0, int W = 0>
__host__ __device__ __forceinline__ uint32_t window_index(uint64_t U, uint32_t s, uint32_t j, const RedqArgs& a) {
    const uint32_t b = B ? B : a.b, w = W ? W : a.w;
    const uint32_t x = (uint32_t)(U >> (b * s));
    if constexpr (B && W && gather3_by_multiply<(B ? B : 1), (W ? W : 1)>()) {
        if (j == 3) {
            constexpr uint32_t wm = (1u << (W ? W : 1)) - 1u;
            constexpr uint32_t fm = wm | (wm << (B ? B : 1)) | (wm << (2 * (B ? B : 1)));
            constexpr uint32_t mul = 1u | (1u << ((B ? B : 1) - (W ? W : 1))) | (1u << (2 * ((B ? B : 1) - (W ? W : 1))));
            constexpr uint32_t sh = 2 * ((B ? B : 1) - (W ? W : 1));
            return ((x & fm) * mul >> sh) & ((1u << (3 * (W ? W : 1))) - 1u);
        }
    }
    const uint32_t wm = (1u << w) - 1u;
    if ((j - 1) * b + w > 32) {
        // the window spans more than 32 bits of U: gather its fields from 64 bits
        const uint64_t y = U >> (b * s);
        uint32_t idx = (uint32_t)(y & wm);
        idx |= (uint32_t)((y >> b) & wm) << w;
        if (j == 3) idx |= (uint32_t)((y >> (2 * b)) & wm) << (2 * w);
        return idx;
    }
    uint32_t idx = x & wm;
    idx |= ((x >> b) & wm) << w;
    if (j == 3) idx |= ((x >> (2 * b)) & wm) << (2 * w);
    return idx;
}

// Full REDQ correction: writes mu_0 .. mu_{nres-1} (section 3.2, second part)
// through `put(i, mu_i)`.  With p | q the compressed residues are final.
template <int NR, int B = 0, int W = 0, class Put>
__host__ __device__ __forceinline__ void redq_correct(uint64_t U, const RedqArgs& a, const uint16_t* tab, Put put) {
    // Every branch fills all of r[] (compile-time indices), and the values are
    // handed to `put` after the branches: the array stays in registers.
    uint32_t r[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) r[i] = field<B, W>(U, i, a);
    if (a.c != 0 && NR > 1) {
        if (a.tabj == 3 && NR >= 3) {
            // windows of 3 residues overlapping by one; the last is shifted down to end at u_{NR-1}
            uint32_t t[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) t[i] = r[i];
#pragma unroll
            for (int s0 = 0; s0 < NR - 1; s0 += 2) {
                const int s = (s0 + 3 > NR) ? NR - 3 : s0;
                const uint32_t e = tab[window_index<B, W>(U, s, 3, a)];
                t[s] = e & 0xFF;
                t[s + 1] = e >> 8;
            }
#pragma unroll
            for (int i = 0; i < NR; ++i) r[i] = t[i];
        } else if (a.tabj >= 2) {
#pragma unroll
            for (int s = 0; s < NR - 1; ++s) r[s] = tab[window_index<B, W>(U, s, 2, a)] & 0xFF;
        } else {
#pragma unroll
            for (int s = 0; s < NR - 1; ++s) r[s] = correct_arith(r[s], r[s + 1], a);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) put(i, r[i]);
}

// Byte `pos` (compile-time) of a little-endian array of 32-bit words.
template <int POS>
__host__ __device__ __forceinline__ uint32_t byte_at(const uint32_t* w) {
    return (w[POS >> 2] >> (8 * (POS & 3))) & 0xFFu;
}

// Deposit byte value v (< 256) at byte position pos (compile-time after unrolling).
__host__ __device__ __forceinline__ void put_byte(uint32_t* w, int pos, uint32_t v) {
    w[pos >> 2] |= v << (8 * (pos & 3));
}

// DQT of the four coefficient bytes of one 32-bit word by one multiply: byte i
// (< 2^W) moves from bit 8i to bit B*i.  Valid when the sixteen partial
// products fall on distinct, non-overlapping W-bit ranges below bit 32.
template <int B, int W>
__host__ __device__ constexpr bool pack4_by_multiply() {
    if (B > 8 || B <= 0 || W <= 0) return false;
    int pos[16] = {};
    int n = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) pos[n++] = 8 * i + (8 - B) * (3 - j);
    for (int x = 0; x < 16; ++x) {
        if (pos[x] + W > 32) return false;
        for (int y = x + 1; y < 16; ++y) {
            const int d = pos[x] > pos[y] ? pos[x] - pos[y] : pos[y] - pos[x];
            if (d < W) return false;
        }
    }
    return true;
}

template <int B, int W>
__host__ __device__ __forceinline__ uint32_t pack4_multiply(uint32_t x) {
    constexpr uint32_t mul = 1u | (1u << (8 - B)) | (1u << (2 * (8 - B))) | (1u << (3 * (8 - B)));
    constexpr uint32_t sh = 3 * (8 - B);
    constexpr uint32_t wm = (1u << W) - 1u;
    constexpr uint32_t m = wm | (wm << B) | (wm << (2 * B)) | (wm << (3 * B));
    return ((x * mul) >> sh) & m;
}

// Byte tiles through LDS for kernels whose per-thread records are long and
// not word-aligned (one polynomial of 48 coefficients, a product of 95): a
// workgroup of 256 threads moves the contiguous bytes of 256 records between
// global memory and LDS with coalesced dword accesses, and each thread then
// reads or writes its own record in LDS.  Tile byte j sits at L[skew + j]
// with skew = (address of global byte 0) mod 4, so that the dwords line up
// on both sides; L is 4-byte aligned and holds len + 4 bytes.  The head and
// tail that do not fill a dword move byte by byte, so nothing outside
// [src, src + len) is touched.  Every thread of the workgroup must call these
// (the caller places the barriers).
__device__ __forceinline__ uint32_t tile_skew(const void* p) { return (uint32_t)((uintptr_t)p & 3u); }

__device__ __forceinline__ void tile_in(const uint8_t* __restrict__ src, uint32_t len, uint8_t* L) {
    const uint32_t sk = tile_skew(src);
    const uint32_t head = min(len, (4u - sk) & 3u);
    const uint32_t nd = (len - head) >> 2;
    const uint32_t tail = head + 4 * nd;
    if (threadIdx.x < head) L[sk + threadIdx.x] = src[threadIdx.x];
    const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src + head);
    uint32_t* l32 = reinterpret_cast<uint32_t*>(L + sk + head);
    for (uint32_t i = threadIdx.x; i < nd; i += 256) l32[i] = __builtin_nontemporal_load(s32 + i);
    if (threadIdx.x < len - tail) L[sk + tail + threadIdx.x] = src[tail + threadIdx.x];
}

__device__ __forceinline__ void tile_out(const uint8_t* L, uint32_t len, uint8_t* __restrict__ dst) {
    const uint32_t sk = tile_skew(dst);
    const uint32_t head = min(len, (4u - sk) & 3u);
    const uint32_t nd = (len - head) >> 2;
    const uint32_t tail = head + 4 * nd;
    if (threadIdx.x < head) dst[threadIdx.x] = L[sk + threadIdx.x];
    uint32_t* d32 = reinterpret_cast<uint32_t*>(dst + head);
    const uint32_t* l32 = reinterpret_cast<const uint32_t*>(L + sk + head);
    for (uint32_t i = threadIdx.x; i < nd; i += 256) __builtin_nontemporal_store(l32[i], d32 + i);
    if (threadIdx.x < len - tail) dst[tail + threadIdx.x] = L[sk + tail + threadIdx.x];
}

// LDS bytes of one tile of n records of len bytes (with its skew slack), a
// multiple of 4.
__host__ __device__ inline uint32_t tile_bytes(uint32_t n, uint32_t len) { return (n * len + 4u + 3u) & ~3u; }

// A record of n bytes at LDS address x (any alignment) as ND dwords: ND + 1
// dwords are read from the one holding x (so the region needs that much slack
// past its last record), realigned with v_alignbyte, and the bytes at
// positions >= n are masked to 0.
template <int ND>
__device__ __forceinline__ void record_read(const uint8_t* x, uint32_t n, uint32_t (&d)[ND]) {
    const uint32_t sh = (uint32_t)((uintptr_t)x & 3u);
    const uint32_t* x32 = reinterpret_cast<const uint32_t*>(x - sh);
    uint32_t r[ND + 1];
#pragma unroll
    for (int k = 0; k <= ND; ++k) r[k] = x32[k];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        const int rem = (int)n - 4 * k;
        const uint32_t m = rem >= 4 ? ~0u : (rem <= 0 ? 0u : (1u << (8 * rem)) - 1u);
        d[k] = __builtin_amdgcn_alignbyte(r[k + 1], r[k], sh) & m;
    }
}

// LDS slack after each operand region of record_tiles: a record read runs up
// to 4 (ND + 1) + 3 bytes past its record's start, a result write up to
// 4 (NO + 1) + 3.
constexpr uint32_t kRecordSlack = 256;

// Dynamic LDS of record_tiles (bytes, a multiple of 4): the operand tiles of
// 256 products, na and nb bytes each, with their slack.  The result tile,
// 256 (na + nb - 1) bytes and the slack of its writes, overlays them.
__host__ __device__ inline uint32_t record_tiles_smem(uint32_t na, uint32_t nb) {
    return tile_bytes(256, na) + kRecordSlack + tile_bytes(256, nb) + kRecordSlack;
}

// Products of records, 256 per workgroup iteration: product t reads record t
// of A (na bytes) and of B (nb bytes) and writes record t of OUT
// (na + nb - 1 bytes), all three arrays contiguous.  The operand bytes of a
// tile are staged in LDS (tile_in); each thread reads its two records as
// dwords (record_read); reduce(xa, xb, ob) puts byte j of the result in byte j
// of the NO-dword stream ob (zero on entry), and must leave every byte at
// j >= na + nb - 1 zero; the region is cleared and each thread ORs its stream
// into place as aligned dwords (ds_or_b32: a dword a record shares with a
// neighbour receives only zero bytes from the other thread); the result tile
// leaves with coalesced stores (tile_out).  Every thread runs reduce, so its
// control flow stays uniform; threads past the last product write nothing.
template <int NDA, int NDB, int NO, typename Reduce>
__device__ __forceinline__ void record_tiles(uint32_t* smem, const uint8_t* __restrict__ A, uint32_t na,
                                             const uint8_t* __restrict__ B, uint32_t nb, uint8_t* __restrict__ OUT,
                                             uint64_t count, Reduce reduce) {
    static_assert(4 * (NDA + 1) + 3 <= (int)kRecordSlack && 4 * (NDB + 1) + 3 <= (int)kRecordSlack, "record slack");
    static_assert(4 * (NO + 1) + 3 <= 2 * (int)kRecordSlack, "result slack");
    const uint32_t nout = na + nb - 1;
    const uint32_t words = record_tiles_smem(na, nb) / 4;
    uint8_t* RA = reinterpret_cast<uint8_t*>(smem);
    uint8_t* RB = RA + tile_bytes(256, na) + kRecordSlack;
    uint8_t* RO = RA;
    const uint32_t u = threadIdx.x;
    for (uint64_t t0 = blockIdx.x * 256ull; t0 < count; t0 += (uint64_t)gridDim.x * 256) {
        const uint32_t n = (uint32_t)min<uint64_t>(256, count - t0);
        const uint8_t* ga = A + t0 * na;
        const uint8_t* gb = B + t0 * nb;
        uint8_t* go = OUT + t0 * nout;
        __syncthreads();   // the previous tile has left LDS
        tile_in(ga, n * na, RA);
        tile_in(gb, n * nb, RB);
        __syncthreads();
        uint32_t xa[NDA], xb[NDB];   // past n: stale bytes, never written out
        record_read<NDA>(RA + tile_skew(ga) + u * na, na, xa);
        record_read<NDB>(RB + tile_skew(gb) + u * nb, nb, xb);
        __syncthreads();   // every record is read: clear the region for the results
        for (uint32_t i = u; i < words; i += 256) smem[i] = 0;
        __syncthreads();
        uint32_t ob[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) ob[j] = 0;
        reduce(xa, xb, ob);
        if (u < n) {
            uint8_t* o = RO + tile_skew(go) + u * nout;
            const uint32_t sh = (uint32_t)((uintptr_t)o & 3u);
            uint32_t* o32 = reinterpret_cast<uint32_t*>(o - sh);
            uint32_t prev = 0;
#pragma unroll
            for (int j = 0; j <= NO; ++j) {
                const uint32_t cur = j < NO ? ob[j] : 0u;
                atomicOr(o32 + j, (uint32_t)((((uint64_t)cur << 32) | prev) >> (32 - 8 * sh)));
                prev = cur;
            }
        }
        __syncthreads();
        tile_out(RO, n * nout, go);
    }
}

}  // namespace dqt
