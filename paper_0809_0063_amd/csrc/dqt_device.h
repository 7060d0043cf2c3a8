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

// x mod p for x < 2^24 and p < 2^8, by the precomputed reciprocal (a REDC).
__device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t p, uint32_t pmagic) {
    uint32_t qt = __umulhi(x, pmagic);
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
__device__ __forceinline__ uint64_t fdiv_floor(uint64_t r, const struct RedqArgs& a) {
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
__device__ __forceinline__ uint64_t redq_compress_t(uint64_t r, const RedqArgs& a) {
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
__device__ __forceinline__ uint64_t redq_compress(uint64_t r, const RedqArgs& a) {
    return redq_compress_t<0, 0, 0, false>(r, a);
}

// Residue i of U (w bits at b*i).
template <int B = 0, int W = 0>
__device__ __forceinline__ uint32_t field(uint64_t U, uint32_t i, const RedqArgs& a) {
    const uint32_t b = B ? B : a.b, w = W ? W : a.w;
    return (uint32_t)(U >> (b * i)) & ((1u << w) - 1u);
}

// Correction of one residue without a table: (u_i - c*u_{i+1}) mod p.
__device__ __forceinline__ uint32_t correct_arith(uint32_t ui, uint32_t ui1, const RedqArgs& a) {
    return mod_small(ui + a.p * a.p - a.c * ui1, a.p, a.pmagic);
}

// Build the correction table in LDS: for window j = tabj, entry
// idx = u_0 | u_1 << w | ... | u_{j-1} << (j-1)w holds the j-1 corrected
// residues mu_t = (u_t - c*u_{t+1}) mod p as bytes (section 3.5: the first
// j-1 rows of Q_{j-1} times a window of j residues, binary indexing).
__device__ __forceinline__ void build_correction_table(uint16_t* tab, const RedqArgs& a) {
    if (a.tabj == 0) return;
    const uint32_t wm = (1u << a.w) - 1u;
    for (uint32_t idx = threadIdx.x; idx < a.tab_entries; idx += blockDim.x) {
        const uint32_t u0 = idx & wm, u1 = (idx >> a.w) & wm;
        uint32_t e = mod_small(u0 + a.p * a.p - a.c * u1, a.p, a.pmagic);
        if (a.tabj == 3) {
            const uint32_t u2 = (idx >> (2 * a.w)) & wm;
            e |= mod_small(u1 + a.p * a.p - a.c * u2, a.p, a.pmagic) << 8;
        }
        tab[idx] = (uint16_t)e;
    }
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
__device__ __forceinline__ uint32_t window_index(uint64_t U, uint32_t s, uint32_t j, const RedqArgs& a) {
    const uint32_t b = B ? B : a.b, w = W ? W : a.w;
    const uint32_t x = (uint32_t)(U >> (b * s));
    if (B && W && gather3_by_multiply<(B ? B : 1), (W ? W : 1)>()) {
        if (j == 3) {
            constexpr uint32_t wm = (1u << (W ? W : 1)) - 1u;
            constexpr uint32_t fm = wm | (wm << (B ? B : 1)) | (wm << (2 * (B ? B : 1)));
            constexpr uint32_t mul = 1u | (1u << ((B ? B : 1) - (W ? W : 1))) | (1u << (2 * ((B ? B : 1) - (W ? W : 1))));
            constexpr uint32_t sh = 2 * ((B ? B : 1) - (W ? W : 1));
            return ((x & fm) * mul >> sh) & ((1u << (3 * (W ? W : 1))) - 1u);
        }
    }
    const uint32_t wm = (1u << w) - 1u;
    uint32_t idx = x & wm;
    idx |= ((x >> b) & wm) << w;
    if (j == 3) idx |= ((x >> (2 * b)) & wm) << (2 * w);
    return idx;
}

// Full REDQ correction: writes mu_0 .. mu_{nres-1} (section 3.2, second part)
// through `put(i, mu_i)`.  With p | q the compressed residues are final.
template <int NR, int B = 0, int W = 0, class Put>
__device__ __forceinline__ void redq_correct(uint64_t U, const RedqArgs& a, const uint16_t* tab, Put put) {
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
__device__ __forceinline__ uint32_t byte_at(const uint32_t* w) {
    return (w[POS >> 2] >> (8 * (POS & 3))) & 0xFFu;
}

// Deposit byte value v (< 256) at byte position pos (compile-time after unrolling).
__device__ __forceinline__ void put_byte(uint32_t* w, int pos, uint32_t v) {
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
__device__ __forceinline__ uint32_t pack4_multiply(uint32_t x) {
    constexpr uint32_t mul = 1u | (1u << (8 - B)) | (1u << (2 * (8 - B))) | (1u << (3 * (8 - B)));
    constexpr uint32_t sh = 3 * (8 - B);
    constexpr uint32_t wm = (1u << W) - 1u;
    constexpr uint32_t m = wm | (wm << B) | (wm << (2 * B)) | (wm << (3 * B));
    return ((x * mul) >> sh) & m;
}

}  // namespace dqt
