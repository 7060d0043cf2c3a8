// Device-side building blocks of the packed-DQT / REDQ path (gfx950).
//
// Notation follows the paper: p the prime, q = 2^b the evaluation point,
// w = ceil(log2 p) the bit width of a residue, nres the number of q-adic
// digits of a packed word (REDQ_nres), c = q mod p the correction constant.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqt {

// Parameters of one REDQ_nres (section 3), precomputed on the host.
struct RedqArgs {
    double invp;       // smallest binary64 >= 1/p (AFDIV: o1 = up, o2 = nearest)
    uint64_t M;        // w-bit field masks at bit b*i, i < nres
    uint64_t G;        // guard 2^(2w) at bit b*i (field-parallel compression)
    uint32_t p, b, w, nres;
    uint32_t c;        // q mod p; 0 means p | q and no correction
    uint32_t fix;      // words may reach B = 2^53/(3+2^-52): one-sided AFDIV test
    uint32_t swar;     // b >= 2w+1: all u_i from one masked multiply-subtract
    uint32_t tabj;     // correction table window: 3 (2 outputs), 2 (1 output), 0 = arithmetic
    uint32_t pmagic;   // ceil(2^32 / p): x mod p = x - p*mulhi(x, pmagic) for x < 2^24
    uint32_t tab_entries;  // 2^(tabj*w), or 0
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
__device__ __forceinline__ uint64_t fdiv_floor(uint64_t r, double invp, uint32_t p, bool fix) {
#pragma clang fp contract(off)
    const double hi = (double)(uint32_t)(r >> 32);
    const double lo = (double)(uint32_t)r;
    const double rd = hi * 4294967296.0 + lo;  // exact: r < 2^53
    const double x = rd * invp;
    const double y = __builtin_floor(x);
    uint64_t s = (uint64_t)y;
    if (fix) {
        if (s * (uint64_t)p > r) s -= 1;
    }
    return s;
}

// REDQ compression (algorithm REDQ, first part, binary case of section 3.3):
// returns U with u_i = floor(r/q^i) - p*floor(s/q^i) in the w low bits of the
// field at bit b*i, zeros elsewhere.  Since u_i < p <= 2^w, only the w low bits
// of floor(r/q^i) and floor(s/q^i) matter; with 2w+1 bits per field all fields
// are computed by one masked multiply-subtract (each field value stays in
// [1, 2^(2w+1)), so no borrow or carry crosses a field).
__device__ __forceinline__ uint64_t redq_compress(uint64_t r, const RedqArgs& a) {
    const uint64_t s = fdiv_floor(r, a.invp, a.p, a.fix != 0);
    if (a.swar) {
        const uint64_t z = (r & a.M) + a.G - (uint64_t)a.p * (s & a.M);
        return z & a.M;
    }
    uint64_t U = 0;
    const uint32_t wm = (1u << a.w) - 1u;
    for (uint32_t i = 0; i < a.nres; ++i) {
        const uint32_t sh = a.b * i;
        const uint32_t ui = ((uint32_t)(r >> sh) - a.p * (uint32_t)(s >> sh)) & wm;
        U |= (uint64_t)ui << sh;
    }
    return U;
}

// Residue i of U (w bits at b*i).
__device__ __forceinline__ uint32_t field(uint64_t U, uint32_t i, const RedqArgs& a) {
    return (uint32_t)(U >> (a.b * i)) & ((1u << a.w) - 1u);
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

// Table index of the window of `j` residues starting at residue s.
__device__ __forceinline__ uint32_t window_index(uint64_t U, uint32_t s, uint32_t j, const RedqArgs& a) {
    const uint32_t x = (uint32_t)(U >> (a.b * s));
    const uint32_t wm = (1u << a.w) - 1u;
    uint32_t idx = x & wm;
    idx |= ((x >> a.b) & wm) << a.w;
    if (j == 3) idx |= ((x >> (2 * a.b)) & wm) << (2 * a.w);
    return idx;
}

// Full REDQ correction: writes mu_0 .. mu_{nres-1} (section 3.2, second part)
// through `put(i, mu_i)`.  With p | q the compressed residues are final.
template <int NR, class Put>
__device__ __forceinline__ void redq_correct(uint64_t U, const RedqArgs& a, const uint16_t* tab, Put put) {
    if (a.c == 0) {
#pragma unroll
        for (int i = 0; i < NR; ++i) put(i, field(U, i, a));
        return;
    }
    put(NR - 1, field(U, NR - 1, a));
    if (NR == 1) return;
    if (a.tabj == 3 && NR >= 3) {
        // windows of 3 residues overlapping by one; the last is shifted down to end at u_{NR-1}
#pragma unroll
        for (int s0 = 0; s0 < NR - 1; s0 += 2) {
            const int s = (s0 + 3 > NR) ? NR - 3 : s0;
            const uint32_t e = tab[window_index(U, s, 3, a)];
            put(s, e & 0xFF);
            put(s + 1, e >> 8);
        }
    } else if (a.tabj >= 2) {
#pragma unroll
        for (int s = 0; s < NR - 1; ++s) put(s, tab[window_index(U, s, 2, a)] & 0xFF);
    } else {
#pragma unroll
        for (int s = 0; s < NR - 1; ++s) put(s, correct_arith(field(U, s, a), field(U, s + 1, a), a));
    }
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

}  // namespace dqt
