// libdqt core: parameter checks, REDQ set-up, and the one-word kernels
// (DQT pack, packed product, REDQ unpack, fused polynomial and GF(p^k)
// products) plus their plain per-entry comparators.
//
// Paper: Dumas, Fousse, Salvy, "Simultaneous Modular Reduction and Kronecker
// Substitution for Small Finite Fields", sections 2-6.

#include <math.h>
#include <string.h>

#include <atomic>

#include <mutex>
#include <string>

#include "dqt_internal.h"

namespace dqt {

// ---------------------------------------------------------------------------
// Errors and device set-up
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

void set_error(const char* msg) { g_last_error = msg ? msg : ""; }

dqt_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return DQT_OK;
    std::string m = what;
    m += ": ";
    m += hipGetErrorString(e);
    set_error(m.c_str());
    return DQT_E_DEVICE;
}

uint32_t residue_bits(uint32_t p) {
    uint32_t w = 0;
    while ((1u << w) < p) ++w;
    return w;
}

static constexpr int kMaxDevices = 64;
static std::mutex g_dev_mu;
static int g_dev_state[kMaxDevices];  // 0 unknown, 1 ready, -1 failed
static int g_dev_cus[kMaxDevices];

// Reads the binary64 rounding field of the MODE register (bits 3:2; 0 = round
// to nearest even) and computes one FDIV that is wrong in any other mode.
// The result lands in a file-scope device array (one per device), read back
// with hipMemcpyFromSymbol, so the check allocates nothing.
__device__ uint32_t g_selfcheck_out[2];

__global__ void k_selfcheck(double invp, uint64_t r) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t mode = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 1);  // MODE[3:0]
        g_selfcheck_out[0] = (mode >> 2) & 3u;
        const double x = (double)r * invp;
        g_selfcheck_out[1] = (uint32_t)(uint64_t)__builtin_floor(x);
    }
}

dqt_status ensure_device_ready() {
    int dev = 0;
    DQT_TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index out of range");
        return DQT_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev_state[dev] == 1) return DQT_OK;
    if (g_dev_state[dev] == -1) {
        set_error("device failed the binary64 rounding-mode self-check");
        return DQT_E_UNSUPPORTED;
    }
    int cus = 0;
    DQT_TRY(hip_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attribute"));
    g_dev_cus[dev] = cus > 0 ? cus : 1;
    // 3*(2^30 + 1) times the nearest binary64 to 1/3 (just below 1/3): the
    // product rounded to nearest is 2^30 + 1, rounded down it is below.
    const double invp = 1.0 / 3.0;
    const uint64_t r = 3ull * ((1ull << 30) + 1);
    hipLaunchKernelGGL(k_selfcheck, dim3(1), dim3(64), 0, 0, invp, r);
    uint32_t h[2] = {99, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(0);
    if (e == hipSuccess) e = hipMemcpyFromSymbol(h, HIP_SYMBOL(g_selfcheck_out), sizeof(h), 0, hipMemcpyDeviceToHost);
    DQT_TRY(hip_status(e, "selfcheck"));
    const uint32_t want = (uint32_t)(uint64_t)floor((double)r * invp);
    if (h[0] != 0 || h[1] != want) {
        g_dev_state[dev] = -1;
        set_error("binary64 rounding mode is not round-to-nearest on this device");
        return DQT_E_UNSUPPORTED;
    }
    g_dev_state[dev] = 1;
    return DQT_OK;
}

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    return g_dev_cus[dev] > 0 ? g_dev_cus[dev] : 256;
}

unsigned stream_grid(uint64_t items, unsigned per_block, unsigned waves_per_cu) {
    uint64_t blocks = (items + per_block - 1) / per_block;
    uint64_t cap = (uint64_t)device_cus() * waves_per_cu;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

// Smallest binary64 >= 1/p (1/p rounded up, o1 of case 2 in table tab:fdiv).
static double inverse_rounded_up(uint32_t p) {
    double v = 1.0 / (double)p;  // nearest
    int e = 0;
    const double f = frexp(v, &e);  // v = f * 2^e, f in [0.5, 1)
    const uint64_t m = (uint64_t)ldexp(f, 53);
    // v >= 1/p  <=>  m * p * 2^(e-53) >= 1  <=>  m * p >= 2^(53-e)
    const unsigned __int128 lhs = (unsigned __int128)m * p;
    const unsigned __int128 rhs = (unsigned __int128)1 << (53 - e);
    if (lhs < rhs) v = nextafter(v, 2.0);
    return v;
}

// Correction-table window chosen by dqt_set_table_window (0 = automatic).
static std::atomic<uint32_t> g_table_window{0};

dqt_status make_redq_args(uint32_t p, uint32_t b, uint32_t nres, uint32_t word_bits, RedqArgs* out) {
    if (p < 2 || p > 255 || b < 1 || b > 32 || nres < 1 || nres > 53 || !out) return DQT_E_INVALID;
    if ((uint64_t)nres * b > 53 || word_bits > 53) return DQT_E_BOUND;
    RedqArgs a;
    memset(&a, 0, sizeof(a));
    a.p = p;
    a.b = b;
    a.nres = nres;
    a.w = residue_bits(p);
    if (a.w == 0) a.w = 1;
    a.invp = inverse_rounded_up(p);
    a.invp52 = ldexp(a.invp, 52);
    a.small = (word_bits <= 51) ? 1u : 0u;
    a.c = (uint32_t)(((b >= 32) ? 0 : ((1ull << b) % p)) % p);
    if (b >= 32) a.c = (uint32_t)((1ull << 32) % p);
    // Words are < 2^word_bits.  AFDIV's single test is needed only if they can
    // reach B = 2^53/(3+2^-52), i.e. from 52 bits on.
    a.fix = (word_bits >= 52) ? 1u : 0u;
    a.swar = (b >= 2 * a.w + 1) ? 1u : 0u;
    for (uint32_t i = 0; i < nres; ++i) {
        a.M |= (uint64_t)((1u << a.w) - 1u) << (b * i);
        if (a.swar) a.G |= (uint64_t)1 << (b * i + 2 * a.w);
    }
    if (a.swar && b * (nres - 1) + 2 * a.w >= 64) return DQT_E_BOUND;
    a.pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    // Correction table window (section 3.5): by default the largest of 3, 2
    // whose table fits 4096 entries; dqt_set_table_window caps it (1: no
    // table, the correction computed arithmetically).
    const uint32_t cap = g_table_window.load(std::memory_order_relaxed);
    if (a.c == 0 || nres == 1 || cap == 1) {
        a.tabj = 0;
    } else if (3 * a.w <= 12 && nres >= 3 && cap != 2) {
        a.tabj = 3;
    } else if (2 * a.w <= 12) {
        a.tabj = 2;
    } else {
        a.tabj = 0;
    }
    a.tab_entries = a.tabj ? (1u << (a.tabj * a.w)) : 0u;
    *out = a;
    return DQT_OK;
}

}  // namespace dqt

using namespace dqt;

// ---------------------------------------------------------------------------
// C ABI: status, parameters
// ---------------------------------------------------------------------------

extern "C" const char* dqt_status_str(dqt_status s) {
    switch (s) {
        case DQT_OK: return "ok";
        case DQT_E_INVALID: return "invalid argument";
        case DQT_E_BOUND: return "parameters violate the a priori bounds";
        case DQT_E_UNSUPPORTED: return "unsupported parameters";
        case DQT_E_DEVICE: return "HIP runtime error";
        case DQT_E_WORKSPACE: return "workspace too small";
        case DQT_E_INPUT: return "input check failed (an entry not a residue in [0, p), or a packed word out of its bounds)";
    }
    return "unknown status";
}

extern "C" const char* dqt_last_error(void) { return g_last_error.c_str(); }

namespace dqt {
__global__ __launch_bounds__(64) void k_flag_clear(uint32_t* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// Any entry >= p sets the flag (every writer stores the same value).
__global__ __launch_bounds__(256) void k_check_input(const uint8_t* __restrict__ x, uint64_t count, uint32_t p,
                                                     uint32_t* flag) {
    bool bad = false;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256)
        bad |= x[t] >= p;
    if (bad) *flag = 1;
}
}  // namespace dqt

extern "C" dqt_status dqt_check_input_u8(const uint8_t* d_x, uint64_t count, uint32_t p, uint32_t* d_flag,
                                         void* stream) {
    if (p < 2 || p > 255 || !d_flag) return DQT_E_INVALID;
    if (count == 0) return DQT_OK;
    if (!d_x) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, s, d_flag);
    DQT_LAUNCH_CHECK("dqt_check_input_u8");
    hipLaunchKernelGGL(k_check_input, dim3(stream_grid(count, 256, 4)), dim3(256), 0, s, d_x, count, p, d_flag);
    DQT_LAUNCH_CHECK("dqt_check_input_u8");
    uint32_t h = 0;
    DQT_TRY(hip_status(hipMemcpyAsync(&h, d_flag, sizeof(h), hipMemcpyDeviceToHost, s), "check_input copy"));
    DQT_TRY(hip_status(hipStreamSynchronize(s), "check_input sync"));
    return h ? DQT_E_INPUT : DQT_OK;
}

extern "C" const char* dqt_version(void) { return "libdqt 0.2 gfx950"; }

extern "C" dqt_status dqt_set_table_window(uint32_t j) {
    if (j > 3) return DQT_E_INVALID;
    g_table_window.store(j, std::memory_order_relaxed);
    return DQT_OK;
}

extern "C" uint32_t dqt_get_table_window(void) { return g_table_window.load(std::memory_order_relaxed); }

extern "C" dqt_status dqt_qadic_check(const dqt_qadic* a) {
    if (!a) return DQT_E_INVALID;
    if (a->p < 2 || a->p > 255 || a->k_coeffs < 1 || a->nres < 1 || a->nres > 32 || a->log2q < 1 ||
        a->log2q > 32 || a->n_accum < 1 || a->word_bits > 64)
        return DQT_E_INVALID;
    // beta: REDQ's one division is one binary64 floor, exact only on words below 2^53
    const uint32_t beta = a->word_bits ? a->word_bits : 53;
    if (beta > 53) return DQT_E_UNSUPPORTED;
    // eq:bounds, first part: q > n k (p-1)^2 (no digit of a sum of n products reaches q)
    const unsigned __int128 need =
        (unsigned __int128)a->n_accum * a->k_coeffs * (uint64_t)(a->p - 1) * (uint64_t)(a->p - 1);
    if (!((unsigned __int128)1 << a->log2q > need)) return DQT_E_BOUND;
    // eq:bounds, second part: the nres digits fit the beta-bit word
    if ((uint64_t)a->nres * a->log2q > beta) return DQT_E_BOUND;
    return DQT_OK;
}

extern "C" dqt_status dqt_qadic_choose(uint32_t p, uint32_t k_coeffs, uint64_t n_accum, uint32_t word_bits,
                                       dqt_qadic* out) {
    if (!out || p < 2 || p > 255 || k_coeffs < 1 || k_coeffs > 16 || n_accum < 1 || word_bits > 64)
        return DQT_E_INVALID;
    dqt_qadic a;
    memset(&a, 0, sizeof(a));
    a.p = p;
    a.k_coeffs = k_coeffs;
    a.nres = 2 * k_coeffs - 1;
    a.n_accum = n_accum;
    a.word_bits = word_bits;
    const uint32_t beta = word_bits ? word_bits : 53;
    if (beta > 53) return DQT_E_UNSUPPORTED;
    for (uint32_t b = 1; b <= 32; ++b) {
        a.log2q = b;
        if (dqt_qadic_check(&a) == DQT_OK) {
            *out = a;
            return DQT_OK;
        }
        if ((uint64_t)a.nres * b > beta) break;
    }
    return DQT_E_BOUND;
}

// ---------------------------------------------------------------------------
// DQT pack, packed product, REDQ unpack (one word per thread)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_pack(const uint8_t* __restrict__ c, uint64_t count, uint32_t k, uint32_t b,
                                              int reverse, uint64_t* __restrict__ words) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        uint64_t v = 0;
        const uint8_t* x = c + t * k;
        for (uint32_t i = 0; i < k; ++i) {
            const uint32_t e = reverse ? (k - 1 - i) : i;
            v |= (uint64_t)x[i] << (b * e);
        }
        words[t] = v;
    }
}

__global__ __launch_bounds__(256) void k_words_mul(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                   uint64_t count, uint64_t* __restrict__ r) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) r[t] = a[t] * b[t];
}

// REDQ of arbitrary words with a runtime number of residues.
__global__ __launch_bounds__(256) void k_redq_unpack(const uint64_t* __restrict__ r, uint64_t count, RedqArgs ra,
                                                     uint8_t* __restrict__ out) {
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    __syncthreads();
    const uint32_t nr = ra.nres;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        const uint64_t U = redq_compress(r[t], ra);
        uint8_t* o = out + t * nr;
        o[nr - 1] = (uint8_t)field(U, nr - 1, ra);
        if (ra.c == 0) {
            for (uint32_t i = 0; i + 1 < nr; ++i) o[i] = (uint8_t)field(U, i, ra);
        } else if (ra.tabj == 3 && nr >= 3) {
            for (uint32_t s0 = 0; s0 + 1 < nr; s0 += 2) {
                const uint32_t s = (s0 + 3 > nr) ? nr - 3 : s0;
                const uint32_t e = tab[window_index(U, s, 3, ra)];
                o[s] = (uint8_t)(e & 0xFF);
                o[s + 1] = (uint8_t)(e >> 8);
            }
        } else if (ra.tabj >= 2) {
            for (uint32_t s = 0; s + 1 < nr; ++s) o[s] = (uint8_t)(tab[window_index(U, s, 2, ra)] & 0xFF);
        } else {
            for (uint32_t s = 0; s + 1 < nr; ++s) o[s] = (uint8_t)correct_arith(field(U, s, ra), field(U, s + 1, ra), ra);
        }
    }
}

// ---------------------------------------------------------------------------
// GF(p^k): the two tables of algorithm FGDP (theorem thm:fgdp), built in LDS
// ---------------------------------------------------------------------------


// Entry il of T_L: (u_0..u_{K-1}) -> sum_{i<K-1} mu_i X^i (already reduced, degree < K-1).
// Entry ih of T_H: (u_{K-1}..u_{2K-2}) -> (sum_{i>=K-1} mu_i X^i) mod P.
template <int K>
__device__ void build_gf_tables(uint64_t* tl, uint64_t* th, const RedqArgs& ra, const GfArgs& ga) {
    const uint32_t wm = (1u << ra.w) - 1u;
    const uint32_t n = 1u << (K * ra.w);
    for (uint32_t idx = threadIdx.x; idx < n; idx += blockDim.x) {
        uint32_t u[K];
#pragma unroll
        for (int j = 0; j < K; ++j) u[j] = (idx >> (j * ra.w)) & wm;
        // T_L
        uint64_t lo = 0;
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
            const uint32_t mu = ra.c ? correct_arith(u[i], u[i + 1], ra) : mod_small(u[i], ra.p, ra.pmagic);
            lo |= (uint64_t)mu << (8 * i);
        }
        tl[idx] = lo;
        // T_H: mu_{K-1+j}, the top one uncorrected
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

// R = H + L coefficient-wise mod p on K byte lanes.
__device__ __forceinline__ uint64_t gf_add_bytes(uint64_t h, uint64_t l, uint32_t p, uint64_t ones) {
    const uint64_t s = h + l;                        // each byte <= 2p-2 < 256
    const uint64_t t = s + (uint64_t)(128 - p) * ones;
    const uint64_t ge = (t >> 7) & ones;             // byte >= p
    return s - (uint64_t)p * ge;
}

template <int K, int B = 0, int W = 0, bool SMALL = false>
__device__ __forceinline__ uint64_t gf_reduce_word(uint64_t r, const RedqArgs& ra, const uint64_t* tl, const uint64_t* th,
                                                   uint64_t ones) {
    const uint64_t U = redq_compress_t<(B ? 2 * K - 1 : 0), B, W, SMALL>(r, ra);
    const uint32_t b = B ? B : ra.b, w = W ? W : ra.w;
    const uint32_t wm = (1u << w) - 1u;
    const uint32_t xl = (uint32_t)U;
    const uint32_t xh = (uint32_t)(U >> (b * (K - 1)));
    uint32_t il = 0, ih = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        il |= ((xl >> (b * j)) & wm) << (w * j);
        ih |= ((xh >> (b * j)) & wm) << (w * j);
    }
    return gf_add_bytes(th[ih], tl[il], ra.p, ones);
}

template <int K>
__global__ __launch_bounds__(256) void k_redq_unpack_gf(const uint64_t* __restrict__ r, uint64_t count, RedqArgs ra,
                                                        GfArgs ga, uint8_t* __restrict__ out) {
    extern __shared__ uint64_t gf_smem[];
    const uint32_t n = 1u << (K * ra.w);
    uint64_t* tl = gf_smem;
    uint64_t* th = gf_smem + n;
    build_gf_tables<K>(tl, th, ra, ga);
    __syncthreads();
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        const uint64_t v = gf_reduce_word<K>(r[t], ra, tl, th, ones);
#pragma unroll
        for (int i = 0; i < K; ++i) out[t * K + i] = (uint8_t)(v >> (8 * i));
    }
}

// ---------------------------------------------------------------------------
// Fused kernels: four products per thread so that every load and store is a
// whole number of 32-bit words (4k input bytes, 4(2k-1) or 4k output bytes).
// ---------------------------------------------------------------------------

// Operand width class of the packed product.
enum { MUL24 = 0, MUL32 = 1, MUL64 = 2 };

template <int MODE>
__device__ __forceinline__ uint64_t packed_mul(uint64_t x, uint64_t y) {
    if (MODE == MUL24) return (uint64_t)((uint32_t)x & 0xFFFFFFu) * (uint64_t)((uint32_t)y & 0xFFFFFFu);
    if (MODE == MUL32) return (uint64_t)(uint32_t)x * (uint64_t)(uint32_t)y;
    return x * y;
}

// DQT of K coefficient bytes starting at compile-time byte position BASE.
template <int K, int BASE, int MODE, int B = 0, int W = 0>
__device__ __forceinline__ uint64_t pack_bytes(const uint32_t* w, uint32_t b_rt) {
    const uint32_t b = B ? B : b_rt;
    if (K == 4 && (BASE & 3) == 0 && B && W && pack4_by_multiply<(B ? B : 1), (W ? W : 1)>())
        return pack4_multiply<(B ? B : 1), (W ? W : 1)>(w[BASE >> 2]);
    if (MODE == MUL64) {
        uint64_t v = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) v |= (uint64_t)((w[(BASE + i) >> 2] >> (8 * ((BASE + i) & 3))) & 0xFFu) << (b * i);
        return v;
    }
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) v |= ((w[(BASE + i) >> 2] >> (8 * ((BASE + i) & 3))) & 0xFFu) << (b * i);
    return v;
}

template <int K, int MODE, int T, int B = 0, int W = 0, bool SMALL = false>
__device__ __forceinline__ void polymul_one(const uint32_t* a, const uint32_t* bw, uint32_t* o, const RedqArgs& ra,
                                            const uint16_t* tab) {
    constexpr int NR = 2 * K - 1;
    const uint64_t x = pack_bytes<K, T * K, MODE, B, W>(a, ra.b);
    const uint64_t y = pack_bytes<K, T * K, MODE, B, W>(bw, ra.b);
    const uint64_t r = packed_mul<MODE>(x, y);
    const uint64_t U = redq_compress_t<(B ? NR : 0), B, W, SMALL>(r, ra);
    redq_correct<NR, B, W>(U, ra, tab, [&](int i, uint32_t v) { put_byte(o, T * NR + i, v); });
}

// Scalar path for the last count % 4 products (byte loads and stores).
template <int K, int MODE>
__device__ void polymul_tail(const uint8_t* A, const uint8_t* B, uint8_t* OUT, uint64_t t, const RedqArgs& ra,
                             const uint16_t* tab) {
    constexpr int NR = 2 * K - 1;
    uint32_t a[(K + 3) / 4] = {0}, b[(K + 3) / 4] = {0}, o[(NR + 3) / 4] = {0};
#pragma unroll
    for (int i = 0; i < K; ++i) {
        put_byte(a, i, A[t * K + i]);
        put_byte(b, i, B[t * K + i]);
    }
    polymul_one<K, MODE, 0>(a, b, o, ra, tab);
#pragma unroll
    for (int i = 0; i < NR; ++i) OUT[t * NR + i] = (uint8_t)((o[i >> 2] >> (8 * (i & 3))) & 0xFF);
}

template <int K, int MODE, int QB = 0, int QW = 0, bool SMALL = false>
__global__ __launch_bounds__(256) void k_polymul_fused(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                       uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra) {
    constexpr int NR = 2 * K - 1;
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    __syncthreads();
    const uint64_t ngroups = count >> 2;
    const uint32_t* A32 = reinterpret_cast<const uint32_t*>(A);
    const uint32_t* B32 = reinterpret_cast<const uint32_t*>(B);
    uint32_t* O32 = reinterpret_cast<uint32_t*>(OUT);
    for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < ngroups; g += (uint64_t)gridDim.x * 256) {
        uint32_t a[K], b[K], o[NR];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            a[i] = __builtin_nontemporal_load(A32 + g * K + i);
            b[i] = __builtin_nontemporal_load(B32 + g * K + i);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) o[i] = 0;
        polymul_one<K, MODE, 0, QB, QW, SMALL>(a, b, o, ra, tab);
        polymul_one<K, MODE, 1, QB, QW, SMALL>(a, b, o, ra, tab);
        polymul_one<K, MODE, 2, QB, QW, SMALL>(a, b, o, ra, tab);
        polymul_one<K, MODE, 3, QB, QW, SMALL>(a, b, o, ra, tab);
#pragma unroll
        for (int i = 0; i < NR; ++i) __builtin_nontemporal_store(o[i], O32 + g * NR + i);
    }
    const uint64_t rem = count & 3;
    if (blockIdx.x == 0 && threadIdx.x < rem) polymul_tail<K, MODE>(A, B, OUT, ngroups * 4 + threadIdx.x, ra, tab);
}

template <int K, int MODE>
__global__ __launch_bounds__(256) void k_polymul_fused_bytes(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                             uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra) {
    __shared__ uint16_t tab[4096];
    build_correction_table(tab, ra);
    __syncthreads();
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256)
        polymul_tail<K, MODE>(A, B, OUT, t, ra, tab);
}

template <int K, int MODE, int T, int B = 0, int W = 0, bool SMALL = false>
__device__ __forceinline__ void gf_one(const uint32_t* a, const uint32_t* bw, uint32_t* o, const RedqArgs& ra,
                                       const uint64_t* tl, const uint64_t* th, uint64_t ones) {
    const uint64_t x = pack_bytes<K, T * K, MODE, B, W>(a, ra.b);
    const uint64_t y = pack_bytes<K, T * K, MODE, B, W>(bw, ra.b);
    const uint64_t v = gf_reduce_word<K, B, W, SMALL>(packed_mul<MODE>(x, y), ra, tl, th, ones);
#pragma unroll
    for (int i = 0; i < K; ++i) put_byte(o, T * K + i, (uint32_t)(v >> (8 * i)) & 0xFFu);
}

template <int K, int MODE, int QB = 0, int QW = 0, bool SMALL = false>
__global__ __launch_bounds__(256) void k_gf_mul_fused(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                      uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra, GfArgs ga) {
    extern __shared__ uint64_t gf_smem[];
    const uint32_t n = 1u << (K * ra.w);
    uint64_t* tl = gf_smem;
    uint64_t* th = gf_smem + n;
    build_gf_tables<K>(tl, th, ra, ga);
    __syncthreads();
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    const uint64_t ngroups = count >> 2;
    const uint32_t* A32 = reinterpret_cast<const uint32_t*>(A);
    const uint32_t* B32 = reinterpret_cast<const uint32_t*>(B);
    uint32_t* O32 = reinterpret_cast<uint32_t*>(OUT);
    for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < ngroups; g += (uint64_t)gridDim.x * 256) {
        uint32_t a[K], b[K], o[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            a[i] = __builtin_nontemporal_load(A32 + g * K + i);
            b[i] = __builtin_nontemporal_load(B32 + g * K + i);
            o[i] = 0;
        }
        gf_one<K, MODE, 0, QB, QW, SMALL>(a, b, o, ra, tl, th, ones);
        gf_one<K, MODE, 1, QB, QW, SMALL>(a, b, o, ra, tl, th, ones);
        gf_one<K, MODE, 2, QB, QW, SMALL>(a, b, o, ra, tl, th, ones);
        gf_one<K, MODE, 3, QB, QW, SMALL>(a, b, o, ra, tl, th, ones);
#pragma unroll
        for (int i = 0; i < K; ++i) __builtin_nontemporal_store(o[i], O32 + g * K + i);
    }
    const uint64_t rem = count & 3;
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const uint64_t t = ngroups * 4 + threadIdx.x;
        uint32_t a[(K + 3) / 4] = {0}, b[(K + 3) / 4] = {0}, o[(K + 3) / 4] = {0};
#pragma unroll
        for (int i = 0; i < K; ++i) {
            put_byte(a, i, A[t * K + i]);
            put_byte(b, i, B[t * K + i]);
        }
        gf_one<K, MODE, 0>(a, b, o, ra, tl, th, ones);
#pragma unroll
        for (int i = 0; i < K; ++i) OUT[t * K + i] = (uint8_t)((o[i >> 2] >> (8 * (i & 3))) & 0xFF);
    }
}

// One product per thread with byte loads (operands not 4-byte aligned).
template <int K>
__global__ __launch_bounds__(256) void k_gf_mul_fused_bytes(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                            uint8_t* __restrict__ OUT, uint64_t count, RedqArgs ra,
                                                            GfArgs ga) {
    extern __shared__ uint64_t gf_smem[];
    const uint32_t n = 1u << (K * ra.w);
    uint64_t* tl = gf_smem;
    uint64_t* th = gf_smem + n;
    build_gf_tables<K>(tl, th, ra, ga);
    __syncthreads();
    const uint64_t ones = 0x0101010101010101ull >> (8 * (8 - K));
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        uint64_t x = 0, y = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            x |= (uint64_t)A[t * K + i] << (ra.b * i);
            y |= (uint64_t)B[t * K + i] << (ra.b * i);
        }
        const uint64_t v = gf_reduce_word<K>(x * y, ra, tl, th, ones);
#pragma unroll
        for (int i = 0; i < K; ++i) OUT[t * K + i] = (uint8_t)(v >> (8 * i));
    }
}

// ---------------------------------------------------------------------------
// Plain per-entry comparators: one coefficient per multiply-add (int32
// accumulation, delayed), one reduction per output coefficient (REDC).
// ---------------------------------------------------------------------------

template <int K>
__device__ __forceinline__ void plain_poly_product(const uint8_t* x, const uint8_t* y, uint32_t* c) {
#pragma unroll
    for (int j = 0; j < 2 * K - 1; ++j) c[j] = 0;
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int l = 0; l < K; ++l) c[i + l] += (uint32_t)x[i] * (uint32_t)y[l];
}

template <int K>
__global__ __launch_bounds__(256) void k_polymul_plain(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                       uint8_t* __restrict__ OUT, uint64_t count, uint32_t p,
                                                       uint32_t pmagic) {
    constexpr int NR = 2 * K - 1;
    const uint64_t ngroups = count >> 2;
    const uint32_t* A32 = reinterpret_cast<const uint32_t*>(A);
    const uint32_t* B32 = reinterpret_cast<const uint32_t*>(B);
    uint32_t* O32 = reinterpret_cast<uint32_t*>(OUT);
    for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < ngroups; g += (uint64_t)gridDim.x * 256) {
        uint32_t a[K], b[K], o[NR];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            a[i] = __builtin_nontemporal_load(A32 + g * K + i);
            b[i] = __builtin_nontemporal_load(B32 + g * K + i);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) o[i] = 0;
        const uint8_t* ab = reinterpret_cast<const uint8_t*>(a);
        const uint8_t* bb = reinterpret_cast<const uint8_t*>(b);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t c[NR];
            plain_poly_product<K>(ab + t * K, bb + t * K, c);
#pragma unroll
            for (int j = 0; j < NR; ++j) put_byte(o, t * NR + j, mod_small(c[j], p, pmagic));
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) __builtin_nontemporal_store(o[i], O32 + g * NR + i);
    }
    const uint64_t rem = count & 3;
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const uint64_t t = ngroups * 4 + threadIdx.x;
        uint8_t x[K], y[K];
        uint32_t c[NR];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            x[i] = A[t * K + i];
            y[i] = B[t * K + i];
        }
        plain_poly_product<K>(x, y, c);
#pragma unroll
        for (int j = 0; j < NR; ++j) OUT[t * NR + j] = (uint8_t)mod_small(c[j], p, pmagic);
    }
}

// Plain product of longer polynomials (9 <= k <= 64 coefficients, padded to
// KMAX): the coefficients of both operands in registers, one v_mad_u32_u24
// per coefficient product (delayed: the sum stays below 64 (p-1)^2 < 2^32),
// one REDC per output coefficient; the records move through LDS in tiles of
// 256 products as in the packed FQT kernels.
template <int KMAX>
__global__ __launch_bounds__(256) void k_polymul_plain_tiles(const uint8_t* __restrict__ A, uint32_t ka,
                                                             const uint8_t* __restrict__ B, uint32_t kb,
                                                             uint8_t* __restrict__ OUT, uint64_t count, uint32_t p,
                                                             uint32_t pmagic) {
    constexpr int ND = KMAX / 4;
    constexpr int NO = (2 * KMAX - 1 + 3) / 4;
    extern __shared__ uint32_t plain_smem[];
    record_tiles<ND, ND, NO>(plain_smem, A, ka, B, kb, OUT, count,
                             [&](const uint32_t (&xa)[ND], const uint32_t (&xb)[ND], uint32_t (&ob)[NO]) {
        uint32_t x[KMAX], y[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            x[i] = (xa[i >> 2] >> (8 * (i & 3))) & 0xFFu;
            y[i] = (xb[i >> 2] >> (8 * (i & 3))) & 0xFFu;
        }
#pragma unroll
        for (int j = 0; j < 2 * KMAX - 1; ++j) {
            uint32_t c = 0;
#pragma unroll
            for (int i = (j >= KMAX ? j - KMAX + 1 : 0); i <= (j < KMAX ? j : KMAX - 1); ++i) c += x[i] * y[j - i];
            ob[j >> 2] |= mod_small(c, p, pmagic) << (8 * (j & 3));
        }
    });
}

// Plain GF(p^k) product of one pair: schoolbook with delayed sums, then long
// division by the monic modulus from the top down in which only the leading
// coefficient of each step is reduced (REDC) and the others take
// lead (p - m_i) unreduced, then one REDC for each of the k remaining
// coefficients: 2k - 1 reductions in all.  Every intermediate stays below
// (2k - 1) (p-1)^2 < 2^24, the range of the REDC.
template <int K>
__device__ __forceinline__ void gf_plain_one(const uint8_t* x, const uint8_t* y, const uint32_t (&negm)[K], uint32_t p,
                                             uint32_t pmagic, uint32_t (&r)[K]) {
    uint32_t c[2 * K - 1];
    plain_poly_product<K>(x, y, c);
#pragma unroll
    for (int j = 2 * K - 2; j >= K; --j) {
        const uint32_t lead = mod_small(c[j], p, pmagic);
#pragma unroll
        for (int i = 0; i < K; ++i) c[j - K + i] += lead * negm[i];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] = mod_small(c[i], p, pmagic);
}

// Four products per thread with whole-dword loads and stores (4k input bytes
// per operand, 4k output bytes), the I/O of the packed GF kernel.
template <int K>
__global__ __launch_bounds__(256) void k_gf_mul_plain4(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                       uint8_t* __restrict__ OUT, uint64_t count, uint32_t p,
                                                       uint32_t pmagic, uint64_t modulus) {
    uint32_t negm[K];
#pragma unroll
    for (int i = 0; i < K; ++i) negm[i] = (p - (uint32_t)((modulus >> (8 * i)) & 0xFF)) % p;
    const uint64_t ngroups = count >> 2;
    const uint32_t* A32 = reinterpret_cast<const uint32_t*>(A);
    const uint32_t* B32 = reinterpret_cast<const uint32_t*>(B);
    uint32_t* O32 = reinterpret_cast<uint32_t*>(OUT);
    for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < ngroups; g += (uint64_t)gridDim.x * 256) {
        uint32_t a[K], b[K], o[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            a[i] = __builtin_nontemporal_load(A32 + g * K + i);
            b[i] = __builtin_nontemporal_load(B32 + g * K + i);
            o[i] = 0;
        }
        const uint8_t* ab = reinterpret_cast<const uint8_t*>(a);
        const uint8_t* bb = reinterpret_cast<const uint8_t*>(b);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t r[K];
            gf_plain_one<K>(ab + t * K, bb + t * K, negm, p, pmagic, r);
#pragma unroll
            for (int i = 0; i < K; ++i) put_byte(o, t * K + i, r[i]);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) __builtin_nontemporal_store(o[i], O32 + g * K + i);
    }
    const uint64_t rem = count & 3;
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const uint64_t t = ngroups * 4 + threadIdx.x;
        uint8_t x[K], y[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            x[i] = A[t * K + i];
            y[i] = B[t * K + i];
        }
        uint32_t r[K];
        gf_plain_one<K>(x, y, negm, p, pmagic, r);
#pragma unroll
        for (int i = 0; i < K; ++i) OUT[t * K + i] = (uint8_t)r[i];
    }
}

// One product per thread with byte loads and stores (operands not 4-byte aligned).
template <int K>
__global__ __launch_bounds__(256) void k_gf_mul_plain(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                      uint8_t* __restrict__ OUT, uint64_t count, uint32_t p,
                                                      uint32_t pmagic, uint64_t modulus) {
    uint32_t negm[K];
#pragma unroll
    for (int i = 0; i < K; ++i) negm[i] = (p - (uint32_t)((modulus >> (8 * i)) & 0xFF)) % p;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        uint8_t x[K], y[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            x[i] = A[t * K + i];
            y[i] = B[t * K + i];
        }
        uint32_t r[K];
        gf_plain_one<K>(x, y, negm, p, pmagic, r);
#pragma unroll
        for (int i = 0; i < K; ++i) OUT[t * K + i] = (uint8_t)r[i];
    }
}

// ---------------------------------------------------------------------------
// C ABI: launches
// ---------------------------------------------------------------------------

static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
static bool aligned4(const void* p) { return ((uintptr_t)p & 3) == 0; }

extern "C" dqt_status dqt_pack(const uint8_t* d_coeffs, uint64_t count, const dqt_qadic* a, int reverse,
                               uint64_t* d_words, void* stream) {
    if (!a) return DQT_E_INVALID;
    DQT_TRY(dqt_qadic_check(a));
    if ((uint64_t)a->k_coeffs * a->log2q > 64) return DQT_E_BOUND;
    if (count == 0) return DQT_OK;
    if (!d_coeffs || !d_words) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    DQT_TRY(debug_gate(S(stream), a->p, {{d_coeffs, count, a->k_coeffs, a->k_coeffs}}));
    hipLaunchKernelGGL(k_pack, dim3(stream_grid(count, 256)), dim3(256), 0, S(stream), d_coeffs, count, a->k_coeffs,
                       a->log2q, reverse, d_words);
    DQT_LAUNCH_CHECK("dqt_pack");
    return DQT_OK;
}

extern "C" dqt_status dqt_polymul(const uint64_t* d_a, const uint64_t* d_b, uint64_t count, const dqt_qadic* a,
                                  uint64_t* d_r, void* stream) {
    if (!a) return DQT_E_INVALID;
    DQT_TRY(dqt_qadic_check(a));
    if (a->nres != 2 * a->k_coeffs - 1) return DQT_E_INVALID;
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_r) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    DQT_TRY(debug_gate(S(stream), a->p, {},
                       {{d_a, count, a->log2q, a->k_coeffs}, {d_b, count, a->log2q, a->k_coeffs}}));
    hipLaunchKernelGGL(k_words_mul, dim3(stream_grid(count, 256)), dim3(256), 0, S(stream), d_a, d_b, count, d_r);
    DQT_LAUNCH_CHECK("dqt_polymul");
    return DQT_OK;
}

// X^i mod P for i = K-1 .. 2K-2 as K coefficient bytes each (host polynomial arithmetic).
dqt_status dqt::gf_setup_args(uint32_t k, uint32_t p, const uint8_t* modulus, GfArgs* ga) {
    if (!modulus || k < 2 || k > 6) return DQT_E_INVALID;
    if (modulus[k] != 1) return DQT_E_INVALID;
    for (uint32_t i = 0; i <= k; ++i)
        if (modulus[i] >= p) return DQT_E_INVALID;
    memset(ga, 0, sizeof(*ga));
    ga->k = k;
    uint32_t cur[8] = {0};  // X^(k-1)
    cur[k - 1] = 1;
    for (uint32_t j = 0; j < k; ++j) {
        uint64_t v = 0;
        for (uint32_t i = 0; i < k; ++i) v |= (uint64_t)cur[i] << (8 * i);
        ga->xpow[j] = v;
        // cur <- X * cur mod P
        const uint32_t top = cur[k - 1];
        for (int i = (int)k - 1; i >= 1; --i) cur[i] = cur[i - 1];
        cur[0] = 0;
        for (uint32_t i = 0; i < k; ++i) cur[i] = (cur[i] + p * p - top * modulus[i]) % p;
    }
    return DQT_OK;
}

static size_t gf_smem_bytes(uint32_t k, uint32_t w) { return 2ull * (1ull << (k * w)) * sizeof(uint64_t); }

template <int K>
static dqt_status launch_redq_gf(const uint64_t* d_r, uint64_t count, const RedqArgs& ra, const GfArgs& ga,
                                 uint8_t* d_out, hipStream_t s) {
    const size_t smem = gf_smem_bytes(K, ra.w);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_redq_unpack_gf<K>), dim3(stream_grid(count, 256, 4)), dim3(256), smem, s, d_r,
                       count, ra, ga, d_out);
    DQT_LAUNCH_CHECK("redq_unpack(gf)");
    return DQT_OK;
}

static constexpr size_t kMaxGfSmem = 64 * 1024;

extern "C" dqt_status redq_unpack(const uint64_t* d_r, uint64_t count, const dqt_qadic* a, const uint8_t* modulus,
                                  uint8_t* d_out, void* stream) {
    // REDQ needs only digits below q (the caller's guarantee) and a word that
    // is exact in binary64: nres * log2q <= 53; each residue field of w bits
    // must fit in its q-adic digit (log2q >= w).
    if (!a || a->p < 2 || a->p > 255 || a->log2q < 1 || a->log2q > 32 || a->nres < 1 || a->word_bits > 64)
        return DQT_E_INVALID;
    // beta: the words are below 2^beta (53 by default, the binary64 mantissa)
    const uint32_t beta = a->word_bits ? a->word_bits : 53;
    if (beta > 53) return DQT_E_UNSUPPORTED;
    if ((uint64_t)a->nres * a->log2q > 53) return DQT_E_BOUND;
    if (a->log2q < residue_bits(a->p)) return DQT_E_UNSUPPORTED;
    RedqArgs ra;
    DQT_TRY(make_redq_args(a->p, a->log2q, a->nres, beta, &ra));
    if (modulus) {
        if (a->nres != 2 * a->k_coeffs - 1) return DQT_E_INVALID;
        GfArgs ga;
        DQT_TRY(gf_setup_args(a->k_coeffs, a->p, modulus, &ga));
        if (gf_smem_bytes(a->k_coeffs, ra.w) > kMaxGfSmem) return DQT_E_UNSUPPORTED;
        if (a->log2q * (a->k_coeffs - 1) + ra.w > 32) return DQT_E_UNSUPPORTED;
        if (count == 0) return DQT_OK;
        if (!d_r || !d_out) return DQT_E_INVALID;
        DQT_TRY(ensure_device_ready());
        DQT_TRY(debug_gate(S(stream), a->p, {}, {{d_r, count, beta, 0}}));
        switch (a->k_coeffs) {
            case 2: return launch_redq_gf<2>(d_r, count, ra, ga, d_out, S(stream));
            case 3: return launch_redq_gf<3>(d_r, count, ra, ga, d_out, S(stream));
            case 4: return launch_redq_gf<4>(d_r, count, ra, ga, d_out, S(stream));
            case 5: return launch_redq_gf<5>(d_r, count, ra, ga, d_out, S(stream));
            case 6: return launch_redq_gf<6>(d_r, count, ra, ga, d_out, S(stream));
        }
        return DQT_E_UNSUPPORTED;
    }
    if (count == 0) return DQT_OK;
    if (!d_r || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    DQT_TRY(debug_gate(S(stream), a->p, {}, {{d_r, count, beta, 0}}));
    hipLaunchKernelGGL(k_redq_unpack, dim3(stream_grid(count, 256)), dim3(256), 0, S(stream), d_r, count, ra, d_out);
    DQT_LAUNCH_CHECK("redq_unpack");
    return DQT_OK;
}

// Width class of a packed operand of k coefficients at b bits each.
static int mul_mode(uint32_t k, uint32_t b, uint32_t w) {
    const uint32_t bits = b * (k - 1) + w;
    if (bits <= 24) return MUL24;
    if (bits <= 32) return MUL32;
    return MUL64;
}

template <int K>
static dqt_status launch_polymul_fused(const uint8_t* A, const uint8_t* B, uint64_t count, const RedqArgs& ra,
                                       uint8_t* out, hipStream_t s) {
    if (!aligned4(A) || !aligned4(B) || !aligned4(out)) {
        const unsigned g1 = stream_grid(count, 256);
        switch (mul_mode(K, ra.b, ra.w)) {
            case MUL24:
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused_bytes<K, MUL24>), dim3(g1), dim3(256), 0, s, A, B, out, count, ra);
                break;
            case MUL32:
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused_bytes<K, MUL32>), dim3(g1), dim3(256), 0, s, A, B, out, count, ra);
                break;
            default:
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused_bytes<K, MUL64>), dim3(g1), dim3(256), 0, s, A, B, out, count, ra);
                break;
        }
        DQT_LAUNCH_CHECK("dqt_polymul_u8");
        return DQT_OK;
    }
    const unsigned grid = stream_grid((count + 3) / 4, 256);
    // compile-time q and residue width for the degree-3 products over F_3 at q = 2^6
    if constexpr (K == 4) {
        if (ra.b == 6 && ra.w == 2 && ra.small && mul_mode(K, ra.b, ra.w) == MUL24) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused<K, MUL24, 6, 2, true>), dim3(grid), dim3(256), 0, s, A, B,
                               out, count, ra);
            DQT_LAUNCH_CHECK("dqt_polymul_u8");
            return DQT_OK;
        }
    }
    switch (mul_mode(K, ra.b, ra.w)) {
        case MUL24:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused<K, MUL24>), dim3(grid), dim3(256), 0, s, A, B, out, count, ra);
            break;
        case MUL32:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused<K, MUL32>), dim3(grid), dim3(256), 0, s, A, B, out, count, ra);
            break;
        default:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_fused<K, MUL64>), dim3(grid), dim3(256), 0, s, A, B, out, count, ra);
            break;
    }
    DQT_LAUNCH_CHECK("dqt_polymul_u8");
    return DQT_OK;
}

// q for a single product: the given one (checked against eq:bounds) or the smallest.
static dqt_status product_qadic(uint32_t p, uint32_t k, uint32_t log2q, dqt_qadic* q) {
    if (log2q == 0) return dqt_qadic_choose(p, k, 1, 0, q) == DQT_OK ? DQT_OK : DQT_E_UNSUPPORTED;
    memset(q, 0, sizeof(*q));
    q->p = p;
    q->k_coeffs = k;
    q->nres = 2 * k - 1;
    q->log2q = log2q;
    q->n_accum = 1;
    return dqt_qadic_check(q);
}

extern "C" dqt_status dqt_polymul_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t k, uint32_t p,
                                     uint32_t log2q, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || k < 1 || k > 32) return DQT_E_INVALID;
    dqt_qadic q;
    DQT_TRY(product_qadic(p, k, log2q, &q));
    RedqArgs ra;
    if (make_redq_args(p, q.log2q, q.nres, q.log2q * q.nres, &ra) != DQT_OK) return DQT_E_UNSUPPORTED;
    if (k > 9) return DQT_E_UNSUPPORTED;
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = S(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, k, k}, {d_b, count, k, k}}));
    switch (k) {
        case 1: return launch_polymul_fused<1>(d_a, d_b, count, ra, d_out, s);
        case 2: return launch_polymul_fused<2>(d_a, d_b, count, ra, d_out, s);
        case 3: return launch_polymul_fused<3>(d_a, d_b, count, ra, d_out, s);
        case 4: return launch_polymul_fused<4>(d_a, d_b, count, ra, d_out, s);
        case 5: return launch_polymul_fused<5>(d_a, d_b, count, ra, d_out, s);
        case 6: return launch_polymul_fused<6>(d_a, d_b, count, ra, d_out, s);
        case 7: return launch_polymul_fused<7>(d_a, d_b, count, ra, d_out, s);
        case 8: return launch_polymul_fused<8>(d_a, d_b, count, ra, d_out, s);
        case 9: return launch_polymul_fused<9>(d_a, d_b, count, ra, d_out, s);
    }
    return DQT_E_UNSUPPORTED;
}

template <int K>
static dqt_status launch_gf_fused(const uint8_t* A, const uint8_t* B, uint64_t count, const RedqArgs& ra,
                                  const GfArgs& ga, uint8_t* out, hipStream_t s) {
    const size_t smem = gf_smem_bytes(K, ra.w);
    if (!aligned4(A) || !aligned4(B) || !aligned4(out)) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_fused_bytes<K>), dim3(stream_grid(count, 256, 4)), dim3(256), smem, s,
                           A, B, out, count, ra, ga);
        DQT_LAUNCH_CHECK("dqt_gf_mul_u8");
        return DQT_OK;
    }
    const unsigned grid = stream_grid((count + 3) / 4, 256, 8);
    // compile-time q and residue width for GF(3^5) at q = 2^5 and GF(7^3) at q = 2^7
    if constexpr (K == 5) {
        if (ra.b == 5 && ra.w == 2 && ra.small && mul_mode(K, ra.b, ra.w) == MUL24) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_fused<K, MUL24, 5, 2, true>), dim3(grid), dim3(256), smem, s, A, B,
                               out, count, ra, ga);
            DQT_LAUNCH_CHECK("dqt_gf_mul_u8");
            return DQT_OK;
        }
    }
    if constexpr (K == 3) {
        if (ra.b == 7 && ra.w == 3 && ra.small && mul_mode(K, ra.b, ra.w) == MUL24) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_fused<K, MUL24, 7, 3, true>), dim3(grid), dim3(256), smem, s, A, B,
                               out, count, ra, ga);
            DQT_LAUNCH_CHECK("dqt_gf_mul_u8");
            return DQT_OK;
        }
    }
    if (mul_mode(K, ra.b, ra.w) == MUL24)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_fused<K, MUL24>), dim3(grid), dim3(256), smem, s, A, B, out, count, ra, ga);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_fused<K, MUL32>), dim3(grid), dim3(256), smem, s, A, B, out, count, ra, ga);
    DQT_LAUNCH_CHECK("dqt_gf_mul_u8");
    return DQT_OK;
}

extern "C" dqt_status dqt_gf_mul_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t k, uint32_t p,
                                    uint32_t log2q, const uint8_t* modulus, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || k < 2 || k > 6 || !modulus) return DQT_E_INVALID;
    GfArgs ga;
    DQT_TRY(gf_setup_args(k, p, modulus, &ga));
    dqt_qadic q;
    DQT_TRY(product_qadic(p, k, log2q, &q));
    RedqArgs ra;
    if (make_redq_args(p, q.log2q, q.nres, q.log2q * q.nres, &ra) != DQT_OK) return DQT_E_UNSUPPORTED;
    if (gf_smem_bytes(k, ra.w) > kMaxGfSmem) return DQT_E_UNSUPPORTED;
    if (q.log2q * (k - 1) + ra.w > 32) return DQT_E_UNSUPPORTED;
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    hipStream_t s = S(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, k, k}, {d_b, count, k, k}}));
    switch (k) {
        case 2: return launch_gf_fused<2>(d_a, d_b, count, ra, ga, d_out, s);
        case 3: return launch_gf_fused<3>(d_a, d_b, count, ra, ga, d_out, s);
        case 4: return launch_gf_fused<4>(d_a, d_b, count, ra, ga, d_out, s);
        case 5: return launch_gf_fused<5>(d_a, d_b, count, ra, ga, d_out, s);
        case 6: return launch_gf_fused<6>(d_a, d_b, count, ra, ga, d_out, s);
    }
    return DQT_E_UNSUPPORTED;
}

namespace dqt {
dqt_status plain_long_enqueue(const uint8_t* A, uint32_t na, const uint8_t* B, uint32_t nb, uint64_t count, uint32_t p,
                              uint8_t* out, hipStream_t s);
}

extern "C" dqt_status dqt_polymul_plain_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t k,
                                           uint32_t p, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || k < 1 || k > 4096) return DQT_E_INVALID;
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    const uint32_t pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    hipStream_t s = S(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, k, k}, {d_b, count, k, k}}));
    if (k > 64) return plain_long_enqueue(d_a, k, d_b, k, count, p, d_out, s);
    const unsigned g4 = stream_grid((count + 3) / 4, 256);
#define DQT_PLAIN_CASE(KK)                                                                                           \
    case KK:                                                                                                         \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_plain<KK>), dim3(g4), dim3(256), 0, s, d_a, d_b, d_out, count, p, \
                           pmagic);                                                                                  \
        break;
    switch (k) {
        DQT_PLAIN_CASE(1)
        DQT_PLAIN_CASE(2)
        DQT_PLAIN_CASE(3)
        DQT_PLAIN_CASE(4)
        DQT_PLAIN_CASE(5)
        DQT_PLAIN_CASE(6)
        DQT_PLAIN_CASE(7)
        DQT_PLAIN_CASE(8)
        default: {
            const dim3 grid(stream_grid(count, 256)), blk(256);
            const size_t sm = record_tiles_smem(k, k);
            if (k <= 16)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_plain_tiles<16>), grid, blk, sm, s, d_a, k, d_b, k, d_out,
                                   count, p, pmagic);
            else if (k <= 32)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_plain_tiles<32>), grid, blk, sm, s, d_a, k, d_b, k, d_out,
                                   count, p, pmagic);
            else if (k <= 48)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_plain_tiles<48>), grid, blk, sm, s, d_a, k, d_b, k, d_out,
                                   count, p, pmagic);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_polymul_plain_tiles<64>), grid, blk, sm, s, d_a, k, d_b, k, d_out,
                                   count, p, pmagic);
        }
    }
#undef DQT_PLAIN_CASE
    DQT_LAUNCH_CHECK("dqt_polymul_plain_u8");
    return DQT_OK;
}

extern "C" dqt_status dqt_gf_mul_plain_u8(const uint8_t* d_a, const uint8_t* d_b, uint64_t count, uint32_t k,
                                          uint32_t p, const uint8_t* modulus, uint8_t* d_out, void* stream) {
    if (p < 2 || p > 255 || k < 2 || k > 6 || !modulus) return DQT_E_INVALID;
    if (modulus[k] != 1) return DQT_E_INVALID;
    uint64_t mod = 0;
    for (uint32_t i = 0; i <= k; ++i) {
        if (modulus[i] >= p) return DQT_E_INVALID;
        mod |= (uint64_t)modulus[i] << (8 * i);
    }
    if (count == 0) return DQT_OK;
    if (!d_a || !d_b || !d_out) return DQT_E_INVALID;
    DQT_TRY(ensure_device_ready());
    const uint32_t pmagic = (uint32_t)(((1ull << 32) + p - 1) / p);
    hipStream_t s = S(stream);
    DQT_TRY(debug_gate(s, p, {{d_a, count, k, k}, {d_b, count, k, k}}));
    const bool al = aligned4(d_a) && aligned4(d_b) && aligned4(d_out);
    const unsigned g = stream_grid(count, 256);
    const unsigned g4 = stream_grid((count + 3) / 4, 256);
#define DQT_GF_PLAIN_CASE(KK)                                                                                      \
    case KK:                                                                                                       \
        if (al)                                                                                                    \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_plain4<KK>), dim3(g4), dim3(256), 0, s, d_a, d_b, d_out, \
                               count, p, pmagic, mod);                                                             \
        else                                                                                                       \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gf_mul_plain<KK>), dim3(g), dim3(256), 0, s, d_a, d_b, d_out,   \
                               count, p, pmagic, mod);                                                             \
        break;
    switch (k) {
        DQT_GF_PLAIN_CASE(2)
        DQT_GF_PLAIN_CASE(3)
        DQT_GF_PLAIN_CASE(4)
        DQT_GF_PLAIN_CASE(5)
        DQT_GF_PLAIN_CASE(6)
    }
#undef DQT_GF_PLAIN_CASE
    DQT_LAUNCH_CHECK("dqt_gf_mul_plain_u8");
    return DQT_OK;
}
