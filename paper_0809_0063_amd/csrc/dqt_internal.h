// Host-side internals shared by the libdqt translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>

#include "../../include/dqt.h"
#include "dqt_device.h"

namespace dqt {

// Record a message for dqt_last_error() (thread-local).
void set_error(const char* msg);
// Map a HIP error to DQT_E_DEVICE (recording its text), hipSuccess to DQT_OK.
dqt_status hip_status(hipError_t e, const char* what);
// One-time per-device set-up and self-check (rounding mode of binary64 is
// round-to-nearest, as algorithm AFDIV's choice of invp assumes).
dqt_status ensure_device_ready();
// Compute units of the current device (cached per device).
int device_cus();
// REDQ_nres parameters for (p, b = log2 q, nres) on words below 2^word_bits.
// DQT_E_BOUND if nres*b > 53 or word_bits > 53.
dqt_status make_redq_args(uint32_t p, uint32_t b, uint32_t nres, uint32_t word_bits, RedqArgs* out);
// ceil(log2 p) for p >= 2.
uint32_t residue_bits(uint32_t p);
// Grid size for a streaming kernel over `items` work items of `per_block` each.
unsigned stream_grid(uint64_t items, unsigned per_block, unsigned waves_per_cu = 8);

// Debug mode (dqt_debug.hip).  A uint8 operand of rows x cols entries with
// leading dimension ld, and a buffer of packed words: nfields fields of b
// bits each (checked: every field < p, nothing above the top field), or,
// with nfields == 0, words that must be below 2^b.
struct DebugU8 {
    const uint8_t* x;
    uint64_t rows, cols, ld;
};
struct DebugWords {
    const uint64_t* w;
    uint64_t count;
    uint32_t b, nfields;
};
bool debug_on();
// With debug mode on: checks the operands on stream s, waits for it and
// returns DQT_E_INPUT if one fails (the status word is read and cleared).
// DQT_OK at once with debug mode off.
dqt_status debug_gate(hipStream_t s, uint32_t p, std::initializer_list<DebugU8> u8s,
                      std::initializer_list<DebugWords> words = {});

// GF(p^k) set-up shared by the GF kernels: X^(k-1+j) mod P for j = 0..k-1,
// k coefficient bytes each (the reductions the two FGDP tables apply).
struct GfArgs {
    uint64_t xpow[7];
    uint32_t k;
};
// Checks the monic modulus (k+1 coefficients below p, leading 1) and fills ga.
dqt_status gf_setup_args(uint32_t k, uint32_t p, const uint8_t* modulus, GfArgs* ga);

}  // namespace dqt

#define DQT_TRY(expr)                         \
    do {                                      \
        dqt_status s_ = (expr);               \
        if (s_ != DQT_OK) return s_;          \
    } while (0)

#define DQT_LAUNCH_CHECK(what) DQT_TRY(::dqt::hip_status(hipGetLastError(), what))
