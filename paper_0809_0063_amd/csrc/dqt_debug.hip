// Debug mode: device-side checks of what the host cannot see, reported
// through a status word in caller-owned device memory.
//
// The packed paths rest on assumptions about the data itself:
//   * every entry is a residue in [0, p) (the a priori bounds eq:bounds and
//     eq:lower are stated for entries of at most p-1; a larger entry breaks
//     them silently);
//   * a packed operand word holds k fields below p and nothing above its top
//     field (so that, by eq:bounds, every digit of a product stays below q:
//     the REQUIRE of algorithm REDQ, section 3.2);
//   * a word handed to REDQ is below 2^53, so that its one division is one
//     binary64 multiply and floor (algorithm AFDIV, section 4).
// With debug mode on, every entry point checks the data it is given against
// these before it enqueues its own work, on its own stream, then waits for
// the stream, reads the status word and returns DQT_E_INPUT without
// launching anything else when a check failed.
//
// Status word bits: 1 = a uint8 entry >= p; 2 = a packed operand field >= p
// or bits above its top field; 4 = a REDQ input word >= 2^53.

#include <mutex>

#include "dqt_internal.h"

namespace dqt {

static std::mutex g_dbg_mu;
static uint32_t* g_dbg_word = nullptr;   // caller's device word; null = debug mode off
static int g_dbg_dev = -1;

bool debug_on() {
    std::lock_guard<std::mutex> lk(g_dbg_mu);
    return g_dbg_word != nullptr;
}

static uint32_t* debug_word(int* dev) {
    std::lock_guard<std::mutex> lk(g_dbg_mu);
    *dev = g_dbg_dev;
    return g_dbg_word;
}

// Rows x cols bytes with leading dimension ld: bit 1 for an entry >= p.
__global__ __launch_bounds__(256) void k_dbg_u8(const uint8_t* __restrict__ x, uint64_t rows, uint64_t cols,
                                                uint64_t ld, uint32_t p, uint32_t* status) {
    const uint64_t n = rows * cols;
    bool bad = false;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n; t += (uint64_t)gridDim.x * 256)
        bad |= x[(t / cols) * ld + t % cols] >= p;
    if (bad) atomicOr(status, 1u);
}

// Packed operand words of nf fields of b bits: bit 2 for a field >= p or a
// set bit above field nf-1.
__global__ __launch_bounds__(256) void k_dbg_fields(const uint64_t* __restrict__ w, uint64_t count, uint32_t b,
                                                    uint32_t nf, uint32_t p, uint32_t* status) {
    const uint64_t fm = (b >= 64) ? ~0ull : ((1ull << b) - 1);
    bool bad = false;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256) {
        uint64_t v = w[t];
        for (uint32_t i = 0; i < nf; ++i) {
            bad |= (v & fm) >= p;
            v = (b >= 64) ? 0 : (v >> b);
        }
        bad |= v != 0;
    }
    if (bad) atomicOr(status, 2u);
}

// REDQ input words: bit 4 for a word >= 2^bits.
__global__ __launch_bounds__(256) void k_dbg_below(const uint64_t* __restrict__ w, uint64_t count, uint32_t bits,
                                                   uint32_t* status) {
    bool bad = false;
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < count; t += (uint64_t)gridDim.x * 256)
        bad |= (w[t] >> bits) != 0;
    if (bad) atomicOr(status, 4u);
}

// Reads and clears the status word after `s` has drained.
static dqt_status read_status(uint32_t* word, hipStream_t s) {
    uint32_t h = 0;
    DQT_TRY(hip_status(hipStreamSynchronize(s), "dqt_sync_status"));
    DQT_TRY(hip_status(hipMemcpy(&h, word, sizeof(h), hipMemcpyDeviceToHost), "dqt_sync_status read"));
    if (h == 0) return DQT_OK;
    const uint32_t zero = 0;
    DQT_TRY(hip_status(hipMemcpy(word, &zero, sizeof(zero), hipMemcpyHostToDevice), "dqt_sync_status clear"));
    if (h & 1u) set_error("debug: an input entry is not a residue in [0, p)");
    else if (h & 2u) set_error("debug: a packed operand has a field >= p or bits above its top field");
    else set_error("debug: a REDQ input word is not below 2^53");
    return DQT_E_INPUT;
}

// Debug-mode gate: launch the checks, wait, report.  Returns DQT_OK at once
// when debug mode is off.
dqt_status debug_gate(hipStream_t s, uint32_t p, std::initializer_list<DebugU8> u8s,
                      std::initializer_list<DebugWords> words) {
    int dev = -1;
    uint32_t* word = debug_word(&dev);
    if (!word) return DQT_OK;
    int cur = 0;
    DQT_TRY(hip_status(hipGetDevice(&cur), "hipGetDevice"));
    if (cur != dev) {
        set_error("debug: the status word belongs to another device");
        return DQT_E_INVALID;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DQT_TRY(hip_status(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing"));
    if (cs != hipStreamCaptureStatusNone) {
        set_error("debug: the checks wait for the stream and cannot run under graph capture");
        return DQT_E_UNSUPPORTED;
    }
    for (const DebugU8& x : u8s) {
        if (!x.x || x.rows == 0 || x.cols == 0) continue;
        hipLaunchKernelGGL(k_dbg_u8, dim3(stream_grid(x.rows * x.cols, 256, 4)), dim3(256), 0, s, x.x, x.rows, x.cols,
                           x.ld, p, word);
        DQT_LAUNCH_CHECK("debug check");
    }
    for (const DebugWords& w : words) {
        if (!w.w || w.count == 0) continue;
        if (w.nfields)
            hipLaunchKernelGGL(k_dbg_fields, dim3(stream_grid(w.count, 256, 4)), dim3(256), 0, s, w.w, w.count, w.b,
                               w.nfields, p, word);
        else
            hipLaunchKernelGGL(k_dbg_below, dim3(stream_grid(w.count, 256, 4)), dim3(256), 0, s, w.w, w.count, w.b,
                               word);
        DQT_LAUNCH_CHECK("debug check");
    }
    return read_status(word, s);
}

}  // namespace dqt

using namespace dqt;

extern "C" dqt_status dqt_debug_enable(uint32_t* d_status) {
    int dev = -1;
    if (d_status) {
        DQT_TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
        const uint32_t zero = 0;
        DQT_TRY(hip_status(hipMemcpy(d_status, &zero, sizeof(zero), hipMemcpyHostToDevice), "dqt_debug_enable"));
    }
    std::lock_guard<std::mutex> lk(g_dbg_mu);
    g_dbg_word = d_status;
    g_dbg_dev = dev;
    return DQT_OK;
}

extern "C" dqt_status dqt_sync_status(void* stream) {
    int dev = -1;
    uint32_t* word = debug_word(&dev);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!word) {
        DQT_TRY(hip_status(hipStreamSynchronize(s), "dqt_sync_status"));
        return DQT_OK;
    }
    return read_status(word, s);
}
