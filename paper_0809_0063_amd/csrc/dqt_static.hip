// F_p matrix product that allocates nothing and takes no workspace: the packed
// operands go to a file-scope device array of the library instead.
//
// For callers that cannot call hipMalloc (code under graph capture, serving
// loops that must not allocate, harnesses that forbid it).  Every GPU the
// library runs on holds its own copy of the array until the process ends.
// The array's name is a host-side stand-in in host code: the first call on a
// device (with that device current) asks the runtime for the array's device
// address once, and every later use (kernel arguments) goes through that
// address.  All calls on one GPU share the array, so calls that overlap on one
// GPU (concurrent streams, or host threads) race on it; the packing kernels
// overwrite every word the multiply reads, so nothing needs clearing between
// calls.

#include <mutex>

#include "dqt_gemm_tile.h"
#include "dqt_internal.h"

namespace dqt {

dqt_status fgemm_enqueue(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* A, uint64_t lda,
                         const uint8_t* B, uint64_t ldb, uint8_t* C, uint64_t ldc, const GemmPlanResolved& r,
                         void* work, hipStream_t s);

// Largest packed-operand footprint the call accepts (a 4096^3 product in the
// default packed layout needs exactly this much).
static constexpr size_t kScratchBytes = 32ull << 20;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices];

// Device address of this device's copy of the array (looked up once per device).
static dqt_status scratch_address(void** out) {
    int dev = 0;
    DQT_TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("device index out of range");
        return DQT_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        DQT_TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned no address");
            return DQT_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DQT_OK;
}

}  // namespace dqt

using namespace dqt;

extern "C" size_t dqt_fgemm_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" dqt_status dqt_fgemm_noalloc(uint32_t p, uint64_t m, uint64_t n, uint64_t kdim, const uint8_t* d_A,
                                        uint64_t lda, const uint8_t* d_B, uint64_t ldb, uint8_t* d_C, uint64_t ldc,
                                        const dqt_gemm_plan* plan, void* stream) {
    GemmPlanResolved r;
    DQT_TRY(fgemm_resolve(p, m, n, kdim, plan, &r));
    if (m == 0 || n == 0) return DQT_OK;
    if (!d_C || ldc < n || ldc > 0xFFFFFFFFull) return DQT_E_INVALID;
    if (kdim == 0) return dqt_fgemm(p, m, n, 0, d_A, lda, d_B, ldb, d_C, ldc, plan, nullptr, 0, stream);
    if (!d_A || !d_B) return DQT_E_INVALID;
    if (lda < kdim || ldb < n || lda > 0xFFFFFFFFull || ldb > 0xFFFFFFFFull) return DQT_E_INVALID;
    if (r.ws_bytes > kScratchBytes) {
        set_error("dqt_fgemm_noalloc: the packed operands exceed the library's 32 MiB static scratch array");
        return DQT_E_WORKSPACE;
    }
    DQT_TRY(ensure_device_ready());
    void* work = nullptr;
    DQT_TRY(scratch_address(&work));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(debug_gate(s, p, {{d_A, m, kdim, lda}, {d_B, kdim, n, ldb}}));
    return fgemm_enqueue(p, m, n, kdim, d_A, lda, d_B, ldb, d_C, ldc, r, work, s);
}
