// Batched F_p matrix products: one packing launch for all products, then
// persistent launches over all (product, tile) work items.
//
// The host builds, once per batch, a device-resident plan in the caller's
// workspace: a header, one descriptor per product (its resolved packing and
// delayed-reduction parameters and its packed-operand slices of the
// workspace), the prefix sums of packing blocks, and the work-item list,
// grouped by kernel variant (packed middle product with or without
// intermediate extraction and with either epilogue, dot4, dot8, plain) and,
// within a variant, sorted by decreasing cost (largest inner dimension first,
// so that the big tiles start early and the small ones fill the tail).
// Running the batch reads only the workspace, so it can be captured in a
// graph and replayed:
//   k_batch_pack:    grid-stride over every packing block of every product
//                    (binary search of the block prefix); resets the item
//                    counters;
//   k_batch_compute: one launch per variant present; its persistent
//                    workgroups take the next item of the variant's range
//                    from an atomic counter until the range is exhausted
//                    (every workgroup exits when its fetched index passes the
//                    end).  A launch per variant gives each its own register
//                    allocation (one kernel holding every variant would need
//                    the largest of them, and more, for all).

#include <string.h>

#include <algorithm>
#include <vector>

#include "dqt_gemm_tile.h"
#include "dqt_internal.h"

namespace dqt {

struct BatchDesc {
    GemmArgs g;        // multiply/epilogue parameters (CA/CB point into the workspace)
    PackArgs pk;       // packing parameters (A/B are the caller's operands)
    uint32_t pack_blocks;
    uint32_t pad[3];
};

// Kernel variants of the multiply: the packed middle product (with or without
// intermediate extraction, REDC or REDQ epilogue), dot4, dot8 and the plain
// per-entry product.  Each variant has its own persistent launch (its own
// register allocation) over its own contiguous range of the item list.
enum BatchVariant : uint32_t {
    BV_DOT2 = 0,        // packed, whole k in one interval, REDC
    BV_DOT2_EPIQ,       // packed, whole k in one interval, REDQ epilogue
    BV_DOT2_FLUSH,      // packed, intermediate extraction, REDC
    BV_DOT2_FLUSH_EPIQ, // packed, intermediate extraction, REDQ epilogue
    BV_DOT4,
    BV_DOT8,
    BV_MAD,
    BV_COUNT
};

struct BatchHeader {
    uint32_t n_desc;
    uint32_t n_items;
    uint32_t total_pack_blocks;
    uint32_t tm, s;                   // tile rows and k-split the plan was built for
    uint32_t pad0[3];
    uint32_t counter[BV_COUNT];       // next work item of each variant (reset before each compute launch)
    uint32_t pad1;
    uint32_t begin[BV_COUNT], end[BV_COUNT];   // item range of each variant
    uint32_t pad2[34];
};

static_assert(sizeof(BatchHeader) == 256, "batch header layout");

struct BatchLayout {
    size_t header, descs, prefix, items, packed, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <int TM, int S>
__global__ __launch_bounds__(256) void k_batch_pack(const BatchHeader* __restrict__ hdr, BatchHeader* hdr_w,
                                                    const BatchDesc* __restrict__ descs,
                                                    const uint32_t* __restrict__ prefix) {
    if (blockIdx.x == 0 && threadIdx.x < BV_COUNT) hdr_w->counter[threadIdx.x] = 0;
    const uint32_t nd = hdr->n_desc;
    const uint32_t total = hdr->total_pack_blocks;
    // each workgroup packs one contiguous range of blocks: one binary search
    // for the product owning its first block, then a forward walk
    const uint32_t chunk = (total + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = blockIdx.x * chunk, b1 = min(total, b0 + chunk);
    if (b0 >= b1) return;
    uint32_t lo = 0, hi = nd;   // prefix[lo] <= b0 < prefix[lo + 1]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b0) lo = mid;
        else hi = mid;
    }
    uint32_t d = __builtin_amdgcn_readfirstlane(lo);
    uint32_t dend = prefix[d + 1];
    PackArgs pk = descs[d].pk;
    for (uint32_t blk = b0; blk < b1; ++blk) {
        while (blk >= dend) {   // next product (empty ones are skipped)
            ++d;
            dend = prefix[d + 1];
            pk = descs[d].pk;
        }
        gemm_pack_block(pk, blk - prefix[d], threadIdx.x);
    }
}

template <int OP, int TM, int TN, int S, bool FLUSH, int EPI>
__global__ __launch_bounds__(64 * S) void k_batch_compute(BatchHeader* hdr, const BatchDesc* __restrict__ descs,
                                                          const uint2* __restrict__ items, uint32_t variant) {
    __shared__ __attribute__((aligned(16))) uint32_t red[TileSmem<TM, TN, S>::words];
    __shared__ uint32_t next;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t begin = hdr->begin[variant], end = hdr->end[variant];
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&hdr->counter[variant], 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(next) + begin;
        __syncthreads();
        if (it >= end) break;
        const uint2 item = items[it];
        const uint32_t d = __builtin_amdgcn_readfirstlane(item.x);
        const uint32_t tile = __builtin_amdgcn_readfirstlane(item.y);
        const GemmArgs g = descs[d].g;
        const uint32_t rb = tile % g.nrb, cb = tile / g.nrb;
        gemm_tile<OP, TM, TN, S, FLUSH, EPI>(g, rb, cb, wave, lane, red);
        __syncthreads();  // the LDS reduction buffer is reused by the next item
    }
}

static uint32_t batch_variant(const GemmPlanResolved& r) {
    switch (r.op) {
        case OP_DOT2:
            if (r.lw) return r.epi ? BV_DOT2_FLUSH_EPIQ : BV_DOT2_FLUSH;
            return r.epi ? BV_DOT2_EPIQ : BV_DOT2;
        case OP_DOT4: return BV_DOT4;
        case OP_DOT8: return BV_DOT8;
        default: return BV_MAD;
    }
}

static BatchLayout batch_layout(const dqt_gemm_desc* descs, uint32_t count, uint32_t tm, uint32_t tn, uint32_t s,
                                std::vector<GemmPlanResolved>* plans, uint64_t* n_items, dqt_status* st) {
    BatchLayout L;
    memset(&L, 0, sizeof(L));
    *st = DQT_OK;
    uint64_t packed = 0, items = 0;
    plans->resize(count);
    for (uint32_t i = 0; i < count; ++i) {
        const dqt_gemm_desc& d = descs[i];
        dqt_gemm_plan pl;
        memset(&pl, 0, sizeof(pl));
        pl.algo = d.algo;
        pl.interval = d.interval;
        pl.log2Q = d.log2Q;
        pl.epilogue = d.epilogue;
        pl.tile_rows = tm;
        pl.tile_cols = tn;
        pl.ksplit = s;
        if (d.algo == DQT_GEMM_MFMA || is_f64_algo(d.algo) || d.algo == DQT_GEMM_BY_SHAPE) {
            *st = DQT_E_UNSUPPORTED;
            return L;
        }
        dqt_status r = fgemm_resolve(d.p, d.m, d.n, d.kdim, &pl, &(*plans)[i]);
        if (r != DQT_OK) {
            *st = r;
            return L;
        }
        packed += align256((*plans)[i].ws_bytes);
        const GemmPlanResolved& R = (*plans)[i];
        items += (uint64_t)(R.m_pad / R.tm) * (R.n_pad / (64 * R.tn));
    }
    if (items > 0xFFFFFFFFull) {
        *st = DQT_E_INVALID;
        return L;
    }
    *n_items = items;
    L.header = 0;
    L.descs = align256(sizeof(BatchHeader));
    L.prefix = L.descs + align256((size_t)count * sizeof(BatchDesc));
    L.items = L.prefix + align256((size_t)(count + 1) * sizeof(uint32_t));
    L.packed = L.items + align256((size_t)items * sizeof(uint2));
    L.total = L.packed + packed;
    return L;
}

}  // namespace dqt

using namespace dqt;

struct dqt_batch {
    uint8_t* work;
    size_t descs_off, prefix_off, items_off;
    uint32_t tm, tn, s, count;
    uint64_t n_items, pack_blocks;
    uint32_t variant_items[BV_COUNT];
};

static dqt_status batch_opts(const dqt_batch_opts* o, uint32_t* tm, uint32_t* tn, uint32_t* s) {
    *tm = (o && o->tile_rows) ? o->tile_rows : 16;
    *tn = (o && o->tile_cols) ? o->tile_cols : 2;
    *s = (o && o->ksplit) ? o->ksplit : 4;
    if (*tm != 8 && *tm != 16) return DQT_E_INVALID;
    if (*tn != 2 && *tn != 4) return DQT_E_INVALID;
    if (*s != 2 && *s != 4 && *s != 8) return DQT_E_INVALID;
    if (*s == 8 && *tm == 16 && *tn == 4) return DQT_E_INVALID;   // 128 KiB of LDS partial sums
    return DQT_OK;
}

extern "C" size_t dqt_fgemm_batched_workspace_size(const dqt_gemm_desc* descs, uint32_t count,
                                                   const dqt_batch_opts* opts) {
    if (!descs || count == 0) return 0;
    uint32_t tm, tn, s;
    if (batch_opts(opts, &tm, &tn, &s) != DQT_OK) return 0;
    std::vector<GemmPlanResolved> plans;
    uint64_t items = 0;
    dqt_status st;
    const BatchLayout L = batch_layout(descs, count, tm, tn, s, &plans, &items, &st);
    return st == DQT_OK ? L.total : 0;
}

extern "C" dqt_status dqt_fgemm_batched_prepare(const dqt_gemm_desc* descs, uint32_t count,
                                                const dqt_batch_opts* opts, void* d_work, size_t work_bytes,
                                                void* stream, dqt_batch** out) {
    if (!descs || count == 0 || !out) return DQT_E_INVALID;
    *out = nullptr;
    uint32_t tm, tn, s;
    DQT_TRY(batch_opts(opts, &tm, &tn, &s));
    for (uint32_t i = 0; i < count; ++i) {
        const dqt_gemm_desc& d = descs[i];
        if (d.m == 0 || d.n == 0) return DQT_E_INVALID;
        if (!d.A || !d.B || !d.C || d.lda < d.kdim || d.ldb < d.n || d.ldc < d.n) return DQT_E_INVALID;
    }
    std::vector<GemmPlanResolved> plans;
    uint64_t n_items = 0;
    dqt_status st;
    const BatchLayout L = batch_layout(descs, count, tm, tn, s, &plans, &n_items, &st);
    DQT_TRY(st);
    if (!d_work || work_bytes < L.total) return DQT_E_WORKSPACE;
    DQT_TRY(ensure_device_ready());
    if (debug_on())
        for (uint32_t i = 0; i < count; ++i) {
            const dqt_gemm_desc& d = descs[i];
            DQT_TRY(debug_gate(reinterpret_cast<hipStream_t>(stream), d.p,
                               {{d.A, d.m, d.kdim, d.lda}, {d.B, d.kdim, d.n, d.ldb}}));
        }

    std::vector<uint8_t> host(L.packed, 0);
    BatchHeader* H = reinterpret_cast<BatchHeader*>(host.data() + L.header);
    BatchDesc* D = reinterpret_cast<BatchDesc*>(host.data() + L.descs);
    uint32_t* prefix = reinterpret_cast<uint32_t*>(host.data() + L.prefix);
    uint2* items = reinterpret_cast<uint2*>(host.data() + L.items);
    uint8_t* base = reinterpret_cast<uint8_t*>(d_work);
    size_t off = L.packed;
    uint64_t blocks = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const dqt_gemm_desc& d = descs[i];
        const GemmPlanResolved& R = plans[i];
        BatchDesc& bd = D[i];
        memset(&bd, 0, sizeof(bd));
        uint32_t* CA = reinterpret_cast<uint32_t*>(base + off);
        uint32_t* CB = CA + (size_t)R.KW * R.m_pad;
        off += align256(R.ws_bytes);
        GemmArgs& g = bd.g;
        g.CA = CA;
        g.CB = CB;
        g.C = d.C;
        g.m = d.m;
        g.n = d.n;
        g.ldc = d.ldc;
        g.m_pad = R.m_pad;
        g.n_pad = R.n_pad;
        g.KW = R.KW;
        uint32_t ks = (R.KW + R.s - 1) / R.s;
        g.kw_split = ks;
        g.lw = R.lw;
        g.nrb = R.m_pad / R.tm;
        g.ncb = R.n_pad / (64 * R.tn);
        g.b = R.b ? R.b : 1;
        g.p = d.p;
        g.pmagic = (uint32_t)(((1ull << 32) + d.p - 1) / d.p);
        g.op = R.op;
        DQT_TRY(fgemm_epilogue_args(d.p, d.kdim, R, &g));
        PackArgs& pk = bd.pk;
        pk.A = d.A;
        pk.B = d.B;
        pk.CA = CA;
        pk.CB = CB;
        pk.m = d.m;
        pk.n = d.n;
        pk.kdim = d.kdim;
        pk.lda = d.lda;
        pk.ldb = d.ldb;
        pk.m_pad = R.m_pad;
        pk.n_pad = R.n_pad;
        pk.KW = R.KW;
        pk.b = R.b;
        pk.op = R.op;
        pk.tm = R.tm;
        pk.cbw = 64 * R.tn;
        pk.al = ((((uintptr_t)d.A & 3) == 0 && (d.lda & 3) == 0) ? 1u : 0u) |
                ((((uintptr_t)d.B & 3) == 0 && (d.ldb & 3) == 0) ? 2u : 0u);
        pk.nba = pack_blocks_for((uint64_t)R.KW * R.m_pad, R.op);
        bd.pack_blocks = pk.nba + pack_blocks_for((uint64_t)R.KW * R.n_pad, R.op);
        prefix[i] = (uint32_t)blocks;
        blocks += bd.pack_blocks;
    }
    prefix[count] = (uint32_t)blocks;
    if (blocks > 0xFFFFFFFFull) return DQT_E_INVALID;
    // work items grouped by kernel variant; within a variant, most expensive products
    // first (cost of a tile ~ the instructions of its k loop: the inner dimension over
    // the entries per word)
    std::vector<uint32_t> order(count);
    for (uint32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        const uint32_t va = batch_variant(plans[a]), vb = batch_variant(plans[b]);
        if (va != vb) return va < vb;
        return (uint64_t)descs[a].kdim * (8 / entries_per_word(plans[a].op)) >
               (uint64_t)descs[b].kdim * (8 / entries_per_word(plans[b].op));
    });
    uint64_t it = 0;
    uint32_t vcount[BV_COUNT] = {0};
    for (uint32_t v = 0; v < BV_COUNT; ++v) H->begin[v] = H->end[v] = 0;
    for (uint32_t oi = 0; oi < count; ++oi) {
        const uint32_t i = order[oi];
        const uint32_t v = batch_variant(plans[i]);
        if (vcount[v] == 0) H->begin[v] = (uint32_t)it;
        const uint32_t tiles = D[i].g.nrb * D[i].g.ncb;
        for (uint32_t t = 0; t < tiles; ++t) items[it++] = make_uint2(i, t);
        vcount[v] += tiles;
        H->end[v] = (uint32_t)it;
    }
    H->n_desc = count;
    H->n_items = (uint32_t)n_items;
    for (uint32_t v = 0; v < BV_COUNT; ++v) H->counter[v] = 0;
    H->total_pack_blocks = (uint32_t)blocks;
    H->tm = tm;
    H->s = s;
    hipStream_t st_ = reinterpret_cast<hipStream_t>(stream);
    DQT_TRY(hip_status(hipMemcpyAsync(d_work, host.data(), L.packed, hipMemcpyHostToDevice, st_), "batch upload"));
    // the host copy is released on return: wait for the upload
    DQT_TRY(hip_status(hipStreamSynchronize(st_), "batch upload sync"));
    dqt_batch* b = new dqt_batch;
    b->work = base;
    b->descs_off = L.descs;
    b->prefix_off = L.prefix;
    b->items_off = L.items;
    b->tm = tm;
    b->tn = tn;
    b->s = s;
    b->count = count;
    b->n_items = n_items;
    b->pack_blocks = blocks;
    for (uint32_t v = 0; v < BV_COUNT; ++v) b->variant_items[v] = vcount[v];
    *out = b;
    return DQT_OK;
}



// Clears the work-item counter before a compute launch that follows no packing
// launch (a kernel rather than a memset, so that the launch can be captured).
__global__ void k_batch_reset(BatchHeader* hdr) {
    if (threadIdx.x < BV_COUNT) hdr->counter[threadIdx.x] = 0;
}

template <int TM, int TN, int S>
static dqt_status batch_launch(const dqt_batch* b, hipStream_t st, bool pack, bool compute) {
    BatchHeader* hdr = reinterpret_cast<BatchHeader*>(b->work);
    const BatchDesc* descs = reinterpret_cast<const BatchDesc*>(b->work + b->descs_off);
    const uint32_t* prefix = reinterpret_cast<const uint32_t*>(b->work + b->prefix_off);
    const uint2* items = reinterpret_cast<const uint2*>(b->work + b->items_off);
    const uint64_t cus = (uint64_t)device_cus();
    if (pack) {
        uint64_t gp = b->pack_blocks < cus * 16 ? b->pack_blocks : cus * 16;
        if (gp < 1) gp = 1;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_batch_pack<TM, S>), dim3((unsigned)gp), dim3(256), 0, st, hdr, hdr,
                           descs, prefix);
        DQT_LAUNCH_CHECK("batched pack");
    } else {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, hdr);
        DQT_LAUNCH_CHECK("batched counter reset");
    }
    if (!compute) return DQT_OK;
    // one persistent launch per variant present: a few workgroups per CU, never more
    // than the variant has items
    const uint64_t per_cu = (S == 2) ? 8 : (S == 4 ? 4 : 2);
    for (uint32_t v = 0; v < BV_COUNT; ++v) {
        const uint64_t nv = b->variant_items[v];
        if (!nv) continue;
        const unsigned gc = (unsigned)(nv < cus * per_cu ? nv : cus * per_cu);
#define DQT_BV(OPV, FL, EP)                                                                                         \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_batch_compute<OPV, TM, TN, S, FL, EP>), dim3(gc), dim3(64 * S), 0, st, hdr, \
                       descs, items, v)
        switch (v) {
            case BV_DOT2: DQT_BV(OP_DOT2, false, 0); break;
            case BV_DOT2_EPIQ: DQT_BV(OP_DOT2, false, 1); break;
            case BV_DOT2_FLUSH: DQT_BV(OP_DOT2, true, 0); break;
            case BV_DOT2_FLUSH_EPIQ: DQT_BV(OP_DOT2, true, 1); break;
            case BV_DOT4: DQT_BV(OP_DOT4, false, 0); break;
            case BV_DOT8: DQT_BV(OP_DOT8, false, 0); break;
            default: DQT_BV(OP_MAD, false, 0); break;
        }
#undef DQT_BV
        DQT_LAUNCH_CHECK("batched compute");
    }
    return DQT_OK;
}

static dqt_status batch_dispatch(const dqt_batch* b, void* stream, bool pack, bool compute) {
    if (!b) return DQT_E_INVALID;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (b->s == 8) {
        if (b->tm == 8 && b->tn == 4) return batch_launch<8, 4, 8>(b, st, pack, compute);
        if (b->tm == 8) return batch_launch<8, 2, 8>(b, st, pack, compute);
        return batch_launch<16, 2, 8>(b, st, pack, compute);
    }
    if (b->tn == 4) {
        if (b->tm == 8 && b->s == 2) return batch_launch<8, 4, 2>(b, st, pack, compute);
        if (b->tm == 8 && b->s == 4) return batch_launch<8, 4, 4>(b, st, pack, compute);
        if (b->tm == 16 && b->s == 2) return batch_launch<16, 4, 2>(b, st, pack, compute);
        return batch_launch<16, 4, 4>(b, st, pack, compute);
    }
    if (b->tm == 8 && b->s == 2) return batch_launch<8, 2, 2>(b, st, pack, compute);
    if (b->tm == 8 && b->s == 4) return batch_launch<8, 2, 4>(b, st, pack, compute);
    if (b->tm == 16 && b->s == 2) return batch_launch<16, 2, 2>(b, st, pack, compute);
    return batch_launch<16, 2, 4>(b, st, pack, compute);
}

extern "C" dqt_status dqt_fgemm_batched_run(const dqt_batch* b, void* stream) {
    return batch_dispatch(b, stream, true, true);
}

extern "C" dqt_status dqt_fgemm_batched_pack(const dqt_batch* b, void* stream) {
    return batch_dispatch(b, stream, true, false);
}

extern "C" dqt_status dqt_fgemm_batched_compute(const dqt_batch* b, void* stream) {
    return batch_dispatch(b, stream, false, true);
}

extern "C" void dqt_batch_free(dqt_batch* b) { delete b; }

extern "C" dqt_status dqt_fgemm_batched(const dqt_gemm_desc* descs, uint32_t count, const dqt_batch_opts* opts,
                                        void* d_work, size_t work_bytes, void* stream) {
    dqt_batch* b = nullptr;
    DQT_TRY(dqt_fgemm_batched_prepare(descs, count, opts, d_work, work_bytes, stream, &b));
    const dqt_status st = dqt_fgemm_batched_run(b, stream);
    dqt_batch_free(b);
    return st;
}
