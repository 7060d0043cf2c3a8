// Host-side run of the FQT block-word reduction (dqt_fqt.h, dqt_device.h): the
// same source the kernels use, compiled for the CPU (under UBSan and ASan by
// tests/test_host_fqt.py).  Reads `count` pairs of records (na and nb coefficient
// bytes) from argv[2], argv[3]; writes the products (na + nb - 1 bytes each) of
// three forms to argv[4] .. argv[6]: compile-time q = 2^8 with the block words
// formed first, the same with each block word formed on demand inside the
// reduction loop, and the run-time form.  F_3, blocks of three coefficients.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../paper_0809_0063_amd/csrc/dqt_fqt.h"
#include "../../paper_0809_0063_amd/csrc/dqt_internal.h"

using namespace dqt;

namespace {

constexpr int BS = 3, MAXB = 16, QB = 8, QW = 2;
constexpr bool SMALL = true;
using F = FqtShape<BS, MAXB>;

std::vector<uint8_t> slurp(const char* path) {
    std::vector<uint8_t> v;
    FILE* f = fopen(path, "rb");
    if (!f) return v;
    uint8_t buf[65536];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) v.insert(v.end(), buf, buf + n);
    fclose(f);
    return v;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 9) {
        fprintf(stderr, "usage: fqt_host count a.bin b.bin out_first.bin out_demand.bin out_runtime.bin na nb\n");
        return 2;
    }
    const size_t count = strtoull(argv[1], nullptr, 10);
    const uint32_t na = (uint32_t)atoi(argv[7]), nb = (uint32_t)atoi(argv[8]);
    if (na < 1 || nb < 1 || na > MAXB * BS || nb > MAXB * BS) return 2;
    const std::vector<uint8_t> A = slurp(argv[2]), B = slurp(argv[3]);
    if (A.size() != count * na || B.size() != count * nb) return 3;
    const uint32_t p = 3, nout = na + nb - 1;
    RedqArgs ra;
    if (make_redq_args(p, QB, 2 * BS - 1, (2 * BS - 1) * QB, &ra) != DQT_OK) return 4;
    if (ra.w != (uint32_t)QW || !ra.small) return 4;
    // the correction table the kernels build in LDS, entry by entry
    std::vector<uint16_t> tab(4096, 0);
    const uint32_t wm = (1u << ra.w) - 1u;
    for (uint32_t idx = 0; idx < ra.tab_entries; ++idx) {
        const uint32_t u0 = idx & wm, u1 = (idx >> ra.w) & wm;
        uint32_t e = mod_small(u0 + ra.p * ra.p - ra.c * u1, ra.p, ra.pmagic);
        if (ra.tabj == 3) e |= mod_small(u1 + ra.p * ra.p - ra.c * ((idx >> (2 * ra.w)) & wm), ra.p, ra.pmagic) << 8;
        tab[idx] = (uint16_t)e;
    }
    std::vector<uint8_t> out[3];
    for (auto& o : out) o.assign(count * nout, 0);
    for (size_t t = 0; t < count; ++t) {
        uint32_t xa[F::ND] = {0}, xb[F::ND] = {0};
        memcpy(xa, &A[t * na], na);
        memcpy(xb, &B[t * nb], nb);
        uint32_t aw[MAXB], bw[MAXB];
        fqt_words<BS, MAXB>(xa, QB, aw);
        fqt_words<BS, MAXB>(xb, QB, bw);
        auto Wof = [&](int w) {
            uint64_t Wt = 0;
            for (int i = 0; i < MAXB; ++i) {
                const int j = w - i;
                if (j >= 0 && j < MAXB) Wt += (uint64_t)aw[i] * (uint64_t)bw[j];
            }
            return Wt;
        };
        uint64_t W[F::NW];
        for (int w = 0; w < F::NW; ++w) W[w] = Wof(w);
        uint32_t ob[3][F::NO] = {{0}};
        fqt_finish<BS, F::NW, QB, QW, SMALL>([&](int w) { return W[w]; }, nout, ra, tab.data(), ob[0]);
        fqt_finish<BS, F::NW, QB, QW, SMALL>(Wof, nout, ra, tab.data(), ob[1]);
        fqt_finish<BS, F::NW, 0, 0, false>(Wof, nout, ra, tab.data(), ob[2]);
        for (int f = 0; f < 3; ++f) memcpy(&out[f][t * nout], ob[f], nout);
    }
    for (int f = 0; f < 3; ++f) {
        FILE* o = fopen(argv[4 + f], "wb");
        if (!o || fwrite(out[f].data(), 1, out[f].size(), o) != out[f].size()) return 5;
        fclose(o);
    }
    return 0;
}
