// Host-side run of REDQ (algorithm REDQ of section 3: the compression by one
// binary64 floor division and the correction by the tabulated windows of
// section 3.5) from the same source the kernels use (dqt_device.h), compiled
// for the CPU under UBSan and ASan by tests/test_host_fqt.py.  For the
// parameters on the command line it draws `count` words r = sum_i d_i q^i,
// q = 2^b, with q-adic digits d_i (the top digit bounded so that r stays below
// 2^word_bits), and checks that the reduction yields d_i mod p for every i.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../../paper_0809_0063_amd/csrc/dqt_internal.h"

using namespace dqt;

namespace {

uint64_t splitmix64(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int NR>
int run(const RedqArgs& ra, const std::vector<uint16_t>& tab, uint32_t word_bits, uint64_t count, uint64_t seed) {
    const uint32_t b = ra.b;
    const uint32_t top_bits = word_bits - b * (NR - 1);
    for (uint64_t t = 0; t < count; ++t) {
        uint64_t d[NR];
        uint64_t r = 0;
        for (int i = 0; i < NR; ++i) {
            const uint32_t bits = (i == NR - 1) ? top_bits : b;
            d[i] = splitmix64(&seed) & ((bits >= 64 ? 0 : (1ull << bits)) - 1);
            if (t % 5 == 0) d[i] = (bits >= 64 ? ~0ull : (1ull << bits) - 1);   // all digits at their maximum
            r |= d[i] << (b * i);
        }
        const uint64_t U = redq_compress(r, ra);
        uint32_t got[NR];
        redq_correct<NR>(U, ra, tab.data(), [&](int i, uint32_t m) { got[i] = m; });
        for (int i = 0; i < NR; ++i)
            if (got[i] != d[i] % ra.p) {
                fprintf(stderr, "p=%u b=%u nres=%d word %llx digit %d: got %u want %llu\n", ra.p, b, NR,
                        (unsigned long long)r, i, got[i], (unsigned long long)(d[i] % ra.p));
                return 1;
            }
    }
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 8) {
        fprintf(stderr, "usage: redq_host p b nres word_bits table_window count seed\n");
        return 2;
    }
    const uint32_t p = (uint32_t)atoi(argv[1]), b = (uint32_t)atoi(argv[2]), nres = (uint32_t)atoi(argv[3]);
    const uint32_t word_bits = (uint32_t)atoi(argv[4]), window = (uint32_t)atoi(argv[5]);
    const uint64_t count = strtoull(argv[6], nullptr, 10), seed = strtoull(argv[7], nullptr, 10);
    if (dqt_set_table_window(window) != DQT_OK) return 2;
    RedqArgs ra;
    if (make_redq_args(p, b, nres, word_bits, &ra) != DQT_OK) return 4;
    std::vector<uint16_t> tab(4096, 0);
    for (uint32_t idx = 0; idx < ra.tab_entries; ++idx) tab[idx] = correction_entry(idx, ra);
    int rc = 2;
    switch (nres) {
        case 2: rc = run<2>(ra, tab, word_bits, count, seed); break;
        case 3: rc = run<3>(ra, tab, word_bits, count, seed); break;
        case 4: rc = run<4>(ra, tab, word_bits, count, seed); break;
        case 5: rc = run<5>(ra, tab, word_bits, count, seed); break;
        case 7: rc = run<7>(ra, tab, word_bits, count, seed); break;
        default: break;
    }
    if (rc == 0) printf("ok tabj=%u\n", ra.tabj);
    return rc;
}
