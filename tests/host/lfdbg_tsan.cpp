// lfdbg_tsan.cpp -- drives the threaded CPU build of the paper's lock-free
// design (oracle/lfdbg_cpu.cpp, linked in directly) for a build under
// ThreadSanitizer: 8 threads on a table of 1 and of 64 buckets (every
// insertion races on a few list heads), on seeded random reads over two and
// four letters, and checks that the result equals the one-thread build.
// Exit status 0 and "ok" on success.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" int lfdbg_build(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                           uint32_t threads, uint64_t buckets, uint64_t **keys_out, uint32_t **counts_out,
                           uint64_t *n_out, double *seconds);
extern "C" void lfdbg_free(void *p);

int main() {
    std::mt19937_64 rng(0x1F2E3D4C5B6A7988ull);
    int failures = 0;
    for (int round = 0; round < 6; ++round) {
        const uint32_t k = round % 2 ? 21 : 5;
        const uint32_t letters = round < 3 ? 2 : 4;
        const uint64_t n = 400;
        std::vector<uint64_t> off(n + 1, 0);
        for (uint64_t i = 0; i < n; ++i) off[i + 1] = off[i] + 20 + rng() % 60;
        std::vector<unsigned char> reads(off[n]);
        for (auto &c : reads) c = (unsigned char)"ACGT"[rng() % letters];
        uint64_t *k1 = nullptr, *k8 = nullptr, n1 = 0, n8 = 0;
        uint32_t *c1 = nullptr, *c8 = nullptr;
        double s = 0;
        if (lfdbg_build(reads.data(), off.data(), n, k, 1, 64, &k1, &c1, &n1, &s) != 0) return 1;
        for (uint64_t buckets : {1ull, 64ull}) {
            if (lfdbg_build(reads.data(), off.data(), n, k, 8, buckets, &k8, &c8, &n8, &s) != 0) return 1;
            if (n8 != n1 || std::memcmp(k1, k8, n1 * 8) != 0 || std::memcmp(c1, c8, n1 * 16) != 0) {
                std::printf("FAIL round %d buckets %llu\n", round, (unsigned long long)buckets);
                ++failures;
            }
            lfdbg_free(k8);
            lfdbg_free(c8);
        }
        lfdbg_free(k1);
        lfdbg_free(c1);
    }
    if (failures) return failures;
    std::printf("ok\n");
    return 0;
}
