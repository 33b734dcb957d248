// Host-side logic of the runtime, checked on the CPU (no device call is
// made): the binned table geometry, the size classes that key captured
// passes, and the host count of windows and k-mers that dbg_build uses to
// validate and size its input.  Prints one line per failure and "ok" at the
// end; the exit status is the number of failures (capped at 100).
#include "dbg_runtime.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            if (failures < 20) {                  \
                std::printf("FAIL %s: ", #cond);  \
                std::printf(__VA_ARGS__);         \
                std::printf("\n");                \
            }                                     \
            ++failures;                           \
        }                                         \
    } while (0)

static void check_geometry(uint64_t cap) {
    uint32_t d1 = 0, fan = 0;
    uint64_t parts = 0;
    const uint64_t want = std::max<uint64_t>(1, (cap + dbgk::kSegSlots - 1) / dbgk::kSegSlots);
    const bool ok = dbgrt::binned_geometry(cap, &d1, &fan, &parts);
    const bool fits = want <= (uint64_t)dbgk::kMaxD1 * dbgk::kMaxFan;
    if (!ok) {
        // refused only when no split into at most kMaxD1 x kMaxFan exists
        CHECK(!fits || std::ceil(std::sqrt((double)want)) > dbgk::kMaxD1, "cap %llu refused",
              (unsigned long long)cap);
        return;
    }
    CHECK(d1 >= 1 && d1 <= dbgk::kMaxD1, "cap %llu d1 %u", (unsigned long long)cap, d1);
    CHECK(fan >= 1 && fan <= dbgk::kMaxFan, "cap %llu fan %u", (unsigned long long)cap, fan);
    CHECK(parts == (uint64_t)d1 * fan, "cap %llu parts %llu", (unsigned long long)cap, (unsigned long long)parts);
    CHECK(parts >= want, "cap %llu: %llu segments for %llu wanted", (unsigned long long)cap,
          (unsigned long long)parts, (unsigned long long)want);
    // no whole bucket of spare segments, and fan never exceeds what d1 requires
    CHECK((uint64_t)(d1 - 1) * fan < want, "cap %llu: d1 %u fan %u over %llu", (unsigned long long)cap, d1, fan,
          (unsigned long long)want);
    CHECK((uint64_t)d1 * (fan - 1) < want, "cap %llu: fan %u larger than needed", (unsigned long long)cap, fan);
}

static void check_size_class() {
    uint64_t prev = 0;
    for (uint64_t x = 0; x < 300000; ++x) {
        const uint64_t s = dbgrt::size_class(x, 64);
        CHECK(s >= x && s >= 64, "size_class(%llu) = %llu", (unsigned long long)x, (unsigned long long)s);
        CHECK(s >= prev, "size_class not monotone at %llu", (unsigned long long)x);
        // at most one eighth of the next power of two above x
        CHECK(x < 64 || s - x < std::max<uint64_t>(x / 4, 1), "size_class(%llu) = %llu too coarse",
              (unsigned long long)x, (unsigned long long)s);
        prev = s;
    }
    for (uint64_t x = 1; x < (1ull << 60); x = x * 5 / 3 + 1) {
        const uint64_t s = dbgrt::size_class(x, 1);
        CHECK(s >= x && s - x <= x / 4 + 1, "size_class(%llu) = %llu", (unsigned long long)x, (unsigned long long)s);
        CHECK(dbgrt::size_class(s, 1) == s, "size_class(%llu) not a fixed point", (unsigned long long)s);
    }
}

static void check_host_counts(std::mt19937_64 &rng) {
    for (int rep = 0; rep < 2000; ++rep) {
        const uint64_t n = rng() % 40;
        const uint32_t k = 2 + rng() % 63;
        std::vector<uint64_t> off(n + 1);
        off[0] = rng() % 1000;
        for (uint64_t i = 0; i < n; ++i) off[i + 1] = off[i] + (rng() % 4 == 0 ? rng() % 8 : rng() % 200);
        const bool decrease = n > 0 && rng() % 5 == 0;
        if (decrease) {
            const uint64_t i = 1 + rng() % n;
            if (off[i] > 0) off[i] = off[i - 1] - (off[i - 1] > 0 ? 1 : 0) * (1 + rng() % std::max<uint64_t>(1, off[i - 1]));
        }
        bool mono = true;
        uint64_t w = 0, e = 0;
        for (uint64_t i = 0; i < n; ++i) {
            if (off[i + 1] < off[i]) mono = false;
            else if (off[i + 1] - off[i] >= k) {
                w += off[i + 1] - off[i] - k + 2;  // windows: L - k + 2 vertices
                e += off[i + 1] - off[i] - k + 1;  // k-mers: L - k + 1 edges
            }
        }
        uint64_t hw = 12345, he = 6789;
        const bool ok = dbgrt::host_counts(off.data(), n, k, &hw, &he);
        CHECK(ok == mono, "rep %d: accepted %d, monotone %d", rep, (int)ok, (int)mono);
        if (ok && mono) CHECK(hw == w && he == e, "rep %d: %llu/%llu vs %llu/%llu", rep, (unsigned long long)hw,
                              (unsigned long long)he, (unsigned long long)w, (unsigned long long)e);
    }
}

// Chunk counts of the two partition passes stay within the capacities the
// runtime reserves (bin_caps): for random instance and bucket sizes, the
// chunk length max(1, floor(tiles / target)) that the plan kernels use gives
// at most chunks1_cap - 1 (pass 1) and chunks2_cap - 1 (pass 2) chunks, and
// the histograms fit.
static uint64_t chunks_of(const std::vector<uint64_t> &tiles, uint64_t target) {
    uint64_t all = 0;
    for (uint64_t t : tiles) all += t;
    const uint64_t chunk = std::max<uint64_t>(1, all / std::max<uint64_t>(target, 1));
    uint64_t n = 0;
    for (uint64_t t : tiles) n += (t + chunk - 1) / chunk;
    return n;
}

static void check_chunks(std::mt19937_64 &rng) {
    for (int round = 0; round < 3000; ++round) {
        const uint32_t m = 1 + (uint32_t)(rng() % (round % 3 ? 8 : 300));
        const uint64_t len = 4096 + rng() % (round % 5 ? (1ull << 24) : (1ull << 33));
        const uint32_t target = 1 + (uint32_t)(rng() % dbgk::kMaxChunkTarget);
        // windows of each instance: a random split of at most len
        std::vector<uint64_t> w(m), tiles(m);
        uint64_t left = len;
        for (uint32_t i = 0; i < m; ++i) {
            w[i] = i + 1 == m ? left : (left ? rng() % (left + 1) : 0);
            left -= w[i];
            tiles[i] = (w[i] + dbgk::kBinTile - 1) / dbgk::kBinTile;
        }
        dbgrt::PassKey k;
        k.binned = 1;
        k.m_cap = (uint32_t)dbgrt::size_class(m, 1);
        k.len_cap = dbgrt::size_class(len, 4096);
        const uint32_t d1 = 1 + (uint32_t)(rng() % dbgk::kMaxD1), fan = 1 + (uint32_t)(rng() % dbgk::kMaxFan);
        const uint64_t G = (uint64_t)m * d1;  // buckets over the launch
        k.buckets_cap = dbgrt::size_class(G, 64);
        k.d1_cap = (uint32_t)std::min<uint64_t>(dbgrt::size_class(d1, 16), dbgk::kMaxD1);
        k.fan_cap = (uint32_t)std::min<uint64_t>(dbgrt::size_class(fan, 16), dbgk::kMaxFan);
        dbgk::BinBuffers bb{};
        dbgrt::bin_caps(k, bb);
        const uint64_t c1 = chunks_of(tiles, target);
        CHECK(c1 + 1 <= bb.chunks1_cap, "pass 1: %llu chunks, cap %llu", (unsigned long long)c1,
              (unsigned long long)bb.chunks1_cap);
        CHECK((uint64_t)d1 * c1 <= bb.hist1_cap, "pass 1 histogram");
        // records (one per window) split over the G buckets
        std::vector<uint64_t> bt(G);
        uint64_t rec_left = len;
        for (uint64_t g = 0; g < G; ++g) {
            const uint64_t sz = g + 1 == G ? rec_left : (rec_left ? rng() % (2 * rec_left / (G - g) + 1) : 0);
            const uint64_t take = std::min(sz, rec_left);
            rec_left -= take;
            bt[g] = (take + dbgk::kRefTile - 1) / dbgk::kRefTile;
        }
        const uint64_t c2 = chunks_of(bt, target);
        CHECK(c2 + 1 <= bb.chunks2_cap, "pass 2: %llu chunks, cap %llu", (unsigned long long)c2,
              (unsigned long long)bb.chunks2_cap);
        CHECK((uint64_t)fan * c2 <= bb.hist2_cap, "pass 2 histogram");
    }
}

int main() {
    for (uint64_t cap = 0; cap < 200000; cap += 7) check_geometry(cap);
    for (uint64_t cap = 1; cap < (1ull << 45); cap = cap * 9 / 8 + 1) check_geometry(cap);
    // around every segment count near the square boundaries
    for (uint64_t s = 1; s <= 2048; ++s)
        for (int64_t d = -2; d <= 2; ++d) {
            const int64_t segs = (int64_t)(s * s) + d;
            if (segs > 0) check_geometry((uint64_t)segs * dbgk::kSegSlots);
        }
    check_size_class();
    std::mt19937_64 rng(20240105);
    check_host_counts(rng);
    check_chunks(rng);
    if (failures) std::printf("%d failures\n", failures);
    else std::printf("ok\n");
    return failures > 100 ? 100 : failures;
}
