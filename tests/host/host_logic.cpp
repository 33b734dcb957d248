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
    if (failures) std::printf("%d failures\n", failures);
    else std::printf("ok\n");
    return failures > 100 ? 100 : failures;
}
